"""Reverse mode of the 2D Euler stage on the forward-step mesh (Example 3.11 boundaries: an
inflow of prescribed state on the left, an outflow on the right, reflective walls at the
top, the bottom and on the step's two faces, solid cells inside the step) on the GPU
against the oracle, with troubled-cell flags, hybrid masks and Lax-Friedrichs speeds held
at their forward values.

A stencil position outside the fluid takes the values of one fluid cell (the position
rule), or the prescribed inflow state, which carries no dependence on the state; the
reverse folds each such position's cotangent back onto its source cell, and at a face
between a fluid cell and a wall or the outflow the non-fluid side's trace is the fluid
cell's own (the face rule), so that side's flux derivative also belongs to the fluid cell.
Solid cells are never updated: their rows of the operator are zero and a step maps them to
themselves.

The oracle side is the complex-step derivative of the oracle's own operator / RK3 step with
the same flags and speeds frozen (pinned against central differences on the CPU in
tests/test_oracle_adjoint.py):
* small meshes: (dL/dU)^T lam and (dU1/dU0)^T lam of one step, column by column, compared
  element by element, max|gpu - oracle| / max|oracle| <= 1e-12; meshes where the step
  reaches the exit (a one-cell-wide step, whose mirror positions lie two cells from their
  source) included;
* a multi-step run with checkpoints: dot-product test <J d, lam> = <d, J^T lam>.
"""
import numpy as np
import pytest

import hweno_inputs as hi
from oracle.scheme2d import Scheme2D

pytestmark = pytest.mark.gpu

TOL = 1e-12
CSH = 1e-30
H = 0.1        # cell size: a mesh of nx x ny cells on [0, nx H] x [0, ny H]


@pytest.fixture(scope="module")
def hw():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2002_08816_amd as hw
    return hw


def make_pair(hw, nx, ny, si, sj, ng, tc):
    dom = (0.0, nx * H, 0.0, ny * H)
    corner = (si * H, sj * H)
    s = hw.Solver(2, nx, ny, domain=dom, eq="euler", ng_edge=ng, tc_mode=tc, bc="step", step=corner)
    o = Scheme2D("euler", nx, ny, *dom, bc="step", ng_edge=ng, tc_mode=tc, step_corner=corner)
    assert o.step_ij == (si, sj)
    return s, o


def oracle_vjp(fn, U, lam):
    g = np.zeros(U.size)
    flat = U.reshape(-1)
    for j in range(U.size):
        Uc = flat.astype(complex)
        Uc[j] += 1j * CSH
        g[j] = np.sum(fn(Uc.reshape(U.shape)).imag / CSH * lam)
    return g.reshape(U.shape)


def rel_err(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def boundary_cells(o):
    """Fluid cells with a non-fluid position among their eight neighbours."""
    fluid = np.pad(~o.solid, 1, constant_values=False)
    ny, nx = o.solid.shape
    near = np.zeros_like(o.solid)
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            near |= ~fluid[1 + dy:1 + dy + ny, 1 + dx:1 + dx + nx]
    return near & ~o.solid


def check_flags(s, o, U, info):
    s.flag_export(True)
    s.apply_operator(U)
    Tg, Hg = s.flags(0)
    s.flag_export(False)
    T, Hm = info["T"].astype(bool), info["H"].astype(bool)
    assert np.array_equal(Tg.astype(bool), T), "troubled-cell flags differ"
    assert np.array_equal(Hg.astype(bool), Hm), "hybrid masks differ"
    edge = boundary_cells(o)
    assert (T & edge).any() and (Hm & ~T & edge).any() and (~Hm & edge).any()


@pytest.mark.parametrize("nx,ny,si,sj,ng,tc", [
    (18, 10, 7, 3, 2, "kxrcf"),
    (12, 7, 5, 3, 3, "all"),
    (10, 7, 9, 3, 2, "all"),       # the step reaches the exit
    (12, 8, 6, 4, 2, "none"),
])
def test_step_operator_adjoint_elementwise(hw, nx, ny, si, sj, ng, tc):
    print(f"step operator adjoint {nx}x{ny} corner ({si},{sj}) ng={ng} tc={tc}", flush=True)
    s, o = make_pair(hw, nx, ny, si, sj, ng, tc)
    U = hi.euler_step_state(nx, ny, si, sj, 5)
    alphas = o.alphas(U)
    _, info = o.operator(U)
    T = info["T"].astype(bool)
    if tc == "kxrcf":
        check_flags(s, o, U, info)
    lam = np.random.default_rng(13).normal(size=U.shape)
    g = s.apply_operator_adjoint(U, lam)
    go = oracle_vjp(lambda X: o.operator(X, alphas=alphas, T_fixed=T)[0], U, lam)
    # solid cells: L does not depend on them, and their rows of L are zero
    assert np.array_equal(go[:, :, o.solid], 0 * go[:, :, o.solid])
    e = rel_err(g, go)
    print(f"  max rel err {e:.3e}; solid cells max |g| {np.abs(g[:, :, o.solid]).max():.1e}")
    assert e < TOL, e
    assert np.abs(g[:, :, o.solid]).max() <= TOL * np.abs(go).max()
    s.close()


def frozen_of(o, U, dt, nsteps=1):
    out, X = [], U
    for _ in range(nsteps):
        X, infos = o.rk3_step(X, dt)
        out.append([(i["alpha"], i["T"].astype(bool)) for i in infos])
    return out, X


@pytest.mark.parametrize("nx,ny,si,sj", [(12, 7, 5, 3), (10, 7, 9, 3)])
def test_step_rk3_adjoint_elementwise(hw, nx, ny, si, sj):
    print(f"step RK3 adjoint {nx}x{ny} corner ({si},{sj}) ng=2 tc=kxrcf", flush=True)
    s, o = make_pair(hw, nx, ny, si, sj, 2, "kxrcf")
    U = hi.euler_step_state(nx, ny, si, sj, 6)
    dt = 0.5 * o.cfl_dt(U, 0.6)
    fz, U1o = frozen_of(o, U, dt)
    s.set_state(U)
    s.flag_export(True)
    s.forward_ckpt(1, dt, 1)
    for st in range(3):
        Tg, _ = s.flags(st)
        assert np.array_equal(Tg.astype(bool), fz[0][st][1]), f"flags of stage {st} differ"
    s.flag_export(False)
    U1, _ = s.get_state()
    assert rel_err(U1, U1o) < 1e-12
    lam = np.random.default_rng(14).normal(size=U.shape)
    g = s.adjoint(lam)
    go = oracle_vjp(lambda X: o.rk3_step(X, dt, frozen=fz[0])[0], U, lam)
    e = rel_err(g, go)
    print(f"  max rel err {e:.3e}")
    assert e < TOL, e
    # a step maps the solid cells to themselves: their gradient is lam there, up to the
    # rounding of the stage weights (1/3 + 1/2 + 1/6 through the three reversed stages)
    assert np.abs(g[:, :, o.solid] - lam[:, :, o.solid]).max() <= 1e-15 * np.abs(lam).max()
    s.close()


def test_step_trajectory_dot_product(hw):
    nx, ny, si, sj, nsteps, k = 30, 12, 10, 4, 5, 2
    print(f"step trajectory dot test {nx}x{ny} corner ({si},{sj}) steps={nsteps} k={k}", flush=True)
    s, o = make_pair(hw, nx, ny, si, sj, 2, "kxrcf")
    U = hi.euler_step_state(nx, ny, si, sj, 8)
    dt = 0.5 * o.cfl_dt(U, 0.6)
    fz, UTo = frozen_of(o, U, dt, nsteps)
    s.set_state(U)
    s.forward_ckpt(nsteps, dt, k)
    UT, _ = s.get_state()
    assert rel_err(UT, UTo) < 1e-11
    lam = np.random.default_rng(23).normal(size=U.shape)
    g = s.adjoint(lam)
    rng = np.random.default_rng(24)
    for r in range(3):
        d = rng.normal(size=U.shape)
        X = U + 1j * CSH * d
        for n in range(nsteps):
            X, _ = o.rk3_step(X, dt, frozen=fz[n])
        Jd = X.imag / CSH
        lhs, rhs = np.sum(Jd * lam), np.sum(d * g)
        e = abs(lhs - rhs) / (np.linalg.norm(Jd) * np.linalg.norm(lam))
        print(f"  direction {r}: rel {e:.2e}")
        assert e < TOL, e
    s.close()
