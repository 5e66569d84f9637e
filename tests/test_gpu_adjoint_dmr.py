"""Reverse mode of the 2D Euler stage on the double Mach reflection's boundaries (Example
3.10: prescribed exact cut-cell moments left of the mesh, above it and below it left of
x = 1/6, a reflective wall below it from x = 1/6 on, an outflow on the right) on the GPU
against the oracle, with troubled-cell flags, hybrid masks and Lax-Friedrichs speeds held
at their forward values.

The prescribed ghosts and the exact states on their faces depend on time only, so they carry
no cotangent; the mirrored ghosts of the wall and the outflow fold theirs back onto the
cells they mirror, as on rectangles with walls.  The time-stepped cases check that the
replay of a recorded run reproduces each stage's prescribed data at that stage's time.

The oracle side is the complex-step derivative of the oracle's own operator / RK3 step with
the same flags and speeds frozen (pinned against central differences on the CPU in
tests/test_oracle_adjoint.py):
* small meshes of square cells, the Mach 10 initial state with jump bands along the inflow
  and outflow sides: (dL/dU)^T lam at t = 0 and t = 0.002 and (dU1/dU0)^T lam of one step,
  column by column, max|gpu - oracle| / max|oracle| <= 1e-12;
* a four-step run with checkpoints every two steps: dot-product test
  <J d, lam> = <d, J^T lam>.
Steps are a fifth of the CFL step and use the 3-point edge rule: on meshes this coarse the
Mach 10 problem loses positivity within a step otherwise.
"""
import numpy as np
import pytest

import hweno_inputs as hi
from oracle.scheme2d import Scheme2D

pytestmark = pytest.mark.gpu

TOL = 1e-12
CSH = 1e-30


@pytest.fixture(scope="module")
def hw():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2002_08816_amd as hw
    return hw


def make_pair(hw, nx, ny, ng, tc):
    h = 1.0 / (2 * ny)
    dom = (0.0, nx * h, 0.0, ny * h)
    s = hw.Solver(2, nx, ny, domain=dom, eq="euler", ng_edge=ng, tc_mode=tc, bc="dmr")
    o = Scheme2D("euler", nx, ny, *dom, bc="dmr", ng_edge=ng, tc_mode=tc)
    return s, o, hi.euler_dmr_state(nx, ny, h, 5)


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


@pytest.mark.parametrize("nx,ny,ng,tc,t0", [
    (14, 7, 2, "kxrcf", 0.0),
    (14, 7, 3, "all", 0.002),
    (16, 8, 2, "kxrcf", 0.002),
])
def test_dmr_operator_adjoint_elementwise(hw, nx, ny, ng, tc, t0):
    print(f"DMR operator adjoint {nx}x{ny} ng={ng} tc={tc} t={t0}", flush=True)
    s, o, U = make_pair(hw, nx, ny, ng, tc)
    alphas = o.alphas(U)
    _, info = o.operator(U, t=t0)
    T = info["T"].astype(bool)
    s.set_state(U)
    s.set_time(t0)
    if tc == "kxrcf":
        s.flag_export(True)
        s.apply_operator(U)
        Tg, Hg = s.flags(0)
        s.flag_export(False)
        assert np.array_equal(Tg.astype(bool), T), "troubled-cell flags differ"
        assert np.array_equal(Hg.astype(bool), info["H"].astype(bool)), "hybrid masks differ"
        # troubled cells on every side, linear cells along the wall and the top
        assert T[:, 0].any() and T[:, -1].any() and T[0, :].any() and T[-1, :].any()
        assert (~info["H"].astype(bool)[0, :]).any() and (~info["H"].astype(bool)[-1, :]).any()
    lam = np.random.default_rng(15).normal(size=U.shape)
    g = s.apply_operator_adjoint(U, lam)
    go = oracle_vjp(lambda X: o.operator(X, alphas=alphas, T_fixed=T, t=t0)[0], U, lam)
    e = rel_err(g, go)
    print(f"  max rel err {e:.3e}")
    assert e < TOL, e
    s.close()


def frozen_of(o, U, dt, t0, nsteps=1):
    out, X, t = [], U, t0
    for _ in range(nsteps):
        X, infos = o.rk3_step(X, dt, t=t)
        t += dt
        out.append([(i["alpha"], i["T"].astype(bool)) for i in infos])
    return out, X


def test_dmr_rk3_adjoint_elementwise(hw):
    nx, ny, ng, t0 = 14, 7, 3, 0.002
    print(f"DMR RK3 adjoint {nx}x{ny} ng={ng} tc=kxrcf t0={t0}", flush=True)
    s, o, U = make_pair(hw, nx, ny, ng, "kxrcf")
    dt = 0.2 * o.cfl_dt(U, 0.6)
    fz, U1o = frozen_of(o, U, dt, t0)
    s.set_state(U)
    s.set_time(t0)
    s.flag_export(True)
    s.forward_ckpt(1, dt, 1)
    for st in range(3):
        Tg, _ = s.flags(st)
        assert np.array_equal(Tg.astype(bool), fz[0][st][1]), f"flags of stage {st} differ"
    s.flag_export(False)
    U1, _ = s.get_state()
    assert rel_err(U1, U1o) < 1e-12
    lam = np.random.default_rng(16).normal(size=U.shape)
    g = s.adjoint(lam)
    go = oracle_vjp(lambda X: o.rk3_step(X, dt, frozen=fz[0], t=t0)[0], U, lam)
    e = rel_err(g, go)
    print(f"  max rel err {e:.3e}")
    assert e < TOL, e
    s.close()


def test_dmr_trajectory_dot_product(hw):
    nx, ny, ng, nsteps, k = 28, 10, 3, 4, 2
    print(f"DMR trajectory dot test {nx}x{ny} ng={ng} steps={nsteps} k={k}", flush=True)
    s, o, U = make_pair(hw, nx, ny, ng, "kxrcf")
    dt = 0.2 * o.cfl_dt(U, 0.6)
    fz, UTo = frozen_of(o, U, dt, 0.0, nsteps)
    s.set_state(U)
    s.forward_ckpt(nsteps, dt, k)
    UT, _ = s.get_state()
    assert rel_err(UT, UTo) < 1e-11
    lam = np.random.default_rng(25).normal(size=U.shape)
    g = s.adjoint(lam)
    rng = np.random.default_rng(26)
    for r in range(3):
        d = rng.normal(size=U.shape)
        X, t = U + 1j * CSH * d, 0.0
        for n in range(nsteps):
            X, _ = o.rk3_step(X, dt, frozen=fz[n], t=t)
            t += dt
        Jd = X.imag / CSH
        lhs, rhs = np.sum(Jd * lam), np.sum(d * g)
        e = abs(lhs - rhs) / (np.linalg.norm(Jd) * np.linalg.norm(lam))
        print(f"  direction {r}: rel {e:.2e}")
        assert e < TOL, e
    s.close()


def test_dmr_reverse_needs_detection(hw):
    from paper_2002_08816_amd import capi
    s = hw.Solver(2, 28, 7, domain=(0.0, 2.0, 0.0, 0.5), eq="euler", ng_edge=3, tc_mode="none",
                  bc="dmr")
    with pytest.raises(capi.HWError) as ei:
        s.forward_ckpt(1, 1e-4, 1)
    assert ei.value.status == capi.HW_EINVAL
    s.close()
