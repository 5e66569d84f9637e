"""Reverse mode on the GPU against the oracle: the hand-written adjoint of the stage
operator and of whole TVD-RK3 runs (2D scalar equations, periodic meshes and meshes with
transmissive sides), with
troubled-cell flags, hybrid masks and Lax-Friedrichs speeds held at their forward values.

The oracle side is the complex-step derivative of the oracle's own operator / RK3 step
with the same flags and speeds frozen: J d = Im F(U + i h d) / h, exact to round-off.
* small meshes: the transposed Jacobian applied to a seeded cotangent is built column by
  column from the oracle (one complex-step evaluation per unknown) and compared element
  by element, max|gpu - oracle| / max|oracle| <= 1e-12;
* multi-step runs: dot-product test <J d, lam> = <d, J^T lam> over seeded directions,
  |difference| / (|J d| |lam|) <= 1e-12;
* the full-size run (256^2 Burgers on [0,4]^2, 200 steps of dt = 1/(200 pi), checkpoints
  every 20 steps): central finite differences of the misfit loss through
  torch.autograd along seeded directions, relative difference <= 1e-6.
"""
import math

import numpy as np
import pytest

import hweno_inputs as hi
from oracle.physics import Equation
from oracle.scheme2d import Scheme2D

pytestmark = pytest.mark.gpu

TOL = 1e-12
CSH = 1e-30     # complex-step size


@pytest.fixture(scope="module")
def hw():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2002_08816_amd as hw
    return hw


def burgers_data(nx, ny, seed, noise=0.0):
    """cfg-5 style smooth field on [0, 4] x [0, 4 ny/nx] (square cells), optionally with
    seeded noise on the first moments so that KXRCF flags some cells."""
    kl, a, phi = hi.burgers_modes_params(5000 + seed)
    f = hi.burgers_modes_func(kl, a, phi)
    U = hi.project_2d(f, 0.0, 4.0, 0.0, 4.0 * ny / nx, nx, ny, nq=5)
    if noise > 0.0:
        rng = np.random.default_rng(77 + seed)
        U[1:] += noise * rng.normal(size=U[1:].shape)
    return U


def make_pair(hw, eq, nx, ny, ng, tc, bc="periodic"):
    kw = dict(domain=(0.0, 4.0, 0.0, 4.0 * ny / nx), eq=eq, adv=(1.0, 0.7), ng_edge=ng, tc_mode=tc, bc=bc)
    s = hw.Solver(2, nx, ny, **kw)
    o = Scheme2D(Equation(eq, 2, adv=(1.0, 0.7)), nx, ny, 0.0, 4.0, 0.0, 4.0 * ny / nx,
                 ng_edge=ng, tc_mode=tc, bc=bc)
    return s, o


def oracle_vjp(fn, U, lam):
    """(dF/dU)^T lam column by column: entry j = <Im F(U + i h e_j) / h, lam>."""
    g = np.zeros(U.size)
    flat = U.reshape(-1)
    for j in range(U.size):
        Uc = flat.astype(complex)
        Uc[j] += 1j * CSH
        g[j] = np.sum(fn(Uc.reshape(U.shape)).imag / CSH * lam)
    return g.reshape(U.shape)


def rel_err(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def gpu_flags_of_operator(s, U):
    s.flag_export(True)
    s.apply_operator(U)
    T, H = s.flags(0)
    s.flag_export(False)
    return T.astype(bool), H.astype(bool)


# ------------------------------------------------------------------ operator, element-wise
@pytest.mark.parametrize("eq,nx,ny,ng,tc", [
    ("burgers", 9, 8, 2, "all"),
    ("burgers", 20, 17, 3, "none"),
    ("burgers", 20, 17, 3, "kxrcf"),
    ("burgers", 20, 17, 3, "all"),
    ("burgers", 20, 17, 2, "kxrcf"),
    ("advection", 20, 17, 2, "kxrcf"),
    ("advection", 18, 18, 3, "all"),
])
def test_operator_adjoint_elementwise(hw, eq, nx, ny, ng, tc):
    print(f"operator adjoint {eq} {nx}x{ny} ng={ng} tc={tc}", flush=True)
    s, o = make_pair(hw, eq, nx, ny, ng, tc)
    U = burgers_data(nx, ny, seed=3, noise=0.02 if tc == "kxrcf" else 0.0)
    alphas = o.alphas(U)
    _, info = o.operator(U)
    T = info["T"].astype(bool)
    if tc == "kxrcf":
        Tg, Hg = gpu_flags_of_operator(s, U)
        assert np.array_equal(Tg, T), "troubled-cell flags differ"
        assert 0 < T.sum() < T.size, T.sum()   # both branches exercised
    lam = np.random.default_rng(11).normal(size=U.shape)
    g = s.apply_operator_adjoint(U, lam)
    go = oracle_vjp(lambda X: o.operator(X, alphas=alphas, T_fixed=T)[0], U, lam)
    e = rel_err(g, go)
    print(f"  max rel err {e:.3e}")
    assert e < TOL, e
    s.close()


TRANSMISSIVE = [
    ("burgers", 20, 17, 2, "kxrcf", ("transmissive", "transmissive")),
    ("burgers", 20, 17, 3, "all", ("transmissive", "periodic")),
    ("burgers", 18, 19, 3, "kxrcf", ("periodic", "transmissive")),
    ("advection", 20, 17, 2, "kxrcf", ("transmissive", "transmissive")),
    ("advection", 17, 18, 3, "none", ("transmissive", "transmissive")),
]


@pytest.mark.parametrize("eq,nx,ny,ng,tc,bc", TRANSMISSIVE)
def test_operator_adjoint_transmissive(hw, eq, nx, ny, ng, tc, bc):
    """Transmissive sides: the ghosts mirror the cells beside a side (the moment normal to
    it negated) and share their flags and hybrid masks; troubled and hybrid cells at the
    sides are required."""
    print(f"operator adjoint {eq} {nx}x{ny} ng={ng} tc={tc} bc={bc}", flush=True)
    s, o = make_pair(hw, eq, nx, ny, ng, tc, bc)
    U = burgers_data(nx, ny, seed=4, noise=0.03 if tc == "kxrcf" else 0.0)
    alphas = o.alphas(U)
    _, info = o.operator(U)
    T = info["T"].astype(bool)
    if tc == "kxrcf":
        Tg, Hg = gpu_flags_of_operator(s, U)
        assert np.array_equal(Tg, T), "troubled-cell flags differ"
        edge = np.zeros_like(T)
        if bc[0] != "periodic":
            edge[:, 0] = edge[:, -1] = True
        if bc[1] != "periodic":
            edge[0, :] = edge[-1, :] = True
        H = info["H"].astype(bool)
        assert (T & edge).any() and (H & ~T & edge).any(), "no troubled / hybrid cell at a side"
    lam = np.random.default_rng(15).normal(size=U.shape)
    g = s.apply_operator_adjoint(U, lam)
    go = oracle_vjp(lambda X: o.operator(X, alphas=alphas, T_fixed=T)[0], U, lam)
    e = rel_err(g, go)
    print(f"  max rel err {e:.3e}")
    assert e < TOL, e
    s.close()


def test_trajectory_dot_product_transmissive(hw):
    nx, ny, nsteps, k, bc = 22, 20, 5, 2, ("transmissive", "transmissive")
    print(f"trajectory dot test burgers {nx}x{ny} bc={bc} steps={nsteps} k={k}", flush=True)
    s, o = make_pair(hw, "burgers", nx, ny, 3, "kxrcf", bc)
    U = burgers_data(nx, ny, seed=9, noise=0.02)
    dt = 0.5 * o.cfl_dt(U, 0.6)
    fz, UTo = frozen_of(o, U, dt, nsteps)
    s.set_state(U)
    s.forward_ckpt(nsteps, dt, k)
    UT, _ = s.get_state()
    assert rel_err(UT, UTo) < 1e-11
    lam = np.random.default_rng(25).normal(size=U.shape)
    g = s.adjoint(lam)
    rng = np.random.default_rng(26)
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


# ------------------------------------------------------------------ one RK3 step, element-wise
def frozen_of(o, U, dt, nsteps=1):
    """Per-step lists of the three stages' (alphas, T) of the oracle's own run."""
    out, X = [], U
    for _ in range(nsteps):
        X, infos = o.rk3_step(X, dt)
        out.append([(i["alpha"], i["T"].astype(bool)) for i in infos])
    return out, X


@pytest.mark.parametrize("tc", ["none", "kxrcf", "all"])
def test_step_adjoint_elementwise(hw, tc):
    nx, ny, ng = 12, 11, 3
    print(f"step adjoint burgers {nx}x{ny} ng={ng} tc={tc}", flush=True)
    s, o = make_pair(hw, "burgers", nx, ny, ng, tc)
    U = burgers_data(nx, ny, seed=5, noise=0.02 if tc == "kxrcf" else 0.0)
    dt = 0.5 * o.cfl_dt(U, 0.6)
    fz, U1o = frozen_of(o, U, dt)
    if tc == "kxrcf":
        assert any(0 < T.sum() < T.size for _, T in fz[0]), "no mixed flags"
    s.set_state(U)
    s.flag_export(True)
    s.forward_ckpt(1, dt, 1)
    for st in range(3):
        Tg, _ = s.flags(st)
        assert np.array_equal(Tg.astype(bool), fz[0][st][1]), f"flags of stage {st} differ"
    U1, _ = s.get_state()
    assert rel_err(U1, U1o) < 1e-12
    lam = np.random.default_rng(12).normal(size=U.shape)
    g = s.adjoint(lam)
    go = oracle_vjp(lambda X: o.rk3_step(X, dt, frozen=fz[0])[0], U, lam)
    e = rel_err(g, go)
    print(f"  max rel err {e:.3e}")
    assert e < TOL, e
    s.close()


# ------------------------------------------------------------------ multi-step dot test
@pytest.mark.parametrize("tc,ng", [("kxrcf", 2), ("all", 3)])
def test_trajectory_dot_product(hw, tc, ng):
    nx, ny, nsteps, k = 24, 22, 7, 3
    print(f"trajectory dot test {nx}x{ny} ng={ng} tc={tc} steps={nsteps} k={k}", flush=True)
    s, o = make_pair(hw, "burgers", nx, ny, ng, tc)
    U = burgers_data(nx, ny, seed=8, noise=0.01 if tc == "kxrcf" else 0.0)
    dt = 0.5 * o.cfl_dt(U, 0.6)
    fz, UTo = frozen_of(o, U, dt, nsteps)
    s.set_state(U)
    s.forward_ckpt(nsteps, dt, k)
    UT, _ = s.get_state()
    assert rel_err(UT, UTo) < 1e-11   # state parity proper is covered by the parity tests
    lam = np.random.default_rng(21).normal(size=U.shape)
    g = s.adjoint(lam)
    rng = np.random.default_rng(22)
    for r in range(3):
        d = rng.normal(size=U.shape)
        X = U + 1j * CSH * d
        for n in range(nsteps):
            X, _ = o.rk3_step(X, dt, frozen=fz[n])
        Jd = X.imag / CSH
        lhs, rhs = np.sum(Jd * lam), np.sum(d * g)
        e = abs(lhs - rhs) / (np.linalg.norm(Jd) * np.linalg.norm(lam))
        print(f"  direction {r}: <Jd,lam> = {lhs:.15e}, <d,J^T lam> = {rhs:.15e}, rel {e:.2e}")
        assert e < TOL, e
    s.close()


def test_adjoint_is_deterministic_and_leaves_state(hw):
    nx = ny = 32
    s, o = make_pair(hw, "burgers", nx, ny, 3, "kxrcf")
    U = burgers_data(nx, ny, seed=1, noise=0.01)
    dt = 0.4 * o.cfl_dt(U, 0.6)
    s.set_state(U)
    s.steps(5, dt)
    Uref, _ = s.get_state()
    s.set_state(U)
    s.forward_ckpt(5, dt, 2)
    UT, _ = s.get_state()
    assert np.array_equal(UT, Uref), "recorded run differs from plain stepping"
    lam = np.random.default_rng(4).normal(size=U.shape)
    g1 = s.adjoint(lam)
    g2 = s.adjoint(lam)
    assert np.array_equal(g1, g2)
    assert np.array_equal(s.get_state()[0], UT)
    s.close()


def test_adjoint_rejections(hw):
    from paper_2002_08816_amd import capi
    # the Euler reverse on the double Mach reflection's boundaries needs troubled-cell
    # detection (tests/test_gpu_adjoint_dmr.py)
    s = hw.Solver(2, 64, 16, domain=(0.0, 4.0, 0.0, 1.0), eq="euler", ng_edge=3, bc="dmr",
                  tc_mode="none")
    with pytest.raises(capi.HWError) as ei:
        s.forward_ckpt(1, 1e-3, 1)
    assert ei.value.status == capi.HW_EINVAL
    s.close()
    # scalar laws: periodic and transmissive sides only (1D handles have no reverse mode)
    s = hw.Solver(1, 64, eq="burgers", bc="transmissive")
    with pytest.raises(capi.HWError) as ei:
        s.forward_ckpt(1, 1e-3, 1)
    assert ei.value.status == capi.HW_EINVAL
    s.close()
    s = hw.Solver(2, 16, 16, eq="burgers")
    with pytest.raises(capi.HWError) as ei:
        s.adjoint(np.zeros(s.shape))
    assert ei.value.status == capi.HW_ESTATE
    with pytest.raises(capi.HWError) as ei:
        s.forward_ckpt(3, -1.0, 1)
    assert ei.value.status == capi.HW_EINVAL
    s.close()


# ------------------------------------------------------------------ full size, autograd + FD
def misfit(torch, UT, Ustar, dx, dy):
    d = UT - Ustar
    return 0.5 * dx * dy * (torch.sum(d[0] ** 2) + 12.0 * torch.sum(d[1] ** 2) + 12.0 * torch.sum(d[2] ** 2))


@pytest.mark.parametrize("tc", ["kxrcf", "all"])
def test_full_size_gradient_finite_differences(hw, tc):
    import torch
    n, nsteps, k = 256, 200, 20
    dt = 1.0 / (200.0 * math.pi)
    print(f"full-size gradient 2D Burgers {n}^2 tc={tc} steps={nsteps} k={k}", flush=True)
    s = hw.Solver(2, n, n, domain=(0.0, 4.0, 0.0, 4.0), eq="burgers", ng_edge=3, tc_mode=tc)
    U0n, _ = hi.burgers_modes_2d(0, n=n)
    Usn, _ = hi.burgers_modes_2d(0, n=n, target=True)
    dev = torch.device("cuda")
    U0 = torch.from_numpy(U0n).to(dev).requires_grad_(True)
    Us = torch.from_numpy(Usn).to(dev)
    dx = dy = 4.0 / n
    UT = hw.solve(U0, s, nsteps, dt, k)
    loss = misfit(torch, UT, Us, dx, dy)
    loss.backward()
    g = U0.grad.detach().cpu().numpy()
    assert np.isfinite(g).all() and np.abs(g).max() > 0

    def loss_at(X):
        with torch.no_grad():
            return float(misfit(torch, hw.solve(torch.from_numpy(X).to(dev), s, nsteps, dt, k), Us, dx, dy))

    rng = np.random.default_rng(31)
    for r in range(2):
        d = rng.normal(size=U0n.shape)
        d[1:] /= 12.0      # moments scaled like the data
        eps = 1e-6
        fd = (loss_at(U0n + eps * d) - loss_at(U0n - eps * d)) / (2 * eps)
        an = float(np.sum(g * d))
        e = abs(fd - an) / abs(an)
        print(f"  direction {r}: adjoint {an:.12e}, central FD {fd:.12e}, rel {e:.2e}")
        assert e < 1e-6, e
    s.close()
