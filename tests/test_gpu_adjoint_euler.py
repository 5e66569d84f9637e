"""Reverse mode of the 2D Euler stage (eq. euler2) on the GPU against the oracle, on
periodic meshes and on meshes with transmissive and reflective sides, with troubled-cell
flags, hybrid masks and Lax-Friedrichs speeds held at their forward values.  The characteristic limiter and HWENO reconstruction (Remark 4) are
differentiated including the eigenvectors' dependence on the cell average.

The oracle side is the complex-step derivative of the oracle's own operator / RK3 steps
with the same flags and speeds frozen (its agreement with central differences is pinned on
the CPU in tests/test_oracle_adjoint.py):
* small meshes: (dL/dU)^T lam and (dU1/dU0)^T lam of one step built column by column and
  compared element by element, max|gpu - oracle| / max|oracle| <= 1e-12; with walls, on
  data whose troubled and hybrid cells reach every side (the ghosts mirror the cells
  beside a side, which the reverse folds back onto those cells);
* multi-step runs with checkpoints: dot-product test <J d, lam> = <d, J^T lam>;
* a 64 x 64 smooth vortex, 40 steps through torch.autograd: the gradient of a misfit loss
  against central differences of the oracle's run with the speeds frozen, and the GPU's
  own central differences against the oracle's, relative difference <= 1e-6 each.
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


def shock_vortex(nx, ny, seed=0):
    """The headline generator's shock + vortex state, projected on a small periodic mesh
    of [0, 1] x [0, ny/nx] (KXRCF flags cells along the shock)."""
    prm = hi.euler_shock_vortex_params(seed)
    return hi.project_2d(hi.euler_shock_vortex_func(prm), 0.0, 1.0, 0.0, ny / nx, nx, ny, nq=5)


def smooth_vortex(n, seed=0):
    """Isentropic vortex of radius 0.15 on the uniform state, no shock (a smooth field)."""
    prm = hi.euler_shock_vortex_params(seed)
    prm.update(ratio=1.0, radius=0.15, centre=np.array([0.5, 0.5]))
    return hi.project_2d(hi.euler_shock_vortex_func(prm), 0.0, 1.0, 0.0, 1.0, n, n, nq=5)


def make_pair(hw, nx, ny, ng, tc):
    s = hw.Solver(2, nx, ny, domain=(0.0, 1.0, 0.0, ny / nx), eq="euler", ng_edge=ng, tc_mode=tc)
    o = Scheme2D("euler", nx, ny, 0.0, 1.0, 0.0, ny / nx, ng_edge=ng, tc_mode=tc)
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


def cotangent(shape, seed):
    lam = np.random.default_rng(seed).normal(size=shape)
    return lam


@pytest.mark.parametrize("nx,ny,ng,tc", [
    (10, 9, 2, "kxrcf"),
    (10, 9, 3, "kxrcf"),
    (9, 10, 3, "all"),
    (11, 10, 2, "none"),
])
def test_euler_operator_adjoint_elementwise(hw, nx, ny, ng, tc):
    print(f"Euler operator adjoint {nx}x{ny} ng={ng} tc={tc}", flush=True)
    s, o = make_pair(hw, nx, ny, ng, tc)
    U = shock_vortex(nx, ny)
    alphas = o.alphas(U)
    _, info = o.operator(U)
    T = info["T"].astype(bool)
    if tc == "kxrcf":
        s.flag_export(True)
        s.apply_operator(U)
        Tg, Hg = s.flags(0)
        s.flag_export(False)
        assert np.array_equal(Tg.astype(bool), T), "troubled-cell flags differ"
        assert np.array_equal(Hg.astype(bool), info["H"].astype(bool)), "hybrid masks differ"
        assert 0 < T.sum() < T.size and 0 < info["H"].sum() < T.size   # every branch
    lam = cotangent(U.shape, 11)
    g = s.apply_operator_adjoint(U, lam)
    go = oracle_vjp(lambda X: o.operator(X, alphas=alphas, T_fixed=T)[0], U, lam)
    e = rel_err(g, go)
    print(f"  max rel err {e:.3e}")
    assert e < TOL, e
    s.close()


WALLS = [
    (("transmissive", "transmissive"), 2, "kxrcf"),
    (("reflective", "reflective"), 2, "kxrcf"),
    (("transmissive", "reflective"), 3, "all"),
    (("reflective", "periodic"), 2, "kxrcf"),
    (("periodic", "transmissive"), 3, "kxrcf"),
    (("reflective", "transmissive"), 2, "none"),
]


def make_wall_pair(hw, nx, ny, ng, tc, bc):
    kw = dict(domain=(0.0, 1.0, 0.0, ny / nx), eq="euler", ng_edge=ng, tc_mode=tc, bc=bc)
    s = hw.Solver(2, nx, ny, **kw)
    o = Scheme2D("euler", nx, ny, 0.0, 1.0, 0.0, ny / nx, ng_edge=ng, tc_mode=tc, bc=bc)
    return s, o


def side_cells(shape, bc):
    edge = np.zeros(shape, dtype=bool)
    if bc[0] != "periodic":
        edge[:, 0] = edge[:, -1] = True
    if bc[1] != "periodic":
        edge[0, :] = edge[-1, :] = True
    return edge


@pytest.mark.parametrize("bc,ng,tc", WALLS)
def test_euler_operator_adjoint_walls(hw, bc, ng, tc):
    nx, ny = 10, 9
    print(f"Euler operator adjoint {nx}x{ny} bc={bc} ng={ng} tc={tc}", flush=True)
    s, o = make_wall_pair(hw, nx, ny, ng, tc, bc)
    U = hi.euler_wall_state(nx, ny, 5)
    alphas = o.alphas(U)
    _, info = o.operator(U)
    T = info["T"].astype(bool)
    if tc == "kxrcf":
        s.flag_export(True)
        s.apply_operator(U)
        Tg, Hg = s.flags(0)
        s.flag_export(False)
        assert np.array_equal(Tg.astype(bool), T), "troubled-cell flags differ"
        assert np.array_equal(Hg.astype(bool), info["H"].astype(bool)), "hybrid masks differ"
        edge = side_cells(T.shape, bc)
        assert (T & edge).any() and (info["H"].astype(bool) & edge & ~T).any()
        assert (~T & ~info["H"].astype(bool) & edge).any()   # linear cells by a side too
    lam = cotangent(U.shape, 13)
    g = s.apply_operator_adjoint(U, lam)
    go = oracle_vjp(lambda X: o.operator(X, alphas=alphas, T_fixed=T)[0], U, lam)
    e = rel_err(g, go)
    print(f"  max rel err {e:.3e}")
    assert e < TOL, e
    s.close()


def test_euler_step_adjoint_walls(hw):
    nx, ny, ng, bc = 9, 9, 2, ("reflective", "transmissive")
    print(f"Euler step adjoint {nx}x{ny} bc={bc} ng={ng} tc=kxrcf", flush=True)
    s, o = make_wall_pair(hw, nx, ny, ng, "kxrcf", bc)
    U = hi.euler_wall_state(nx, ny, 6)
    dt = 0.5 * o.cfl_dt(U, 0.6)
    fz, U1o = frozen_of(o, U, dt)
    s.set_state(U)
    s.forward_ckpt(1, dt, 1)
    U1, _ = s.get_state()
    assert rel_err(U1, U1o) < 1e-12
    lam = cotangent(U.shape, 14)
    g = s.adjoint(lam)
    go = oracle_vjp(lambda X: o.rk3_step(X, dt, frozen=fz[0])[0], U, lam)
    e = rel_err(g, go)
    print(f"  max rel err {e:.3e}")
    assert e < TOL, e
    s.close()


def test_euler_trajectory_dot_product_walls(hw):
    nx, ny, nsteps, k, bc = 18, 16, 4, 2, ("transmissive", "reflective")
    print(f"Euler trajectory dot test {nx}x{ny} bc={bc} steps={nsteps} k={k}", flush=True)
    s, o = make_wall_pair(hw, nx, ny, 2, "kxrcf", bc)
    U = hi.euler_wall_state(nx, ny, 8)
    dt = 0.5 * o.cfl_dt(U, 0.6)
    fz, UTo = frozen_of(o, U, dt, nsteps)
    s.set_state(U)
    s.forward_ckpt(nsteps, dt, k)
    UT, _ = s.get_state()
    assert rel_err(UT, UTo) < 1e-11
    lam = cotangent(U.shape, 23)
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


def frozen_of(o, U, dt, nsteps=1):
    out, X = [], U
    for _ in range(nsteps):
        X, infos = o.rk3_step(X, dt)
        out.append([(i["alpha"], i["T"].astype(bool)) for i in infos])
    return out, X


def test_euler_step_adjoint_elementwise(hw):
    nx, ny, ng = 9, 9, 2
    print(f"Euler step adjoint {nx}x{ny} ng={ng} tc=kxrcf", flush=True)
    s, o = make_pair(hw, nx, ny, ng, "kxrcf")
    U = shock_vortex(nx, ny, seed=1)
    dt = 0.5 * o.cfl_dt(U, 0.6)
    fz, U1o = frozen_of(o, U, dt)
    assert any(0 < T.sum() < T.size for _, T in fz[0]), "no mixed flags"
    s.set_state(U)
    s.flag_export(True)
    s.forward_ckpt(1, dt, 1)
    for st in range(3):
        Tg, _ = s.flags(st)
        assert np.array_equal(Tg.astype(bool), fz[0][st][1]), f"flags of stage {st} differ"
    U1, _ = s.get_state()
    assert rel_err(U1, U1o) < 1e-12
    lam = cotangent(U.shape, 12)
    g = s.adjoint(lam)
    go = oracle_vjp(lambda X: o.rk3_step(X, dt, frozen=fz[0])[0], U, lam)
    e = rel_err(g, go)
    print(f"  max rel err {e:.3e}")
    assert e < TOL, e
    s.close()


@pytest.mark.parametrize("tc,ng", [("kxrcf", 2), ("all", 3)])
def test_euler_trajectory_dot_product(hw, tc, ng):
    nx, ny, nsteps, k = 18, 16, 5, 2
    print(f"Euler trajectory dot test {nx}x{ny} ng={ng} tc={tc} steps={nsteps} k={k}", flush=True)
    s, o = make_pair(hw, nx, ny, ng, tc)
    U = shock_vortex(nx, ny, seed=2)
    dt = 0.5 * o.cfl_dt(U, 0.6)
    fz, UTo = frozen_of(o, U, dt, nsteps)
    s.set_state(U)
    s.forward_ckpt(nsteps, dt, k)
    UT, _ = s.get_state()
    assert rel_err(UT, UTo) < 1e-11
    lam = cotangent(U.shape, 21)
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


def test_euler_adjoint_is_deterministic_and_leaves_state(hw):
    n = 32
    s, o = make_pair(hw, n, n, 2, "kxrcf")
    U = shock_vortex(n, n, seed=3)
    dt = 0.4 * o.cfl_dt(U, 0.6)
    s.set_state(U)
    s.steps(5, dt)
    Uref, _ = s.get_state()
    s.set_state(U)
    s.forward_ckpt(5, dt, 2)
    UT, _ = s.get_state()
    assert np.array_equal(UT, Uref), "recorded run differs from plain stepping"
    lam = cotangent(U.shape, 4)
    g1 = s.adjoint(lam)
    g2 = s.adjoint(lam)
    assert np.array_equal(g1, g2)
    assert np.array_equal(s.get_state()[0], UT)
    s.close()


def test_euler_gradient_finite_differences(hw):
    """The adjoint holds the Lax-Friedrichs speeds fixed (their dependence on the state
    is through a max over cells); central differences of the real forward run see that
    dependence too.  So the gradient is compared with central differences of the oracle's
    run with the speeds and flags frozen at the unperturbed run's, and the GPU's own
    central differences with the oracle's unfrozen ones."""
    import torch
    n, nsteps, k = 64, 40, 10
    print(f"Euler gradient {n}^2 smooth vortex, steps={nsteps} k={k}", flush=True)
    s = hw.Solver(2, n, n, eq="euler", ng_edge=2, tc_mode="kxrcf")
    o = Scheme2D("euler", n, n, ng_edge=2, tc_mode="kxrcf")
    U0n = smooth_vortex(n)
    dt = 0.5 * o.cfl_dt(U0n, 0.6)
    rng = np.random.default_rng(41)
    Usn = U0n * (1.0 + 0.01 * rng.normal(size=U0n.shape))
    dev = torch.device("cuda")
    U0 = torch.from_numpy(U0n).to(dev).requires_grad_(True)
    Us = torch.from_numpy(Usn).to(dev)

    def misfit(UT, Ust):
        d = UT - Ust
        return 0.5 * ((d[0] ** 2).sum() + 12.0 * (d[1] ** 2).sum() + 12.0 * (d[2] ** 2).sum()) / n ** 2

    UT = hw.solve(U0, s, nsteps, dt, k)
    loss = misfit(UT, Us)
    loss.backward()
    g = U0.grad.detach().cpu().numpy()
    assert np.isfinite(g).all() and np.abs(g).max() > 0

    # the oracle's run: flags (none on this smooth field) and speeds of every stage
    X, fz = U0n, []
    for _ in range(nsteps):
        X, infos = o.rk3_step(X, dt)
        fz.append([(i["alpha"], i["T"].astype(bool)) for i in infos])
    assert not any(T.any() for st in fz for _, T in st), "the smooth vortex raises no flag"

    def oracle_loss(U, frozen):
        for m in range(nsteps):
            U, _ = o.rk3_step(U, dt, frozen=fz[m] if frozen else None)
        return float(misfit(U, Usn))

    def gpu_loss(X):
        with torch.no_grad():
            return float(misfit(hw.solve(torch.from_numpy(X).to(dev), s, nsteps, dt, k), Us))

    d = rng.normal(size=U0n.shape)
    d[1:] /= 12.0
    eps = 1e-6

    def cd(F):
        return (F(U0n + eps * d) - F(U0n - eps * d)) / (2 * eps)

    fd_frozen = cd(lambda X: oracle_loss(X, True))
    fd_free = cd(lambda X: oracle_loss(X, False))
    fd_gpu = cd(gpu_loss)
    an = float(np.sum(g * d))
    e1 = abs(an - fd_frozen) / abs(fd_frozen)
    e2 = abs(fd_gpu - fd_free) / abs(fd_free)
    print(f"  adjoint {an:.12e}, oracle FD (speeds frozen) {fd_frozen:.12e}, rel {e1:.2e}")
    print(f"  GPU FD {fd_gpu:.12e}, oracle FD {fd_free:.12e}, rel {e2:.2e}; "
          f"the speeds' own share {abs(fd_free - fd_frozen) / abs(fd_free):.2e}")
    assert e1 < 1e-6, e1
    assert e2 < 1e-6, e2
    s.close()
