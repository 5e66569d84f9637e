"""Pins of the oracle's semi-discrete operators and time integration (oracle/scheme1d.py,
oracle/scheme2d.py) against facts the paper and the mathematics fix:

* consistency: for a linear flux and polynomial data the operator returns the exact
  moments of -(a u_x + b u_y) (the Lax-Friedrichs jump vanishes, the reconstruction and
  the quadrature rules are exact to the stated degree; eqs. odeH, ode2)
* conservation: periodic runs keep sum(ubar) to round-off (telescoping fluxes)
* fifth order on smooth linear advection, with no troubled cells and with every cell
  troubled under random linear weights per step (Section 3.1)
* Table 3 of the paper (2D Burgers, 40 x 40, new hybrid: no troubled cell) reproduced
* magnitudes of Tables 1, 2 and 4 and of the "New HWENO" columns
* troubled-cell behaviour: smooth data raise no flag, a jump raises flags next to it
* boundary handling: transmissive boundaries keep a constant state and mirror symmetry
* characteristic HWENO with the weights forced to the linear weights equals the
  component-wise linear reconstruction (linear maps commute with the projection)
"""
import math

import numpy as np
import pytest

import hweno_inputs as hi
from oracle import scheme1d, scheme2d, weno
from oracle.physics import Equation


def poly_moments_1d(coef, x0, dx, ncell):
    f = lambda x: sum(c * np.asarray(x) ** m for m, c in enumerate(coef))[None]
    return hi.project_1d(f, x0, x0 + ncell * dx, ncell, nq=8)


# ----------------------------------------------------------------------------- consistency


@pytest.mark.parametrize("mode,deg", [("none", 5), ("all", 1)])
def test_1d_operator_exact_for_polynomials(mode, deg):
    rng = np.random.default_rng(deg)
    n = 9
    dx = 0.1
    a = -0.8
    s = scheme1d.Scheme1D(Equation("advection", 1, adv=(a,)), n, 0.0, n * dx, tc_mode=mode)
    coef = rng.normal(size=deg + 1)
    Up = poly_moments_1d(coef, -3 * dx, dx, n + 6)
    dcoef = [m * coef[m] for m in range(1, deg + 1)]
    Le = -a * poly_moments_1d(dcoef, 0.0, dx, n) / dx if dcoef else np.zeros((2, 1, n))
    # d/dx in physical units: the moments of u_x
    f = lambda x: (-a * sum(m * coef[m] * np.asarray(x) ** (m - 1) for m in range(1, deg + 1)))[None]
    Le = hi.project_1d(f, 0.0, n * dx, n, nq=8)
    L, T, H, _ = s.operator_padded(Up, abs(a))
    assert np.abs(L - Le).max() < 1e-11 * max(1.0, np.abs(Le).max())
    assert T[3:-3].all() == (mode == "all")


@pytest.mark.parametrize("mode,ng,deg", [("none", 3, 4), ("none", 2, 3), ("all", 3, 1), ("all", 2, 1)])
def test_2d_operator_exact_for_polynomials(mode, ng, deg):
    rng = np.random.default_rng(10 * ng + deg)
    n = 6
    dx = 0.25
    a, b = 0.7, -0.4
    s = scheme2d.Scheme2D(Equation("advection", 2, adv=(a, b)), n, n, 0, n * dx, 0, n * dx,
                          tc_mode=mode, ng_edge=ng)
    mons = [(p, t - p) for t in range(deg + 1) for p in range(t, -1, -1)]
    c = rng.normal(size=len(mons))
    u = lambda x, y: sum(ci * x ** p * y ** q for ci, (p, q) in zip(c, mons))[None]

    def ut(x, y):
        r = 0.0 * x
        for ci, (p, q) in zip(c, mons):
            if p > 0:
                r = r - a * ci * p * x ** (p - 1) * y ** q
            if q > 0:
                r = r - b * ci * q * x ** p * y ** (q - 1)
        return r[None]

    Up = hi.project_2d(u, -3 * dx, (n + 3) * dx, -3 * dx, (n + 3) * dx, n + 6, n + 6, nq=6)
    Le = hi.project_2d(ut, 0, n * dx, 0, n * dx, n, n, nq=6)
    L, info = s.operator_padded(Up, abs(a), abs(b))
    assert np.abs(L - Le).max() < 1e-11 * max(1.0, np.abs(Le).max())


# ----------------------------------------------------------------------------- conservation


def test_1d_periodic_conservation_burgers_with_flags():
    n = 64
    U0 = hi.example_3_1(n)
    s = scheme1d.Scheme1D("burgers", n, 0.0, 2.0, tc_mode="kxrcf")
    U, t, k, infos = s.run(U0, T=1.5 / math.pi, cfl=0.6)   # past the shock time (Ex. 3.5)
    assert sum(i["T"].sum() for i in infos) > 0
    m0, m1 = U0[0].sum(), U[0].sum()
    assert abs(m1 - m0) <= 1e-13 * abs(m0)


def test_2d_periodic_conservation_euler_with_flags():
    n = 32
    U0, _ = hi.euler_shock_vortex_2d(0, n)
    s = scheme2d.Scheme2D("euler", n, n, ng_edge=2, tc_mode="kxrcf")
    U, t, k, infos = s.run(U0, nsteps=4, cfl=0.6)
    assert sum(i["T"].sum() for i in infos) > 0
    for c in range(4):
        m0, m1 = U0[0, c].sum(), U[0, c].sum()
        assert abs(m1 - m0) <= 1e-12 * np.abs(U0[0, c]).sum()


# ----------------------------------------------------------------------------- accuracy


def advection_errors(mode, ns, weights_rng=None):
    out = []
    for n in ns:
        U0, _ = hi.advection_1d(0, n)
        s = scheme1d.Scheme1D(Equation("advection", 1, adv=(1.0,)), n, 0.0, 2.0, tc_mode=mode)
        dx = 2.0 / n
        dt = 0.5 * dx * (dx / (2.0 / ns[0])) ** (2.0 / 3.0)
        wf = None
        if weights_rng is not None:
            def wf(k):
                g = weights_rng.uniform(0.05, 1.0, 3)
                h = weights_rng.uniform(0.05, 1.0, 3)
                return tuple(g / g.sum()), tuple(h / h.sum())
        U, t, k, _ = s.run(U0, T=2.0, dt=dt, weights_fn=wf)
        e = np.abs(U[0, 0] - U0[0, 0])     # the exact solution after one period is u0
        out.append((e.mean(), e.max()))
    return out


def orders(errs, ns):
    return [(math.log(errs[i][0] / errs[i + 1][0]) / math.log(ns[i + 1] / ns[i]),
             math.log(errs[i][1] / errs[i + 1][1]) / math.log(ns[i + 1] / ns[i]))
            for i in range(len(ns) - 1)]


def test_fifth_order_linear_advection_plain():
    ns = (40, 80, 160)
    o = orders(advection_errors("none", ns), ns)
    assert o[-1][0] >= 4.7 and o[-1][1] >= 4.7, o


def test_fifth_order_linear_advection_all_troubled_random_weights():
    ns = (40, 80, 160)
    o = orders(advection_errors("all", ns, np.random.default_rng(123)), ns)
    assert o[-1][0] >= 4.7 and o[-1][1] >= 4.7, o


def test_limited_moments_must_enter_the_stage_combination():
    """Pins the reading that the limited first moments of a stage input replace the stored
    ones in the TVD-RK3 combination (eq. RK applied to the state the limiter returns).
    The paper's all-troubled scheme is fifth order on smooth data (Table 1); combining the
    unmodified stored moments instead makes it inconsistent: on linear advection with every
    cell troubled its error stalls near 1e-2 while the write-back form converges."""
    def step_without_write_back(o, U, dt):
        L0, _ = o.operator(U)
        U1 = U + dt * L0
        L1, _ = o.operator(U1)
        U2 = 0.75 * U + 0.25 * U1 + 0.25 * dt * L1
        L2, _ = o.operator(U2)
        return U / 3.0 + 2.0 / 3.0 * U2 + 2.0 / 3.0 * dt * L2

    errs = {}
    for n in (40, 80):
        U0, _ = hi.advection_1d(0, n)
        o = scheme1d.Scheme1D("advection", n, 0.0, 2.0, tc_mode="all")
        dt = 0.2 * 2.0 / n
        A, B = U0.copy(), U0.copy()
        for _ in range(int(round(2.0 / dt))):
            A, _ = o.rk3_step(A, dt)
            B = step_without_write_back(o, B, dt)
        errs[n] = (np.abs(A[0] - U0[0]).max(), np.abs(B[0] - U0[0]).max())
    assert errs[80][0] < 1e-5 and errs[40][0] / errs[80][0] > 8.0        # converging
    assert errs[80][1] > 1e-2 and errs[40][1] / errs[80][1] < 4.0        # not


def burgers2d_exact(n, T):
    def u(x, y):
        s = x + y
        w = 0.5 + np.sin(math.pi * s / 2)
        for _ in range(60):
            F = w - (0.5 + np.sin(math.pi * (s - 2 * w * T) / 2))
            dF = 1 + math.pi * T * np.cos(math.pi * (s - 2 * w * T) / 2)
            w = w - F / dF
        return w[None]
    return hi.project_2d(u, 0, 4, 0, 4, n, n, nq=6)


def test_table3_new_hybrid_40x40():
    """Table 3, new hybrid scheme, 40 x 40: L1 2.70E-06, Linf 2.49E-05 (no troubled cell in
    this smooth test, so the scheme is the linear one; small time step so that the spatial
    error dominates)."""
    n = 40
    T = 0.5 / math.pi
    U0 = hi.example_3_3(n)
    s = scheme2d.Scheme2D("burgers", n, n, 0, 4, 0, 4, tc_mode="kxrcf", ng_edge=3)
    U, t, k, infos = s.run(U0, T=T, dt=0.02 * 4.0 / n)
    assert all(i["T"].sum() == 0 for i in infos)
    e = np.abs(U[0, 0] - burgers2d_exact(n, T)[0, 0])
    assert abs(e.mean() / 2.70e-6 - 1.0) < 0.1
    assert abs(e.max() / 2.49e-5 - 1.0) < 0.1


def test_table3_new_hweno_80x80_magnitude():
    """Table 3, New HWENO (every cell troubled), 80 x 80: Linf 2.25E-06."""
    n = 80
    T = 0.5 / math.pi
    U0 = hi.example_3_3(n)
    s = scheme2d.Scheme2D("burgers", n, n, 0, 4, 0, 4, tc_mode="all", ng_edge=3)
    U, t, k, infos = s.run(U0, T=T, dt=0.02 * 4.0 / n)
    e = np.abs(U[0, 0] - burgers2d_exact(n, T)[0, 0])
    assert 0.5 < e.max() / 2.25e-6 < 2.0
    assert 0.3 < e.mean() / 2.86e-7 < 3.0


def burgers1d_exact(n, T):
    def u(x):
        x = np.asarray(x, float)
        w = 0.5 + np.sin(math.pi * x)
        for _ in range(100):
            F = w - (0.5 + np.sin(math.pi * (x - w * T)))
            dF = 1 + math.pi * T * np.cos(math.pi * (x - w * T))
            w = w - F / dF
        return w[None]
    return hi.project_1d(u, 0.0, 2.0, n, nq=12)


def test_table1_magnitudes():
    """Table 1 (1D Burgers, T = 0.5/pi): new hybrid and New HWENO columns at N = 80, 160.
    The paper does not state its time step; with a small one the errors agree to within
    an order of magnitude and decrease at fifth order or better."""
    T = 0.5 / math.pi
    paper = {("none", 80): 1.46e-8, ("none", 160): 2.66e-10,
             ("all", 80): 4.20e-7, ("all", 160): 8.83e-9}
    for mode in ("none", "all"):
        errs = []
        for n in (80, 160):
            s = scheme1d.Scheme1D("burgers", n, 0.0, 2.0, tc_mode=mode)
            U, t, k, _ = s.run(hi.example_3_1(n), T=T, dt=0.01 * 2.0 / n)
            e = np.abs(U[0, 0] - burgers1d_exact(n, T)[0, 0]).mean()
            errs.append(e)
            assert 0.05 < e / paper[(mode, n)] < 10.0, (mode, n, e)
        assert math.log2(errs[0] / errs[1]) > 4.7


def test_table2_magnitude():
    """Table 2 (1D Euler density wave), new hybrid, N = 40: L1 1.02E-09 (domain [0, 2])."""
    n = 40
    s = scheme1d.Scheme1D("euler", n, 0.0, 2.0, tc_mode="kxrcf")
    U0 = hi.example_3_2(n)
    U, t, k, infos = s.run(U0, T=2.0, dt=0.01 * 2.0 / n)
    assert all(i["T"].sum() == 0 for i in infos)
    e = np.abs(U[0, 0] - U0[0, 0]).mean()
    assert 0.05 < e / 1.02e-9 < 10.0


@pytest.mark.slow
def test_table4_magnitude():
    """Table 4 (2D Euler density wave), new hybrid, 30 x 30: L1 3.11E-07."""
    n = 30
    s = scheme2d.Scheme2D("euler", n, n, 0, 2, 0, 2, tc_mode="kxrcf", ng_edge=3)
    U0 = hi.example_3_4(n)
    U, t, k, infos = s.run(U0, T=2.0, dt=0.05 * 2.0 / n)
    e = np.abs(U[0, 0] - U0[0, 0]).mean()
    assert 0.1 < e / 3.11e-7 < 10.0


# ----------------------------------------------------------------------------- flags


def test_smooth_data_raise_no_flags():
    s = scheme1d.Scheme1D("burgers", 80, 0.0, 2.0)
    assert s.operator(hi.example_3_1(80))[1]["T"].sum() == 0
    s = scheme2d.Scheme2D("burgers", 40, 40, 0, 4, 0, 4)
    assert s.operator(hi.example_3_3(40))[1]["T"].sum() == 0
    s = scheme1d.Scheme1D("euler", 80, 0.0, 2.0)
    assert s.operator(hi.example_3_2(80))[1]["T"].sum() == 0


def test_jump_raises_flags_at_the_jump():
    n = 200
    f = lambda x: hi.primitive_to_conserved(np.where(np.asarray(x) < 0.5, 1.0, 0.125),
                                            [np.zeros_like(np.asarray(x, float))],
                                            np.where(np.asarray(x) < 0.5, 1.0, 0.1))
    U0 = hi.project_1d(f, 0.0, 1.0, n, breakpoints=[0.5 + 0.3 / n])
    s = scheme1d.Scheme1D("euler", n, 0.0, 1.0, bc="transmissive")
    U, t, k, infos = s.run(U0, nsteps=5, cfl=0.6)
    T = infos[0]["T"]
    idx = np.nonzero(T)[0]
    assert idx.size > 0
    assert np.all(np.abs(idx - n // 2) <= 10)


# ----------------------------------------------------------------------------- boundaries


def test_transmissive_constant_state_is_steady():
    n = 20
    U0 = np.zeros((2, 3, n))
    U0[0] = hi.primitive_to_conserved(np.full(n, 0.7), [np.full(n, 0.3)], np.full(n, 0.9))
    s = scheme1d.Scheme1D("euler", n, 0.0, 1.0, bc="transmissive")
    L, info = s.operator(U0)
    assert np.abs(L).max() < 1e-13
    U0 = np.zeros((3, 4, 8, 10))
    one = np.ones((8, 10))
    U0[0] = hi.primitive_to_conserved(0.7 * one, [0.3 * one, -0.2 * one], 0.9 * one)
    s = scheme2d.Scheme2D("euler", 10, 8, bc=("transmissive", "transmissive"))
    L, info = s.operator(U0)
    assert np.abs(L).max() < 1e-13


def test_transmissive_mirror_symmetry():
    n = 60
    U0, _ = hi.euler_riemann_1d(1, n)
    # symmetrise: rho, E even and momentum odd about x = 1/2; first moments flip parity
    S = U0.copy()
    S[0] = 0.5 * (U0[0] + U0[0][:, ::-1] * np.array([[1.0], [-1.0], [1.0]]))
    S[1] = 0.5 * (U0[1] - U0[1][:, ::-1] * np.array([[1.0], [-1.0], [1.0]]))
    s = scheme1d.Scheme1D("euler", n, 0.0, 1.0, bc="transmissive")
    U, t, k, _ = s.run(S, nsteps=10, cfl=0.6)
    sign = np.array([[1.0], [-1.0], [1.0]])
    assert np.abs(U[0] - U[0][:, ::-1] * sign).max() < 1e-12
    assert np.abs(U[1] + U[1][:, ::-1] * sign).max() < 1e-12


# ----------------------------------------------------------------------------- characteristic


def test_characteristic_hweno_with_linear_weights_is_linear(monkeypatch):
    monkeypatch.setattr(scheme1d, "nonlinear_weights",
                        lambda betas, g, eps: np.array(g)[:, None] * np.ones_like(np.asarray(betas)))
    monkeypatch.setattr(scheme2d, "nonlinear_weights",
                        lambda betas, g, eps: np.array(g)[:, None] * np.ones_like(np.asarray(betas)))
    n = 40
    U0, _ = hi.euler_riemann_1d(0, n)
    s = scheme1d.Scheme1D("euler", n, 0.0, 1.0, bc="transmissive")
    Up = s.pad(U0)
    idx = np.arange(2, n + 4)
    lh, rh = s._traces(Up, Up[1], np.ones(n + 6, bool), idx)
    ll, rl = s._traces(Up, Up[1], np.zeros(n + 6, bool), idx)
    assert np.abs(lh - ll).max() < 1e-12 and np.abs(rh - rl).max() < 1e-12
    U0, _ = hi.euler_shock_vortex_2d(1, 12)
    s = scheme2d.Scheme2D("euler", 12, 12, ng_edge=3)
    Up = s.pad(U0)
    vh, _ = s._edge_values(Up, Up[1], Up[2], np.ones(Up.shape[-2:], bool))
    vl, _ = s._edge_values(Up, Up[1], Up[2], np.zeros(Up.shape[-2:], bool))
    for k in "LRBT":
        assert np.abs(vh[k] - vl[k]).max() < 1e-11 * np.abs(vl[k]).max()


def test_limiter_accuracy_on_smooth_data():
    """Step 1: with smooth data the modified first moment is a fifth-order approximation
    of the exact one."""
    errs = []
    for n in (40, 80):
        U0 = hi.example_3_1(n)
        s = scheme1d.Scheme1D("burgers", n, 0.0, 2.0, tc_mode="all")
        lim = s.operator(U0)[1]["limited"]
        errs.append(np.abs(lim[1] - U0[1]).max())
    assert math.log2(errs[0] / errs[1]) > 4.5
