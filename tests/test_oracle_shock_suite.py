"""Shock tests of Section 3.2 on the oracle, and the pins of the exact Riemann solver
they are measured against (CPU only).

* The exact solver (oracle/riemann.py) is pinned to the star states tabulated for two
  standard Riemann problems in Toro's textbook (Sod's shock tube; the symmetric double
  rarefaction), to the Rankine-Hugoniot conditions across the shocks it computes, to
  isentropy and the Riemann invariant across its rarefactions, to mirror symmetry and to
  a uniform state.
* The scheme on the Lax problem (Example 3.6, N = 200, T = 0.16) converges to that
  solution: the L1 error of the density averages is below 1e-2 at N = 200 and falls as
  the mesh is refined (at the rate of a scheme whose error is set by the discontinuities).
* Troubled cells (Step 1 flags): the time-averaged share of troubled cells on the Lax,
  Shu-Osher (Example 3.7, N = 400, T = 1.8) and discontinuous Burgers (Example 3.5,
  N = 80, T = 1.5/pi) problems is reported, is a small fraction of the mesh, and the last
  step's troubled cells of the Lax problem all lie next to a wave of the exact solution.
  The paper quotes 13.41 % (Lax), 3.54 % (Shu-Osher) and 13.94 % (blast) without stating
  how the share is averaged; the oracle gives 6.0 %, 2.6 % and 5.7 % as the mean over all
  Runge-Kutta stages of the troubled share, so the comparison is one of magnitude only.
* Reflective walls (the blast problem, Example 3.8): the scheme on [0, 1] with a wall at
  each end equals, to round-off and with mirrored troubled sets, the periodic scheme on
  [-1, 1] started from the mirror-extended state (density and energy even, momentum odd),
  restricted to [0, 1]; the periodic scheme is pinned on its own by the tests above.
"""
import math

import numpy as np
import pytest

import hweno_inputs as hi
from oracle.riemann import RiemannExact
from oracle.scheme1d import Scheme1D

G = 1.4
LAX = ((0.445, 0.698, 3.528), (0.5, 0.0, 0.571))


def conserved(rho, u, p):
    return np.array([rho, rho * u, p / (G - 1.0) + 0.5 * rho * u * u])


def flux(rho, u, p):
    E = p / (G - 1.0) + 0.5 * rho * u * u
    return np.array([rho * u, rho * u * u + p, u * (E + p)])


def run_with_flags(o, U, T, cfl=0.6):
    """Runs to T (last step clipped); returns the state, the step count and the troubled
    and hybrid cell counts of every stage, shape (steps, 3)."""
    t, k, nt, nh, last = 0.0, 0, [], [], None
    while t < T:
        h = o.cfl_dt(U, cfl)
        if t + h > T:
            h = T - t
        U, infos = o.rk3_step(U, h)
        nt.append([int(i["T"].sum()) for i in infos])
        nh.append([int(i["H"].sum()) for i in infos])
        last = infos
        t += h
        k += 1
    return U, k, np.array(nt), np.array(nh), last


# ------------------------------------------------------------------ exact Riemann solver


@pytest.mark.parametrize("left,right,ref", [
    # Sod's shock tube: p*, u*, rho*_L, rho*_R
    ((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), (0.30313, 0.92745, 0.42632, 0.26557)),
    # two symmetric rarefactions ("123 problem")
    ((1.0, -2.0, 0.4), (1.0, 2.0, 0.4), (0.00189, 0.0, 0.02185, 0.02185)),
])
def test_riemann_textbook_star_states(left, right, ref):
    r = RiemannExact(left, right, G)
    got = (r.ps, r.us, r.rho_star[0], r.rho_star[1])
    for a, b in zip(got, ref):
        assert abs(a - b) <= 6e-6, (got, ref)


@pytest.mark.parametrize("left,right,side", [
    (LAX[0], LAX[1], 1),                          # Lax: right-moving shock
    ((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 1),      # Sod: right-moving shock
    ((0.125, 0.0, 0.1), (1.0, 0.0, 1.0), 0),      # mirrored Sod: left-moving shock
])
def test_riemann_shocks_satisfy_rankine_hugoniot(left, right, side):
    r = RiemannExact(left, right, G)
    far = right if side == 1 else left
    star = (r.rho_star[side], r.us, r.ps)
    # the shock speed from the mass balance, then momentum and energy must balance too
    Uf, Us = conserved(*far), conserved(*star)
    Ff, Fs = flux(*far), flux(*star)
    S = (Fs[0] - Ff[0]) / (Us[0] - Uf[0])
    for c in (1, 2):
        assert abs((Fs[c] - Ff[c]) - S * (Us[c] - Uf[c])) <= 1e-12 * max(abs(Fs[c]), abs(Ff[c]), 1.0)
    # and the sampled solution jumps there: far state just outside, star state inside
    t = 0.1
    x_out = S * t + (1e-9 if side == 1 else -1e-9)
    x_in = S * t - (1e-9 if side == 1 else -1e-9)
    assert np.allclose(r.sample(np.array([x_out]), t)[:, 0], far, rtol=0, atol=1e-12)
    assert np.allclose(r.sample(np.array([x_in]), t)[:, 0], star, rtol=0, atol=1e-12)


def test_riemann_rarefaction_isentropic_with_constant_invariant():
    r = RiemannExact(*LAX, gamma=G)   # the Lax problem's left wave is a rarefaction
    rl, ul, pl = LAX[0]
    cl = math.sqrt(G * pl / rl)
    t = 0.16
    cs = cl * (r.ps / pl) ** ((G - 1.0) / (2.0 * G))
    head, tail = (ul - cl) * t, (r.us - cs) * t
    x = np.linspace(head, tail, 41)
    rho, u, p = r.sample(x, t)
    c = np.sqrt(G * p / rho)
    assert np.allclose(p / rho ** G, pl / rl ** G, rtol=1e-12, atol=0)
    assert np.allclose(u + 2.0 * c / (G - 1.0), ul + 2.0 * cl / (G - 1.0), rtol=1e-12, atol=0)
    # the fan's characteristic family: u - c = x / t
    assert np.allclose(u - c, x / t, rtol=0, atol=1e-12)
    # continuous at both ends of the fan
    for xe, st in ((head, LAX[0]), (tail, (r.rho_star[0], r.us, r.ps))):
        v = r.sample(np.array([xe - 1e-12, xe + 1e-12]), t)
        assert np.allclose(v[:, 0], v[:, 1], rtol=1e-9, atol=1e-9)
        assert np.allclose(v[:, 0], st, rtol=1e-9, atol=1e-9)


def test_riemann_mirror_symmetry_and_uniform_state():
    a = RiemannExact(*LAX, gamma=G)
    (rl, ul, pl), (rr, ur, pr) = LAX
    b = RiemannExact((rr, -ur, pr), (rl, -ul, pl), G)
    x = np.linspace(-0.5, 0.5, 101)[1:-1]
    va, vb = a.sample(x, 0.16), b.sample(-x, 0.16)
    off = [i for i in range(x.size) if not np.isclose(abs(x[i]), 0.0)]
    assert np.allclose(va[0, off], vb[0, off], rtol=1e-12, atol=1e-12)
    assert np.allclose(va[1, off], -vb[1, off], rtol=1e-12, atol=1e-12)
    assert np.allclose(va[2, off], vb[2, off], rtol=1e-12, atol=1e-12)
    u = RiemannExact((0.7, 0.3, 2.0), (0.7, 0.3, 2.0), G)
    assert abs(u.ps - 2.0) < 1e-12 and abs(u.us - 0.3) < 1e-12
    assert np.allclose(u.sample(x, 1.0), np.array([0.7, 0.3, 2.0])[:, None], rtol=0, atol=1e-12)


# ------------------------------------------------------------------ the scheme's shock tests


def lax_run(n):
    o = Scheme1D("euler", n, -0.5, 0.5, bc="transmissive", tc_mode="kxrcf")
    return run_with_flags(o, hi.example_3_6(n), 0.16)


def test_lax_converges_to_the_exact_solution():
    exact = RiemannExact(*LAX, gamma=G)
    errs = []
    for n in (100, 200, 400):
        U, k, nt, _, _ = lax_run(n)
        ex = exact.cell_averages(-0.5, 0.5, n, 0.16, per_cell=200)
        errs.append(np.abs(U[0, 0] - ex[0]).mean())   # L1 of the density averages
        assert np.isfinite(U).all()
        p = (G - 1.0) * (U[0, 2] - 0.5 * U[0, 1] ** 2 / U[0, 0])
        assert (U[0, 0] > 0).all() and (p > 0).all()
    print("Lax L1 density errors at N = 100, 200, 400:", errs)
    assert errs[1] < 1e-2
    assert errs[0] > errs[1] > errs[2]
    assert errs[0] / errs[2] > 2.0


def test_troubled_cells_are_few_and_sit_on_the_waves():
    n = 200
    U, k, nt, nh, last = lax_run(n)
    frac = nt.sum() / (3 * k * n)
    print(f"Lax N={n}: {k} steps, troubled share {frac:.4f}, hybrid share {nh.sum() / (3 * k * n):.4f}")
    assert 0.0 < frac < 0.15
    # every troubled cell of the last step lies within 6 cells of a wave of the exact
    # solution (rarefaction head and tail, contact, shock)
    r = RiemannExact(*LAX, gamma=G)
    rl, ul, pl = LAX[0]
    cl = math.sqrt(G * pl / rl)
    cs = cl * (r.ps / pl) ** ((G - 1.0) / (2.0 * G))
    rr, ur, pr = LAX[1]
    cr = math.sqrt(G * pr / rr)
    S = ur + cr * math.sqrt((G + 1.0) / (2.0 * G) * r.ps / pr + (G - 1.0) / (2.0 * G))
    waves = np.array([ul - cl, r.us - cs, r.us, S]) * 0.16
    dx = 1.0 / n
    xc = -0.5 + (np.arange(n) + 0.5) * dx
    for st in range(3):
        cells = np.nonzero(last[st]["T"])[0]
        assert cells.size > 0
        dist = np.min(np.abs(xc[cells][:, None] - waves[None, :]), axis=1)
        assert (dist <= 6 * dx).all(), (st, xc[cells][dist > 6 * dx])


@pytest.mark.parametrize("name", ["shu_osher", "burgers_shock"])
def test_shock_tests_troubled_share(name):
    if name == "shu_osher":
        n, T = 400, 1.8
        o = Scheme1D("euler", n, -5.0, 5.0, bc="transmissive", tc_mode="kxrcf")
        U0 = hi.example_3_7(n)
    else:
        n, T = 80, 1.5 / math.pi
        o = Scheme1D("burgers", n, 0.0, 2.0, bc="periodic", tc_mode="kxrcf")
        U0 = hi.example_3_1(n)
    U, k, nt, nh, _ = run_with_flags(o, U0, T)
    frac = nt.sum() / (3 * k * n)
    print(f"{name} N={n}: {k} steps, troubled share {frac:.4f}")
    assert np.isfinite(U).all()
    assert 0.0 < frac < 0.1
    if name == "burgers_shock":
        # periodic: the mean is conserved through the shock
        assert abs(U[0, 0].mean() - U0[0, 0].mean()) < 1e-13


def mirror_extend(U):
    """The state on [-1, 1] whose right half is U on [0, 1] and whose left half is its
    mirror image with the velocity reversed (density and energy even, momentum odd; first
    moments pick up the opposite parity)."""
    n = U.shape[-1]
    M = np.concatenate([U[:, :, ::-1], U], axis=-1).copy()
    M[0, 1, :n] *= -1.0
    M[1, 0, :n] *= -1.0
    M[1, 2, :n] *= -1.0
    return M


def test_reflective_walls_equal_the_mirror_extended_periodic_problem():
    n = 200
    U = hi.example_3_8(n)
    r = Scheme1D("euler", n, 0.0, 1.0, bc="reflective", tc_mode="kxrcf")
    p = Scheme1D("euler", 2 * n, -1.0, 1.0, bc="periodic", tc_mode="kxrcf")
    dt = 0.5 * r.cfl_dt(U, 0.6)
    A, B = U, mirror_extend(U)
    for k in range(40):
        A, ia = r.rk3_step(A, dt)
        B, ib = p.rk3_step(B, dt)
        assert np.abs(A - B[:, :, n:]).max() <= 1e-13 * np.abs(A).max(), k
        for st in range(3):
            Tr, Tp = ia[st]["T"], ib[st]["T"]
            assert np.array_equal(Tr, Tp[n:]) and np.array_equal(Tr[::-1], Tp[:n]), (k, st)
    assert sum(int(i["T"].sum()) for i in ia) > 0


def test_blast_waves_troubled_share():
    n, T = 800, 0.038
    o = Scheme1D("euler", n, 0.0, 1.0, bc="reflective", tc_mode="kxrcf")
    U, k, nt, _, _ = run_with_flags(o, hi.example_3_8(n), T)
    frac = nt.sum() / (3 * k * n)
    rho = U[0, 0]
    p = (G - 1.0) * (U[0, 2] - 0.5 * U[0, 1] ** 2 / rho)
    print(f"blast N={n}: {k} steps, troubled share {frac:.4f}, density {rho.min():.4f}..{rho.max():.4f}")
    assert np.isfinite(U).all() and (rho > 0).all() and (p > 0).all()
    assert 0.0 < frac < 0.15
    # walls: no mass crosses them, so the total mass is that of the initial state
    assert abs(rho.sum() - hi.example_3_8(n)[0, 0].sum()) <= 1e-12 * rho.sum()
