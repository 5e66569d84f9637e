"""Pins of the one-dimensional scheme on meshes of cells of different sizes
(oracle/mesh1d.py): the polynomials of Section 2.1 defined by their moment conditions on
cells of different sizes, the artificial linear weights unchanged."""
import math

import numpy as np
import pytest

import hweno_inputs as hi
from oracle import exact
from oracle.mesh1d import Scheme1DNU, coefficient_maps, first_moment_rows, gram, point_rows
from oracle.physics import Equation
from oracle.scheme1d import NG, Scheme1D


def test_equal_cells_give_the_uniform_maps():
    """On equal cells every coefficient map equals the exact rational one of the uniform
    scheme (itself pinned to the paper's printed formulas)."""
    one = np.ones(3)
    pairs = [
        (coefficient_maps(one, one, 4, [("u", -1), ("u", 0), ("u", 1), ("v", -1), ("v", 1)]), exact.limiter_ops_1d()[0]),
        (coefficient_maps(one, one, 1, [("u", -1), ("u", 0)]), exact.limiter_ops_1d()[1]),
        (coefficient_maps(one, one, 5, [("u", -1), ("u", 0), ("u", 1), ("v", -1), ("v", 0), ("v", 1)]), exact.recon_ops_1d()[0]),
        (coefficient_maps(one, one, 2, [("u", 0), ("u", 1), ("v", 0)]), exact.recon_ops_1d()[2]),
    ]
    for C, E in pairs:
        Ef = exact.to_float(E)
        assert np.abs(C[0] - Ef).max() <= 1e-12 * max(1.0, np.abs(Ef).max())
    for r in (1, 2, 4, 5):
        assert np.abs(gram(r) - exact.to_float(exact.gram_1d(r))).max() <= 1e-12 * np.abs(gram(r)).max()


@pytest.mark.parametrize("eq,bc", [("euler", "periodic"), ("euler", "transmissive"),
                                   ("burgers", "periodic"), ("euler", "reflective")])
@pytest.mark.parametrize("tc", ["kxrcf", "all"])
def test_equal_cells_give_the_uniform_operator(eq, bc, tc):
    n = 48
    if eq == "euler":
        U, _ = hi.euler_riemann_1d(seed=1, n=n)
    else:
        U, _ = hi.advection_1d(0, n)
        U[1] += 0.05 * np.random.default_rng(2).normal(size=U[1].shape)
    o = Scheme1D(eq, n, 0.0, 1.0, bc=bc, tc_mode=tc)
    q = Scheme1DNU(eq, np.linspace(0.0, 1.0, n + 1), bc=bc, tc_mode=tc)
    L, i = o.operator(U)
    Lq, iq = q.operator(U)
    assert np.array_equal(i["T"], iq["T"]) and i["T"].any()
    assert np.abs(L - Lq).max() <= 1e-13 * np.abs(L).max()


def _poly_moments(coef, faces):
    """Exact averages and first moments of the polynomial sum coef[m] x^m per cell."""
    P = np.polynomial.Polynomial(coef)
    I = P.integ()
    a, b = faces[:-1], faces[1:]
    dx, c = b - a, 0.5 * (a + b)
    avg = (I(b) - I(a)) / dx
    xP = np.polynomial.Polynomial([0.0, 1.0]) * P
    J = xP.integ()
    mom = ((J(b) - J(a)) - c * (I(b) - I(a))) / (dx * dx)
    return avg, mom, P


@pytest.mark.parametrize("seed", [0, 1])
def test_polynomial_data_are_reproduced_on_random_meshes(seed):
    """Degree-5 data: the quintic p0 of Step 2 returns the exact point values at the faces
    and at the interior Gauss-Lobatto points; degree-4 data: the quartic of Step 1 returns
    the cell's own first moment; degree 2 / 1: p1, p2 / q1, q2 are exact."""
    n = 16
    faces = hi.random_faces(seed, n, -1.0, 1.5, ratio=3.0)
    rng = np.random.default_rng(10 + seed)
    q = Scheme1DNU("advection", faces, bc="transmissive")
    inner = np.arange(NG + 1, NG + n - 1)          # padded positions with mesh stencils
    cells = inner - NG
    dx = np.diff(faces)
    for deg, checks in ((5, "p0"), (4, "q0"), (2, "p12"), (1, "q12")):
        avg, mom, P = _poly_moments(rng.normal(size=deg + 1), faces)
        d = np.stack([avg[cells - 1], avg[cells], avg[cells + 1],
                      mom[cells - 1], mom[cells], mom[cells + 1]])     # (6, k)
        c = q.cell_of[inner]
        xc = 0.5 * (faces[cells] + faces[cells + 1])
        scale = np.abs(P(np.linspace(faces[0], faces[-1], 50))).max()
        if checks == "p0":
            for xi, rows in ((-0.5, q.nu_face[0][0]), (0.5, q.nu_face[0][1]),
                             (-math.sqrt(5) / 10, q.nu_int[0]), (math.sqrt(5) / 10, q.nu_int[1])):
                got = np.einsum("ks,sk->k", rows[c], d)
                assert np.abs(got - P(xc + xi * dx[cells])).max() <= 1e-12 * scale
        elif checks == "q0":
            got = np.einsum("ks,sk->k", q.nu_lim_q[0][c], d)
            assert np.abs(got - mom[cells]).max() <= 1e-12 * scale
        elif checks == "p12":
            for F in q.nu_face[1:]:
                for side, xi in ((0, -0.5), (1, 0.5)):
                    got = np.einsum("ks,sk->k", F[side][c], d)
                    assert np.abs(got - P(xc + xi * dx[cells])).max() <= 1e-12 * scale
        else:
            for qq in q.nu_lim_q[1:]:
                got = np.einsum("ks,sk->k", qq[c], d)
                assert np.abs(got - mom[cells]).max() <= 1e-12 * scale


def test_mass_is_conserved_on_a_periodic_random_mesh():
    n = 60
    faces = hi.random_faces(3, n, 0.0, 1.0, ratio=2.5)
    prm = hi.euler_riemann_params(np.random.default_rng(2003))
    U = hi.project_1d_faces(hi.euler_riemann_func(*prm), faces)
    q = Scheme1DNU("euler", faces, bc="periodic", tc_mode="kxrcf")
    dx = np.diff(faces)
    m0 = (U[0] * dx).sum(axis=1)
    X = U
    flagged = 0
    for _ in range(20):
        X, infos = q.rk3_step(X, q.cfl_dt(X, 0.6))
        flagged += sum(int(i["T"].sum()) for i in infos)
    assert flagged > 0
    m = (X[0] * dx).sum(axis=1)
    assert np.abs(m - m0).max() <= 1e-13 * np.abs(m0).max()


def test_fifth_order_on_a_stretched_mesh():
    """Smooth advection on [0, 2] over one period on x = s + 0.3 sin(2 pi s)/(2 pi): cell
    sizes vary by 1.86 across the mesh; L1 and Linf orders of the averages >= 4.7, with the
    time step shrinking like dx^(5/3) so that time errors stay below space errors."""
    ns = (40, 80, 160)
    _, prm = hi.advection_1d(0, 8)
    errs = []
    for n in ns:
        faces = hi.stretched_faces(n, 0.0, 2.0, amp=0.3)
        U0 = hi.project_1d_faces(prm["func"], faces)
        q = Scheme1DNU(Equation("advection", 1, adv=(1.0,)), faces, bc="periodic", tc_mode="none")
        h = q._min_dx()
        h0 = (2.0 / ns[0]) * 0.7
        dt = 0.5 * h * (h / h0) ** (2.0 / 3.0)
        U, t, k, _ = q.run(U0, T=2.0, dt=dt)
        e = np.abs(U[0, 0] - U0[0, 0])
        errs.append((e.mean(), e.max()))
    o = [(math.log(errs[i][0] / errs[i + 1][0]) / math.log(2.0),
          math.log(errs[i][1] / errs[i + 1][1]) / math.log(2.0)) for i in range(len(ns) - 1)]
    assert o[-1][0] >= 4.7 and o[-1][1] >= 4.7, (errs, o)
