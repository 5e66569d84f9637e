"""Pins of the oracle's exact operator derivation (oracle/exact.py) against the paper's
printed one-dimensional rationals (Section 2.1, golden fixture), polynomial exactness,
quadrature exactness and the constrained least-squares conditions of Step 5.1."""
import itertools
import os
from fractions import Fraction as Q

import numpy as np
import pytest
import scipy.linalg

from oracle import exact

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_1d_operators.txt")


def load_golden():
    entries = {}
    cur = None
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("["):
                cur = line[1:line.index("]")]
                entries[cur] = {"row": None, "sqrt5": None, "square": []}
                continue
            key, val = line.split(":", 1)
            if key == "square":
                w, row = val.split("|")
                entries[cur]["square"].append((Q(w.strip()), [Q(x) for x in row.split()]))
            else:
                entries[cur][key] = [Q(x) for x in val.split()]
    return entries


G = load_golden()


def quad_form_from_squares(squares):
    M = [[Q(0)] * 6 for _ in range(6)]
    for w, r in squares:
        for i in range(6):
            for j in range(6):
                M[i][j] += w * r[i] * r[j]
    return M


def test_golden_parses():
    assert len(G) == 17


def test_step1_first_moments():
    C0, C1, C2 = exact.limiter_ops_1d()
    assert exact.first_moment_row_1d(C0) == G["step1.q0"]["row"]
    assert exact.first_moment_row_1d(C1) == G["step1.q1"]["row"]
    assert exact.first_moment_row_1d(C2) == G["step1.q2"]["row"]


def test_step1_smoothness_indicators():
    C0, C1, C2 = exact.limiter_ops_1d()
    # the quartic's indicator on the data it uses (v_0 is not part of the stencil)
    B0 = exact.beta_form_1d(C0)
    assert B0 == quad_form_from_squares(G["step1.beta0_corrected"]["square"])
    # the form exactly as printed differs from the definition (misprint in the last square)
    assert B0 != quad_form_from_squares(G["step1.beta0_printed"]["square"])
    assert exact.beta_form_1d(C1) == quad_form_from_squares(G["step1.beta1"]["square"])
    assert exact.beta_form_1d(C2) == quad_form_from_squares(G["step1.beta2"]["square"])


def test_step1_misprint_is_only_the_last_square():
    printed = G["step1.beta0_printed"]["square"]
    corrected = G["step1.beta0_corrected"]["square"]
    assert printed[:4] == corrected[:4]
    assert printed[4][0] == corrected[4][0]


def test_step21_point_values_and_indicators():
    C0, C1, C2 = exact.recon_ops_1d()
    half = Q(1, 2)
    assert exact.point_row_1d(C0, half) == G["step21.p0_right"]["row"]
    assert exact.point_row_1d(C1, half) == G["step21.p1_right"]["row"]
    assert exact.point_row_1d(C2, half) == G["step21.p2_right"]["row"]
    assert exact.beta_form_1d(C0) == quad_form_from_squares(G["step21.beta0"]["square"])
    assert exact.beta_form_1d(C1) == quad_form_from_squares(G["step21.beta1"]["square"])
    assert exact.beta_form_1d(C2) == quad_form_from_squares(G["step21.beta2"]["square"])


def test_step22_linear_interface_values():
    C0, _, _ = exact.recon_ops_1d()
    assert exact.point_row_1d(C0, Q(-1, 2)) == G["step22.u_plus_left"]["row"]
    assert exact.point_row_1d(C0, Q(1, 2)) == G["step22.u_minus_right"]["row"]


def test_step23_interior_values():
    C0, _, _ = exact.recon_ops_1d()
    rat, irr = exact.point_row_1d_sqrt(C0, 0, Q(-1, 10), 5)
    assert rat == G["step23.u_minus_sqrt5"]["row"] and irr == G["step23.u_minus_sqrt5"]["sqrt5"]
    rat, irr = exact.point_row_1d_sqrt(C0, 0, Q(1, 10), 5)
    assert rat == G["step23.u_plus_sqrt5"]["row"] and irr == G["step23.u_plus_sqrt5"]["sqrt5"]


# ----------------------------------------------------------------------------- exactness


def moments_1d_of_poly(coef):
    """Exact (u_{-1}, u_0, u_1, v_{-1}, v_0, v_1) of the polynomial sum coef[m] xi^m."""
    d = []
    for j in (-1, 0, 1):
        d.append(sum(c * exact.cell_mom0(m, j) for m, c in enumerate(coef)))
    for j in (-1, 0, 1):
        d.append(sum(c * exact.cell_mom1(m, j) for m, c in enumerate(coef)))
    return d


def test_1d_operators_polynomial_exact():
    rng = np.random.default_rng(7)
    C0, C1, C2 = exact.recon_ops_1d()
    L0, L1, L2 = exact.limiter_ops_1d()
    for deg in range(7):
        coef = [Q(int(x)) for x in rng.integers(-9, 10, deg + 1)]
        d = moments_1d_of_poly(coef)
        val = lambda row: sum(r * x for r, x in zip(row, d))
        p = lambda x: sum(c * x ** m for m, c in enumerate(coef))
        # quintic: exact interface values for degree <= 5
        ok = val(exact.point_row_1d(C0, Q(1, 2))) == p(Q(1, 2))
        assert ok == (deg <= 5)
        if deg <= 5:
            assert val(exact.point_row_1d(C0, Q(-1, 2))) == p(Q(-1, 2))
        # quartic limiter moment exact for degree <= 4
        if deg <= 4:
            assert val(exact.first_moment_row_1d(L0)) == d[4]
        if deg <= 2:
            assert val(exact.point_row_1d(C1, Q(1, 2))) == p(Q(1, 2))
            assert val(exact.point_row_1d(C2, Q(-1, 2))) == p(Q(-1, 2))
        if deg <= 1:
            assert val(exact.first_moment_row_1d(L1)) == d[4]
            assert val(exact.first_moment_row_1d(L2)) == d[4]
    # degree 5 data: the quartic's first moment is no longer exact
    coef = [Q(0)] * 5 + [Q(1)]
    d = moments_1d_of_poly(coef)
    assert sum(r * x for r, x in zip(exact.first_moment_row_1d(L0), d)) != d[4]


def moments_2d_of_poly(terms):
    """Exact 27-vector of the polynomial sum c xi^p eta^q (terms: {(p, q): c})."""
    d = [Q(0)] * 27
    for k in range(1, 10):
        a, b = exact.label_offset(k)
        for (p, q), c in terms.items():
            d[k - 1] += c * exact.cell_mom0(p, a) * exact.cell_mom0(q, b)
            d[9 + k - 1] += c * exact.cell_mom1(p, a) * exact.cell_mom0(q, b)
            d[18 + k - 1] += c * exact.cell_mom0(p, a) * exact.cell_mom1(q, b)
    return d


def eval_poly2(C, d, x, y):
    r = {1: 0, 3: 1, 6: 2, 10: 3, 15: 4}[len(C)]
    coef = [sum(C[s][k] * d[k] for k in range(27)) for s in range(len(C))]
    return sum(c * Q(x) ** p * Q(y) ** q for c, (p, q) in zip(coef, exact.monomials_2d(r)))


def test_2d_least_squares_quartic_exact_to_degree_4():
    Cs = exact.recon_ops_2d()
    pts = [(Q(1, 2), Q(1, 3)), (Q(-1, 2), Q(-1, 5)), (Q(1, 7), Q(1, 2)), (Q(0), Q(0))]
    for p in range(6):
        for q in range(6 - p):
            d = moments_2d_of_poly({(p, q): Q(1)})
            for x, y in pts:
                got = eval_poly2(Cs[0], d, x, y)
                want = Q(x) ** p * Q(y) ** q
                if p + q <= 4:
                    assert got == want
    # not exact for every degree-5 monomial
    bad = 0
    for p in range(6):
        d = moments_2d_of_poly({(p, 5 - p): Q(1)})
        bad += any(eval_poly2(Cs[0], d, x, y) != Q(x) ** p * Q(y) ** (5 - p) for x, y in pts)
    assert bad > 0


def _point_row(C, x, y):
    """Coefficients of the 27 data (u_1..u_9, v_1..v_9, w_1..w_9) in the value at (x, y)."""
    return [sum((C[s][k] * Q(x) ** p * Q(y) ** q for s, (p, q) in enumerate(exact.monomials_2d(4))),
                Q(0)) for k in range(27)]


def test_2d_least_squares_quartic_closed_form_values():
    """The Step 5.2 quartic (averages of the 3 x 3 block and the centre cell's moments
    exact, the edge neighbours' moments in least squares) at the cell centre and at the
    right edge midpoint, against closed forms derived independently of this code.  Labels
    1..9 run row by row from the bottom-left cell (Figure 1)."""
    C0 = exact.recon_ops_2d()[0]
    u = lambda k: k - 1
    v = lambda k: 9 + k - 1
    w = lambda k: 18 + k - 1
    centre = {u(5): Q(419, 288), u(2): Q(-133, 1152), u(4): Q(-133, 1152), u(6): Q(-133, 1152),
              u(8): Q(-133, 1152), u(1): Q(1, 576), u(3): Q(1, 576), u(7): Q(1, 576), u(9): Q(1, 576),
              v(6): Q(27, 64), v(4): Q(-27, 64), w(8): Q(27, 64), w(2): Q(-27, 64)}
    edge = {u(1): Q(1, 144), u(7): Q(1, 144), u(2): Q(-121, 1152), u(8): Q(-121, 1152),
            u(3): Q(-1, 72), u(9): Q(-1, 72), u(4): Q(17, 99), u(5): Q(457, 576), u(6): Q(205, 792),
            v(4): Q(3, 4), v(6): Q(-3, 4), v(5): Q(60, 11), w(8): Q(27, 64), w(2): Q(-27, 64)}
    for (x, y), want in [((0, 0), centre), ((Q(1, 2), 0), edge)]:
        got = _point_row(C0, x, y)
        assert got == [want.get(k, Q(0)) for k in range(27)], (x, y)
        assert sum(got[:9]) == 1


def test_2d_quadratics_exact_to_degree_2():
    Cs = exact.recon_ops_2d()
    for n in range(1, 5):
        for p in range(3):
            for q in range(3 - p):
                d = moments_2d_of_poly({(p, q): Q(1)})
                for x, y in [(Q(1, 2), Q(-1, 3)), (Q(-1, 2), Q(1, 2))]:
                    assert eval_poly2(Cs[n], d, x, y) == Q(x) ** p * Q(y) ** q


def test_2d_quadratics_use_only_their_substencil():
    Cs = exact.recon_ops_2d()
    for n, cells in exact.SUBSTENCILS_2D.items():
        used = {k for row in Cs[n] for k in range(27) if row[k] != 0}
        allowed = {c - 1 for c in cells} | {9 + 4, 18 + 4}
        assert used <= allowed


def test_2d_least_squares_conditions_brute_force():
    """p0 meets the exact rows, and no polynomial that also meets them has a smaller
    least-squares residual (first-order optimality checked against an independently
    computed null space of the exact rows)."""
    Cs = exact.recon_ops_2d()
    C0 = exact.to_float(Cs[0])
    mons = exact.monomials_2d(4)
    exact_rows = [("u", k) for k in range(1, 10)] + [("v", 5), ("w", 5)]
    ls_rows = [("v", k) for k in (2, 4, 6, 8)] + [("w", k) for k in (2, 4, 6, 8)]

    def row(kind, k):
        a, b = exact.label_offset(k)
        out = []
        for p, q in mons:
            if kind == "u":
                out.append(float(exact.cell_mom0(p, a) * exact.cell_mom0(q, b)))
            elif kind == "v":
                out.append(float(exact.cell_mom1(p, a) * exact.cell_mom0(q, b)))
            else:
                out.append(float(exact.cell_mom0(p, a) * exact.cell_mom1(q, b)))
        return out

    col = {"u": 0, "v": 9, "w": 18}
    E = np.array([row(*r) for r in exact_rows])
    B = np.array([row(*r) for r in ls_rows])
    assert np.linalg.matrix_rank(E) == 11
    N = scipy.linalg.null_space(E)
    assert N.shape[1] == 4
    rng = np.random.default_rng(3)
    for _ in range(5):
        d = rng.normal(size=27)
        c = C0 @ d
        dE = np.array([d[col[kd] + k - 1] for kd, k in exact_rows])
        dB = np.array([d[col[kd] + k - 1] for kd, k in ls_rows])
        assert np.allclose(E @ c, dE, atol=1e-12)
        grad = N.T @ (B.T @ (B @ c - dB))
        assert np.abs(grad).max() < 1e-11
        # any move inside the constraint set does not decrease the residual
        r0 = np.sum((B @ c - dB) ** 2)
        for _ in range(10):
            z = N @ rng.normal(size=4) * 1e-3
            assert np.sum((B @ (c + z) - dB) ** 2) >= r0 - 1e-15


# ----------------------------------------------------------------------------- quadrature


@pytest.mark.parametrize("rule,degree", [("gl4", 5), ("g3", 5), ("g2", 3)])
def test_quadrature_exactness(rule, degree):
    if rule == "gl4":
        x, w = exact.gauss_lobatto4()
    else:
        x, w = exact.gauss(3 if rule == "g3" else 2)
    for m in range(degree + 3):
        want = float(exact.int_mono(m, Q(-1, 2), Q(1, 2)))
        got = sum(wi * xi ** m for xi, wi in zip(x, w))
        if m <= degree:
            assert abs(got - want) < 1e-15
        elif m == degree + 1:
            assert abs(got - want) > 1e-6


# ----------------------------------------------------------------------------- smoothness


def test_gram_1d_hand_values():
    # beta of xi: int 1 = 1; beta of xi^2 with r = 2: int (2 xi)^2 + int 2^2 = 1/3 + 4
    G2 = exact.gram_1d(2)
    assert G2[1][1] == 1 and G2[2][2] == Q(13, 3) and G2[1][2] == 0
    assert G2[0][0] == 0


def test_gram_2d_hand_values():
    parts = exact.gram_2d_parts(2)
    mons = exact.monomials_2d(2)
    i_xy = mons.index((1, 1))
    i_x2 = mons.index((2, 0))
    # xi*eta: first derivatives (eta, xi) -> 1/12 + 1/12; second mixed derivative 1 -> 1
    tot = sum(G[i_xy][i_xy] for G in parts.values())
    assert tot == Q(1, 12) + Q(1, 12) + 1
    # xi^2: (2 xi)^2 -> 1/3, second derivative 2 -> 4
    tot = sum(G[i_x2][i_x2] for G in parts.values())
    assert tot == Q(1, 3) + 4
    assert len(parts) == 2 + 3   # (1,0),(0,1),(2,0),(1,1),(0,2): each multi-index once
