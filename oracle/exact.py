"""Exact rational derivation of the reconstruction operators (oracle; test infrastructure).

Every operator of the scheme is a linear map from the stencil's moments to polynomial
coefficients, fixed by moment conditions the paper states.  This module writes those
conditions down in reference coordinates and solves them exactly with ``fractions``:

* reference coordinate of cell I_i: xi = (x - x_i)/dx in [-1/2, 1/2]; the neighbour
  I_{i+j} occupies [j - 1/2, j + 1/2].  The zeroth moment of a polynomial P over I_{i+j}
  is the integral of P over that interval, the first moment the integral of
  P*(xi - j) (Section 2.1, definitions below eq. odeH).
* 2D: (xi, eta) in [-1/2, 1/2]^2, cells labelled 1..9 as in Figure 1 (label 5 is the
  target cell, 1 the lower-left, 9 the upper-right).

1D operators (Section 2.1):
  limiter_ops_1d()    Step 1: quartic p0 (averages of I_{i-1..i+1}, first moments of
                      I_{i-1}, I_{i+1}) and linear p1, p2 (two averages each).
  recon_ops_1d()      Step 2.1: quintic p0 (averages and first moments of I_{i-1..i+1})
                      and quadratics p1, p2 (two averages plus the first moment of I_i).
2D operators (Section 2.2, Step 5.1):
  recon_ops_2d()      quartic p0 (all nine averages and the first moments of I_5 exactly,
                      the first moments of I_2, I_4, I_6, I_8 in the least-squares sense)
                      and quadratics p1..p4 on the four 2x2 sub-stencils of Figure 2.

Smoothness indicators (eqs. GHYZ and 2dGHYZ) are quadratic forms c^T G c in the
polynomial coefficients c; gram_1d / gram_2d give G exactly.

Pins (tests/test_oracle_exact.py): the derived 1D operators equal the rationals the paper
prints in Steps 1, 2.1, 2.2, 2.3 (golden fixture); every operator reproduces polynomial
data of its degree exactly; the least-squares quartic is unique and exact for total
degree <= 4.
"""
from fractions import Fraction as Q
from functools import lru_cache
import math

# --------------------------------------------------------------------------------------
# exact linear algebra


def solve_exact(A, B):
    """Solve A X = B exactly (Gauss-Jordan over the rationals).

    A: n x n list of lists, B: n x k list of lists.  Raises if A is singular.
    """
    n = len(A)
    k = len(B[0])
    M = [[Q(x) for x in A[r]] + [Q(x) for x in B[r]] for r in range(n)]
    for col in range(n):
        piv = None
        for r in range(col, n):
            if M[r][col] != 0:
                piv = r
                break
        if piv is None:
            raise ZeroDivisionError("singular system")
        M[col], M[piv] = M[piv], M[col]
        p = M[col][col]
        M[col] = [x / p for x in M[col]]
        for r in range(n):
            if r != col and M[r][col] != 0:
                f = M[r][col]
                M[r] = [a - f * b for a, b in zip(M[r], M[col])]
    return [row[n:n + k] for row in M]


def matmul_exact(A, B):
    return [[sum((A[i][t] * B[t][j] for t in range(len(B))), Q(0)) for j in range(len(B[0]))]
            for i in range(len(A))]


def transpose(A):
    return [list(r) for r in zip(*A)]


def rank_exact(A):
    M = [[Q(x) for x in row] for row in A]
    rows, cols = len(M), len(M[0])
    r = 0
    for c in range(cols):
        piv = None
        for i in range(r, rows):
            if M[i][c] != 0:
                piv = i
                break
        if piv is None:
            continue
        M[r], M[piv] = M[piv], M[r]
        for i in range(rows):
            if i != r and M[i][c] != 0:
                f = M[i][c] / M[r][c]
                M[i] = [a - f * b for a, b in zip(M[i], M[r])]
        r += 1
        if r == rows:
            break
    return r


# --------------------------------------------------------------------------------------
# monomial integrals


def int_mono(m, a, b):
    """Integral of xi^m over [a, b], exactly."""
    a, b = Q(a), Q(b)
    return (b ** (m + 1) - a ** (m + 1)) / (m + 1)


def cell_mom0(m, j):
    """Zeroth moment of xi^m over the reference cell centred at j."""
    return int_mono(m, Q(2 * j - 1, 2), Q(2 * j + 1, 2))


def cell_mom1(m, j):
    """First moment of xi^m over the cell centred at j: integral of xi^m (xi - j)."""
    a, b = Q(2 * j - 1, 2), Q(2 * j + 1, 2)
    return int_mono(m + 1, a, b) - j * int_mono(m, a, b)


def dpow(m, alpha):
    """Coefficient and exponent of d^alpha/dxi^alpha xi^m."""
    if alpha > m:
        return Q(0), 0
    c = 1
    for t in range(alpha):
        c *= (m - t)
    return Q(c), m - alpha


# --------------------------------------------------------------------------------------
# 1D: data vector d = (u_{-1}, u_0, u_{+1}, v_{-1}, v_0, v_{+1})

D1_NAMES = ("u_m1", "u_0", "u_p1", "v_m1", "v_0", "v_p1")
D1_OFFSET = {"u": {-1: 0, 0: 1, 1: 2}, "v": {-1: 3, 0: 4, 1: 5}}


def _poly_1d(deg, conditions):
    """Coefficient map (deg+1) x 6 of the polynomial of degree deg fixed by the given
    conditions, each a pair (kind, j): kind 'u' = zeroth moment over cell j equals the
    stencil average u_j; kind 'v' = first moment over cell j equals v_j."""
    assert len(conditions) == deg + 1
    A, B = [], []
    for kind, j in conditions:
        row = [cell_mom0(m, j) if kind == "u" else cell_mom1(m, j) for m in range(deg + 1)]
        rhs = [Q(0)] * 6
        rhs[D1_OFFSET[kind][j]] = Q(1)
        A.append(row)
        B.append(rhs)
    return solve_exact(A, B)


@lru_cache(None)
def limiter_ops_1d():
    """Step 1 polynomials: returns (C0, C1, C2), coefficient maps of the quartic p0 on S0
    and the linear p1 on S1 = {I_{i-1}, I_i}, p2 on S2 = {I_i, I_{i+1}}."""
    C0 = _poly_1d(4, [("u", -1), ("u", 0), ("u", 1), ("v", -1), ("v", 1)])
    C1 = _poly_1d(1, [("u", -1), ("u", 0)])
    C2 = _poly_1d(1, [("u", 0), ("u", 1)])
    return C0, C1, C2


@lru_cache(None)
def recon_ops_1d():
    """Step 2.1 polynomials: (C0, C1, C2) for the quintic p0 on S0 and the quadratics
    p1 (averages of I_{i-1}, I_i and first moment of I_i) and p2 (I_i, I_{i+1}, I_i)."""
    C0 = _poly_1d(5, [("u", -1), ("u", 0), ("u", 1), ("v", -1), ("v", 0), ("v", 1)])
    C1 = _poly_1d(2, [("u", -1), ("u", 0), ("v", 0)])
    C2 = _poly_1d(2, [("u", 0), ("u", 1), ("v", 0)])
    return C0, C1, C2


def first_moment_row_1d(C):
    """Row (length 6) mapping stencil data to the first moment over I_i of the polynomial
    with coefficient map C (the q_n of Step 1)."""
    deg = len(C) - 1
    return [sum((cell_mom1(m, 0) * C[m][k] for m in range(deg + 1)), Q(0)) for k in range(6)]


def point_row_1d(C, xi):
    """Row mapping stencil data to the polynomial's value at the rational point xi."""
    xi = Q(xi)
    deg = len(C) - 1
    return [sum((xi ** m * C[m][k] for m in range(deg + 1)), Q(0)) for k in range(6)]


def point_row_1d_sqrt(C, a, b, s):
    """Value of the polynomial at xi = a + b*sqrt(s) (a, b rational), returned as the
    pair (rational part, sqrt(s) part) of each of the six row entries."""
    deg = len(C) - 1
    # powers of (a + b r) with r^2 = s, as (rational, r) pairs
    pw = [(Q(1), Q(0))]
    for _ in range(deg):
        x, y = pw[-1]
        pw.append((x * a + y * b * s, x * b + y * a))
    rat = [sum((pw[m][0] * C[m][k] for m in range(deg + 1)), Q(0)) for k in range(6)]
    irr = [sum((pw[m][1] * C[m][k] for m in range(deg + 1)), Q(0)) for k in range(6)]
    return rat, irr


@lru_cache(None)
def gram_1d(r):
    """G[m][n] = sum_{alpha=1..r} int_{-1/2}^{1/2} D^alpha xi^m D^alpha xi^n dxi,
    m, n = 0..r: smoothness indicator of eq. GHYZ in reference coordinates
    (the dx^{2 alpha - 1} factor makes the physical-coordinate form equal to this)."""
    G = [[Q(0)] * (r + 1) for _ in range(r + 1)]
    for m in range(r + 1):
        for n in range(r + 1):
            s = Q(0)
            for alpha in range(1, r + 1):
                cm, em = dpow(m, alpha)
                cn, en = dpow(n, alpha)
                if cm == 0 or cn == 0:
                    continue
                s += cm * cn * int_mono(em + en, Q(-1, 2), Q(1, 2))
            G[m][n] = s
    return G


def beta_form_1d(C):
    """Quadratic form (6x6) in the stencil data equal to the smoothness indicator of the
    polynomial with coefficient map C."""
    r = len(C) - 1
    G = gram_1d(r)
    return matmul_exact(transpose(C), matmul_exact(G, C))


# --------------------------------------------------------------------------------------
# 2D: data vector d of length 27 = (u_1..u_9, v_1..v_9, w_1..w_9), labels of Figure 1


def label_offset(k):
    """Offsets (a, b) of cell label k (1..9) of Figure 1 relative to I_{i,j}."""
    return ((k - 1) % 3) - 1, ((k - 1) // 3) - 1


def monomials_2d(r):
    """Exponent pairs (p, q) of the monomials xi^p eta^q with p + q <= r."""
    return [(p, t - p) for t in range(r + 1) for p in range(t, -1, -1)]


def _mom2d(kind, k, p, q):
    a, b = label_offset(k)
    if kind == "u":
        return cell_mom0(p, a) * cell_mom0(q, b)
    if kind == "v":
        return cell_mom1(p, a) * cell_mom0(q, b)
    return cell_mom0(p, a) * cell_mom1(q, b)


def _col27(kind, k):
    return {"u": 0, "v": 9, "w": 18}[kind] + (k - 1)


def _interp_2d(r, conditions):
    mons = monomials_2d(r)
    assert len(conditions) == len(mons)
    A, B = [], []
    for kind, k in conditions:
        A.append([_mom2d(kind, k, p, q) for (p, q) in mons])
        rhs = [Q(0)] * 27
        rhs[_col27(kind, k)] = Q(1)
        B.append(rhs)
    return solve_exact(A, B)


SUBSTENCILS_2D = {1: (1, 2, 4, 5), 2: (2, 3, 5, 6), 3: (4, 5, 7, 8), 4: (5, 6, 8, 9)}


@lru_cache(None)
def recon_ops_2d():
    """Step 5.1 polynomials: (C0, C1, C2, C3, C4).

    C0 (15 x 27): the quartic that matches the nine averages and the two first moments of
    I_5 exactly and the first moments of I_2, I_4, I_6, I_8 in the least-squares sense
    (unweighted, reference coordinates), computed from the KKT system
        [2 B^T B  E^T] [c     ]   [2 B^T d_B]
        [E        0  ] [lambda] = [d_E      ]
    with E the exact rows and B the least-squares rows.
    Cn (6 x 27, n = 1..4): the quadratic interpolating the four averages of S_n and the
    first moments of I_5.
    """
    mons = monomials_2d(4)
    nm = len(mons)
    exact_rows = [("u", k) for k in range(1, 10)] + [("v", 5), ("w", 5)]
    ls_rows = [("v", 2), ("w", 2), ("v", 4), ("w", 4), ("v", 6), ("w", 6), ("v", 8), ("w", 8)]
    E = [[_mom2d(kd, k, p, q) for (p, q) in mons] for kd, k in exact_rows]
    B = [[_mom2d(kd, k, p, q) for (p, q) in mons] for kd, k in ls_rows]
    BtB = matmul_exact(transpose(B), B)
    ne = len(E)
    K = [[Q(0)] * (nm + ne) for _ in range(nm + ne)]
    for i in range(nm):
        for j in range(nm):
            K[i][j] = 2 * BtB[i][j]
        for j in range(ne):
            K[i][nm + j] = E[j][i]
    for i in range(ne):
        for j in range(nm):
            K[nm + i][j] = E[i][j]
    R = [[Q(0)] * 27 for _ in range(nm + ne)]
    for i in range(nm):
        for t, (kd, k) in enumerate(ls_rows):
            R[i][_col27(kd, k)] += 2 * B[t][i]
    for i, (kd, k) in enumerate(exact_rows):
        R[nm + i][_col27(kd, k)] = Q(1)
    X = solve_exact(K, R)
    C0 = X[:nm]
    Cs = [C0]
    for n in (1, 2, 3, 4):
        conds = [("u", k) for k in SUBSTENCILS_2D[n]] + [("v", 5), ("w", 5)]
        Cs.append(_interp_2d(2, conds))
    return tuple(Cs)


@lru_cache(None)
def gram_2d_parts(r):
    """Exact per-multi-index Gram matrices of eq. 2dGHYZ in reference coordinates.

    Returns a dict {(l1, l2): G} with G[s][t] = integral over [-1/2,1/2]^2 of
    d^l(mono_s) d^l(mono_t), for every multi-index with 1 <= l1 + l2 <= r (each counted
    once).  With |I| = dx*dy the physical-coordinate term for (l1, l2) equals the
    reference one times (dy/dx)^(l1 - l2)."""
    mons = monomials_2d(r)
    out = {}
    for L in range(1, r + 1):
        for l1 in range(L, -1, -1):
            l2 = L - l1
            G = [[Q(0)] * len(mons) for _ in mons]
            for s, (p, q) in enumerate(mons):
                cp, ep = dpow(p, l1)
                cq, eq_ = dpow(q, l2)
                if cp == 0 or cq == 0:
                    continue
                for t, (p2, q2) in enumerate(mons):
                    cp2, ep2 = dpow(p2, l1)
                    cq2, eq2 = dpow(q2, l2)
                    if cp2 == 0 or cq2 == 0:
                        continue
                    G[s][t] = (cp * cq * cp2 * cq2 * int_mono(ep + ep2, Q(-1, 2), Q(1, 2))
                               * int_mono(eq_ + eq2, Q(-1, 2), Q(1, 2)))
            out[(l1, l2)] = G
    return out


def gram_2d(r, aspect=1.0):
    """Float Gram matrix of eq. 2dGHYZ for cells of aspect ratio dy/dx = aspect."""
    import numpy as np
    parts = gram_2d_parts(r)
    n = len(monomials_2d(r))
    G = np.zeros((n, n))
    for (l1, l2), Gl in parts.items():
        G += float(aspect) ** (l1 - l2) * np.array([[float(x) for x in row] for row in Gl])
    return G


def to_float(M):
    import numpy as np
    return np.array([[float(x) for x in row] for row in M])


def point_values_2d(C, pts):
    """Float matrix (len(pts) x 27) of the values of the polynomial with coefficient map C
    at the reference points pts (floats); the monomials are evaluated exactly on the
    rational value of each float coordinate and rounded once."""
    import numpy as np
    nm = len(C)
    r = {1: 0, 3: 1, 6: 2, 10: 3, 15: 4}[nm]
    mons = monomials_2d(r)
    out = np.zeros((len(pts), 27))
    for i, (x, y) in enumerate(pts):
        qx, qy = Q(x), Q(y)
        vals = [qx ** p * qy ** q for (p, q) in mons]
        for k in range(27):
            out[i, k] = float(sum((vals[s] * C[s][k] for s in range(nm)), Q(0)))
    return out


def point_values_1d(C, pts):
    """Float matrix (len(pts) x 6) of the values of a 1D polynomial map at float points."""
    import numpy as np
    out = np.zeros((len(pts), 6))
    for i, x in enumerate(pts):
        qx = Q(x)
        for k in range(6):
            out[i, k] = float(sum((qx ** m * C[m][k] for m in range(len(C))), Q(0)))
    return out


# quadrature rules used by the scheme (eq. odeH: 4-point Gauss-Lobatto; Section 2.2:
# 3-point Gauss; the 2-point Gauss rule is the edge rule of the reduced-order variant)
SQRT5 = math.sqrt(5.0)
SQRT15 = math.sqrt(15.0)
SQRT3 = math.sqrt(3.0)


def gauss_lobatto4():
    """Nodes and weights on [-1/2, 1/2] of the four-point Gauss-Lobatto rule of eq. odeH."""
    return [-0.5, -SQRT5 / 10.0, SQRT5 / 10.0, 0.5], [1.0 / 12, 5.0 / 12, 5.0 / 12, 1.0 / 12]


def gauss(ng):
    """Nodes and weights on [-1/2, 1/2] of the ng-point Gauss-Legendre rule (ng = 2, 3)."""
    if ng == 3:
        return [-SQRT15 / 10.0, 0.0, SQRT15 / 10.0], [5.0 / 18, 4.0 / 9, 5.0 / 18]
    if ng == 2:
        return [-SQRT3 / 6.0, SQRT3 / 6.0], [0.5, 0.5]
    raise ValueError("ng must be 2 or 3")
