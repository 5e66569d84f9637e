"""The one-dimensional hybrid HWENO scheme on a mesh of cells of different sizes (oracle;
test infrastructure).

Section 2.1 fixes each polynomial of the scheme by moment conditions on the cells of its
stencil (averages, and first moments of the cells whose moments it uses) and measures it
with the smoothness indicator of eq. GHYZ; the linear weights that combine the polynomials
are artificial positive numbers summing to one (the point of the paper, Introduction): they
do not depend on the geometry.  So on a mesh with cells of different sizes the scheme is
the same sequence of steps with the same definitions, only the polynomials change.  Here,
for every cell I_i and in its local coordinate xi = (x - x_i) / dx_i, the neighbours lie
at [-1/2 - a_i, -1/2] and [1/2, 1/2 + b_i], a_i = dx_{i-1}/dx_i, b_i = dx_{i+1}/dx_i, and

  average of p over a cell of centre c and width w (xi units)   (1/w) int p dxi
  first moment of p over it                                      (1/w) int p (xi - c)/w dxi

(the first moment of cell j in x, (1/dx_j) int u (x - x_j)/dx_j dx, is exactly this in xi).
Each polynomial's coefficient map follows from a linear solve per cell (numpy, float64):
the quartic of Step 1 (averages of the three cells, first moments of the two neighbours),
its linear q1, q2 (averages of two cells), the quintic p0 of Step 2 (averages and first
moments of the three cells), the quadratics p1, p2 (two averages and the cell's first
moment).  The smoothness indicators are eq. GHYZ on I_i, whose dx_i^(2l-1) factors turn it
into the same integral over [-1/2, 1/2] in xi for every cell.  The KXRCF indicator uses
h = dx_i / 2 of each cell, the right-hand sides of eq. odeH divide by dx_i, and the CFL
step uses the smallest cell.

Ghost cells: a periodic mesh wraps (so do the neighbour sizes); at a transmissive or
reflective boundary a ghost is the mirror image of the cell it faces, so it has that cell's
size.

Pins (tests/test_oracle_mesh1d.py): on equal cells the maps equal the uniform scheme's
(Scheme1D, itself pinned to the paper's printed formulas) and so does the operator;
polynomial data of the right degree are reproduced exactly on random meshes; mass is
conserved on periodic meshes; smooth advection converges at fifth order on a smoothly
stretched mesh.
"""
import numpy as np

from .scheme1d import NG, Scheme1D
from .weno import combine, nonlinear_weights

# data slots of the stencil vector d = (u_{-1}, u_0, u_{+1}, v_{-1}, v_0, v_{+1})
SLOT = {("u", -1): 0, ("u", 0): 1, ("u", 1): 2, ("v", -1): 3, ("v", 0): 4, ("v", 1): 5}


def _int_mono(m, lo, hi):
    return (hi ** (m + 1) - lo ** (m + 1)) / (m + 1)


def _condition_row(kind, c, w, deg):
    """Coefficients of xi^0..xi^deg in the average ('u') or first moment ('v') over the cell
    [c - w/2, c + w/2]; c and w are arrays over cells, the result is (k, deg + 1)."""
    lo, hi = c - 0.5 * w, c + 0.5 * w
    rows = []
    for m in range(deg + 1):
        if kind == "u":
            rows.append(_int_mono(m, lo, hi) / w)
        else:
            rows.append((_int_mono(m + 1, lo, hi) - c * _int_mono(m, lo, hi)) / (w * w))
    return np.stack(rows, axis=-1)


def coefficient_maps(a, b, deg, conditions):
    """(k, deg + 1, 6): the monomial coefficients of the polynomial of degree deg fixed by
    the conditions [(kind, j)] on cells j = -1, 0, 1 of widths a, 1, b, as linear maps of
    the stencil vector."""
    k = len(a)
    geom = {-1: (-0.5 - 0.5 * a, a), 0: (np.zeros(k), np.ones(k)), 1: (0.5 + 0.5 * b, b)}
    A = np.stack([_condition_row(kind, *geom[j], deg) for kind, j in conditions], axis=1)
    B = np.zeros((k, deg + 1, 6))
    for r, key in enumerate(conditions):
        B[:, r, SLOT[key]] = 1.0
    return np.linalg.solve(A, B)


def gram(r):
    """sum_{l=1..r} int_{-1/2}^{1/2} D^l xi^m D^l xi^n dxi (eq. GHYZ in xi)."""
    G = np.zeros((r + 1, r + 1))
    for m in range(r + 1):
        for n in range(r + 1):
            for l in range(1, r + 1):
                if l > m or l > n:
                    continue
                cm = np.prod(np.arange(m - l + 1, m + 1, dtype=float))
                cn = np.prod(np.arange(n - l + 1, n + 1, dtype=float))
                G[m, n] += cm * cn * _int_mono(m + n - 2 * l, -0.5, 0.5)
    return G


def point_rows(C, xi):
    """(k, 6): value at xi of the polynomials with coefficient maps C (k, deg + 1, 6)."""
    p = xi ** np.arange(C.shape[1])
    return np.einsum("m,kms->ks", p, C)


def first_moment_rows(C):
    """(k, 6): first moment over [-1/2, 1/2] of the polynomials with maps C."""
    mom = np.array([_int_mono(m + 1, -0.5, 0.5) for m in range(C.shape[1])])
    return np.einsum("m,kms->ks", mom, C)


def neighbour_ratios(dx, bc):
    """a_i = dx_{i-1}/dx_i and b_i = dx_{i+1}/dx_i with the ghost rule of bc."""
    if bc == "periodic":
        left, right = np.roll(dx, 1), np.roll(dx, -1)
    else:
        left = np.concatenate([dx[:1], dx[:-1]])
        right = np.concatenate([dx[1:], dx[-1:]])
    return left / dx, right / dx


class Scheme1DNU(Scheme1D):
    """Scheme1D on the mesh with face coordinates faces[0] < faces[1] < ... < faces[n]."""

    def __init__(self, eq, faces, bc="periodic", **kw):
        faces = np.asarray(faces, dtype=float)
        if faces.ndim != 1 or faces.size < 8 or not np.all(np.diff(faces) > 0.0):
            raise ValueError("faces must be at least 8 increasing coordinates")
        n = faces.size - 1
        super().__init__(eq, n, faces[0], faces[-1], bc=bc, **kw)
        self.faces = faces
        self.dxs = np.diff(faces)
        a, b = neighbour_ratios(self.dxs, bc)
        # cell of every padded position (ghosts: the wrapped or mirrored cell)
        p = np.arange(n + 2 * NG) - NG
        if bc == "periodic":
            self.cell_of = p % n
        else:
            self.cell_of = np.where(p < 0, -p - 1, np.where(p >= n, 2 * n - 1 - p, p))
        L0 = coefficient_maps(a, b, 4, [("u", -1), ("u", 0), ("u", 1), ("v", -1), ("v", 1)])
        L1 = coefficient_maps(a, b, 1, [("u", -1), ("u", 0)])
        L2 = coefficient_maps(a, b, 1, [("u", 0), ("u", 1)])
        R0 = coefficient_maps(a, b, 5, [("u", -1), ("u", 0), ("u", 1), ("v", -1), ("v", 0), ("v", 1)])
        R1 = coefficient_maps(a, b, 2, [("u", -1), ("u", 0), ("v", 0)])
        R2 = coefficient_maps(a, b, 2, [("u", 0), ("u", 1), ("v", 0)])
        self.nu_lim_C = [L0, L1, L2]
        self.nu_lim_q = [first_moment_rows(C) for C in (L0, L1, L2)]
        self.nu_rec_C = [R0, R1, R2]
        self.nu_face = [(point_rows(C, -0.5), point_rows(C, 0.5)) for C in (R0, R1, R2)]
        s5 = np.sqrt(5.0) / 10.0
        self.nu_int = (point_rows(R0, -s5), point_rows(R0, s5))
        self.nu_G = {r: gram(r) for r in (1, 2, 4, 5)}

    # ------------------------------------------------------------------ mesh hooks
    def _min_dx(self):
        return float(self.dxs.min())

    def _cell_dx(self, pos):
        return self.dxs[self.cell_of[pos]]

    def _linear_faces(self, d, pos):
        c = self.cell_of[pos]
        P0 = self.nu_face[0]
        return np.einsum("ks,sck->ck", P0[0][c], d), np.einsum("ks,sck->ck", P0[1][c], d)

    def _linear_interior(self, d, pos):
        c = self.cell_of[pos]
        return (np.einsum("ks,sck->ck", self.nu_int[0][c], d),
                np.einsum("ks,sck->ck", self.nu_int[1][c], d))

    def _beta(self, C, d):
        cf = np.einsum("kms,sk->mk", C, d)
        G = self.nu_G[C.shape[1] - 1]
        return np.einsum("ik,ij,jk->k", cf, G, cf)

    def _limit_scalar(self, d, pos=None):
        c = self.cell_of[pos]
        betas = [self._beta(C[c], d) for C in self.nu_lim_C]
        qs = [np.einsum("ks,sk->k", q[c], d) for q in self.nu_lim_q]
        w = nonlinear_weights(betas, self.lim_w, self.eps)
        return combine(w, self.lim_w, qs)

    def _hweno_scalar(self, d, pos=None):
        c = self.cell_of[pos]
        betas = [self._beta(C[c], d) for C in self.nu_rec_C]
        w = nonlinear_weights(betas, self.rec_w, self.eps)
        left = combine(w, self.rec_w, [np.einsum("ks,sk->k", F[0][c], d) for F in self.nu_face])
        right = combine(w, self.rec_w, [np.einsum("ks,sk->k", F[1][c], d) for F in self.nu_face])
        return left, right
