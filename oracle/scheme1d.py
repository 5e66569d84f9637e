"""One-dimensional hybrid HWENO scheme (oracle; test infrastructure).

Implements, in the paper's order, one evaluation of the semi-discrete operator of
eq. odeH and the TVD-RK3 update of eq. RK (Section 2.1, Steps 1-3):

  0. ghost cells: periodic wrap, or at a transmissive boundary the even mirror (average
     copied, first moment negated: the P1 trace is continuous across the boundary); a
     reflective wall (Euler) also reverses the velocity (momentum average negated, its
     first moment kept)
  1. Lax-Friedrichs speed alpha = max over cells of |f'(ubar)| (Euler: |u| + c) at the
     cell averages of the stage input (global Lax-Friedrichs)
  2. troubled cells T (KXRCF on the unmodified stage input; tc_mode 'none' -> none,
     'all' -> every cell, the "New HWENO" variant of Section 3)
  3. Step 1: the first moment of every troubled cell is replaced by the HWENO limiter
     value computed from unmodified neighbours (q_n, beta_n, tau, omega_n); for Euler in
     the characteristic fields of the cell's average state (Remark 2).  The modified
     moments are the stage's limited state; rk3_step combines those (not the stored
     moments) in the Runge-Kutta stages.
  4. Step 2: H_i = T_{i-1} or T_i or T_{i+1}.  Interface values u^+_{i-1/2}, u^-_{i+1/2}:
     HWENO (Step 2.1, characteristic-wise for Euler, one set of weights per cell used at
     both faces) when H_i, else the quintic p0 (Step 2.2).  Interior Gauss-Lobatto
     values u_{i -/+ sqrt5/10} always from p0 (Step 2.3).  All use the modified moments.
  5. Lax-Friedrichs fluxes and the four-point Gauss-Lobatto volume term F_i built from
     the cell's own interface values and interior values.
  6. right-hand sides of eq. odeH.

Ghost cells at a transmissive or reflective boundary are mirror images of the cells
they copy in every respect, not only in their stored moments: a ghost's troubled flag is
the flag of the cell it mirrors, its limited moments are that cell's limited moments
under the same sign rule as the state, and its trace on the boundary face is the inner
cell's trace there (momentum reversed at a wall).  So the boundary face carries one
state on both sides and the Lax-Friedrichs flux there has no jump term at a transmissive
boundary.  The paper defines no boundary treatment for the moments; this reading is the
same in one and two dimensions (Scheme2D).

State layout: U has shape (2, ncomp, n): U[0] cell averages, U[1] first moments.
"""
import numpy as np

from . import exact
from .kxrcf import troubled_1d
from .physics import Equation
from .weno import nonlinear_weights, combine

NG = 3  # ghost layers: the operator at cell i reads cells i-3 .. i+3


class Scheme1D:
    def __init__(self, eq, n, x0=0.0, x1=1.0, bc="periodic", lim_w=(0.98, 0.01, 0.01),
                 rec_w=(0.98, 0.01, 0.01), eps=1e-6, tc_mode="kxrcf"):
        if isinstance(eq, str):
            eq = Equation(eq, 1)
        self.eq = eq
        self.n = int(n)
        self.x0, self.x1 = float(x0), float(x1)
        self.dx = (self.x1 - self.x0) / self.n
        self.bc = bc
        self.eps = float(eps)
        self.tc_mode = tc_mode
        self.set_linear_weights(lim_w, rec_w)
        # operators from the exact derivation, rounded once to float
        L0, L1, L2 = exact.limiter_ops_1d()
        self.lim_C = [exact.to_float(C) for C in (L0, L1, L2)]
        self.lim_q = [np.array([float(x) for x in exact.first_moment_row_1d(C)]) for C in (L0, L1, L2)]
        self.lim_G = [exact.to_float(exact.gram_1d(len(C) - 1)) for C in (L0, L1, L2)]
        R0, R1, R2 = exact.recon_ops_1d()
        self.rec_C = [exact.to_float(C) for C in (R0, R1, R2)]
        self.rec_G = [exact.to_float(exact.gram_1d(len(C) - 1)) for C in (R0, R1, R2)]
        # point values: faces xi = -1/2, +1/2 for every polynomial; p0 at -/+ sqrt5/10
        self.rec_face = [exact.point_values_1d(C, [-0.5, 0.5]) for C in (R0, R1, R2)]
        rat_m, irr_m = exact.point_row_1d_sqrt(R0, 0, exact.Q(-1, 10), 5)
        rat_p, irr_p = exact.point_row_1d_sqrt(R0, 0, exact.Q(1, 10), 5)
        self.int_rows = np.array([[float(a) + float(b) * exact.SQRT5 for a, b in zip(rat_m, irr_m)],
                                  [float(a) + float(b) * exact.SQRT5 for a, b in zip(rat_p, irr_p)]])

    def set_linear_weights(self, lim_w, rec_w):
        for w in (lim_w, rec_w):
            if len(w) != 3 or min(w) <= 0.0 or abs(sum(w) - 1.0) > 1e-14:
                raise ValueError("linear weights must be three positive numbers summing to one")
        self.lim_w = tuple(float(x) for x in lim_w)
        self.rec_w = tuple(float(x) for x in rec_w)

    # ------------------------------------------------------------------ ghost cells
    def pad(self, U):
        n = self.n
        Up = np.zeros(U.shape[:-1] + (n + 2 * NG,))
        Up[..., NG:NG + n] = U
        if self.bc == "periodic":
            Up[..., :NG] = U[..., n - NG:]
            Up[..., NG + n:] = U[..., :NG]
        elif self.bc == "transmissive":
            for g in range(1, NG + 1):
                Up[0, :, NG - g] = U[0, :, g - 1]
                Up[1, :, NG - g] = -U[1, :, g - 1]
                Up[0, :, NG + n - 1 + g] = U[0, :, n - g]
                Up[1, :, NG + n - 1 + g] = -U[1, :, n - g]
        elif self.bc == "reflective":
            # a wall: the mirror image with the normal velocity reversed, i.e. the
            # transmissive ghost with the momentum's average and first moment negated
            if self.eq.name != "euler":
                raise ValueError("reflective walls are defined for the Euler equations")
            for g in range(1, NG + 1):
                for gi, si in ((NG - g, g - 1), (NG + n - 1 + g, n - g)):
                    Up[0, :, gi] = U[0, :, si]
                    Up[1, :, gi] = -U[1, :, si]
                    Up[0, 1, gi] = -U[0, 1, si]
                    Up[1, 1, gi] = U[1, 1, si]
        else:
            raise ValueError(self.bc)
        return Up

    # ------------------------------------------------------------------ speeds
    def alpha(self, U):
        return float(np.max(self.eq.spectral_radius(U[0], 0)))

    def cfl_dt(self, U, cfl):
        return cfl * self._min_dx() / self.alpha(U)

    # ------------------------------------------------------------------ mesh hooks
    # (a uniform mesh here; oracle/mesh1d.py overrides them for cells of different sizes)
    def _min_dx(self):
        return self.dx

    def _cell_dx(self, pos):
        """Sizes of the cells at padded positions pos."""
        return self.dx

    def _linear_faces(self, d, pos):
        """Quintic p0 (Step 2.2) at the faces xi = -1/2, +1/2 of the cells at padded
        positions pos; d (6, ncomp, k) their stencil data."""
        P0 = self.rec_face[0]
        return np.einsum("s,sck->ck", P0[0], d), np.einsum("s,sck->ck", P0[1], d)

    def _linear_interior(self, d, pos):
        """p0 at the interior Gauss-Lobatto points xi = -/+ sqrt5/10 (Step 2.3)."""
        return np.einsum("s,sck->ck", self.int_rows[0], d), np.einsum("s,sck->ck", self.int_rows[1], d)

    # ------------------------------------------------------------------ Step 1
    def _troubled(self, Up):
        m = Up.shape[-1]
        T = np.zeros(m, dtype=bool)
        if self.tc_mode == "none":
            return T
        if self.tc_mode == "all":
            T[1:m - 1] = True
            return T
        ub, vb = Up[0], Up[1]
        vel = self.eq.velocity(Up[0][:, 1:m - 1], 0)
        comps = (0, 2) if self.eq.name == "euler" else (0,)
        t = np.zeros(m - 2, dtype=bool)
        for c in comps:
            t |= troubled_1d(ub[c, 1:m - 1], vb[c, 1:m - 1], ub[c, :m - 2], vb[c, :m - 2],
                             ub[c, 2:], vb[c, 2:], vel, self._cell_dx(np.arange(1, m - 1)))
        T[1:m - 1] = t
        return T

    def _limit_scalar(self, d, pos=None):
        """Step 1 for one field: d has shape (6, k) = stencil data of k cells (the first
        moment of the cell itself, d[4], is not used), pos their padded positions.
        Returns the modified moment."""
        cs = [C @ d for C in self.lim_C]
        betas = [np.einsum("ik,ij,jk->k", c, G, c) for c, G in zip(cs, self.lim_G)]
        qs = [q @ d for q in self.lim_q]
        w = nonlinear_weights(betas, self.lim_w, self.eps)
        return combine(w, self.lim_w, qs)

    def _stencil(self, ub, vb, idx):
        """Stencil data (6, ncomp, k) of the cells with padded indices idx."""
        return np.stack([ub[:, idx - 1], ub[:, idx], ub[:, idx + 1],
                         vb[:, idx - 1], vb[:, idx], vb[:, idx + 1]])

    def _limit(self, Up, T):
        Vt = Up[1].copy()
        idx = np.nonzero(T)[0]
        if idx.size == 0:
            return Vt
        d = self._stencil(Up[0], Up[1], idx)          # (6, ncomp, k)
        if self.eq.name != "euler":
            Vt[0, idx] = self._limit_scalar(d[:, 0, :], idx)
            return Vt
        Lm, Rm = self.eq.eigen_pair(Up[0][:, idx], 0)        # (k, ncomp, ncomp)
        dc = np.einsum("kab,sbk->sak", Lm, d)                # characteristic data
        nc = dc.shape[1]
        vc = self._limit_scalar(dc.reshape(6, -1), np.tile(idx, nc)).reshape(nc, -1)
        Vt[:, idx] = np.einsum("kab,bk->ak", Rm, vc)
        return Vt

    # ------------------------------------------------------------------ Step 2
    def _hweno_scalar(self, d, pos=None):
        """Step 2.1 for one field, d (6, k) of the cells at padded positions pos.
        Returns (u^+_{i-1/2}, u^-_{i+1/2})."""
        cs = [C @ d for C in self.rec_C]
        betas = [np.einsum("ik,ij,jk->k", c, G, c) for c, G in zip(cs, self.rec_G)]
        w = nonlinear_weights(betas, self.rec_w, self.eps)
        left = combine(w, self.rec_w, [P[0] @ d for P in self.rec_face])
        right = combine(w, self.rec_w, [P[1] @ d for P in self.rec_face])
        return left, right

    def _traces(self, Up, Vt, H, idx):
        """Interface values (left face, right face) of cells idx, shape (ncomp, k) each."""
        d = self._stencil(Up[0], Vt, idx)               # (6, ncomp, k)
        left, right = self._linear_faces(d, idx)
        hsel = np.nonzero(H[idx])[0]
        if hsel.size:
            if self.eq.name != "euler":
                l, r = self._hweno_scalar(d[:, 0, hsel], idx[hsel])
                left[0, hsel] = l
                right[0, hsel] = r
            else:
                cells = idx[hsel]
                Lm, Rm = self.eq.eigen_pair(Up[0][:, cells], 0)
                dc = np.einsum("kab,sbk->sak", Lm, d[:, :, hsel])
                nc = dc.shape[1]
                l, r = self._hweno_scalar(dc.reshape(6, -1), np.tile(cells, nc))
                left[:, hsel] = np.einsum("kab,bk->ak", Rm, l.reshape(nc, -1))
                right[:, hsel] = np.einsum("kab,bk->ak", Rm, r.reshape(nc, -1))
        return left, right

    # ------------------------------------------------------------------ mirror ghosts
    def _ghost_signs(self):
        """Signs (average, first moment) per component that a ghost cell's values pick up
        against the cell it mirrors: (1, -1) at a transmissive boundary; a reflective
        wall also negates the momentum component (average -1, first moment +1)."""
        nc = self.eq.ncomp
        sa = np.ones(nc)
        sm = -np.ones(nc)
        if self.bc == "reflective":
            sa[1] = -1.0
            sm[1] = 1.0
        return sa, sm

    def _mirror(self, A, sign=1.0):
        """Overwrites the ghost layers of a padded (..., m) array with the mirror images
        of the inner cells they face, times sign (only at a non-periodic boundary)."""
        if self.bc == "periodic":
            return A
        A = A.copy()
        n = self.n
        for g in range(1, NG + 1):
            A[..., NG - g] = sign * A[..., NG + g - 1]
            A[..., NG + n - 1 + g] = sign * A[..., NG + n - g]
        return A

    # ------------------------------------------------------------------ L(U)
    def operator_padded(self, Up, alpha, T=None, mirror=False):
        """L at the cells NG .. m-NG-1 of a padded state Up (m cells including ghosts),
        given the Lax-Friedrichs speed.  T (optional, length m) fixes the troubled flags.
        mirror: Up is pad() of a mesh state, and its transmissive / reflective ghost cells
        are the mirror images of the cells they copy in every respect (flags, limited
        moments, traces on the boundary face).
        Returns (L, T, H, Vt) on the padded grid (L on the inner cells only)."""
        m = Up.shape[-1]
        n = m - 2 * NG
        a = float(alpha)
        T = self._troubled(Up) if T is None else T.copy()
        if mirror:
            T = self._mirror(T.astype(float)) > 0.5
        # the outermost layer has a neighbour on one side only; its flag is never used
        T[0] = T[m - 1] = False
        Vt = self._limit(Up, T)
        sa, sm = self._ghost_signs()
        if mirror:
            Vt = self._mirror(Vt, sm)
        H = np.zeros(m, dtype=bool)
        H[1:m - 1] = T[:m - 2] | T[1:m - 1] | T[2:]
        # traces of cells NG-1 .. NG+n (inner cells plus one neighbour on each side)
        idx = np.arange(NG - 1, NG + n + 1)
        left, right = self._traces(Up, Vt, H, idx)
        if mirror and self.bc != "periodic":
            # the ghost's trace on the boundary face is the inner cell's trace there
            right[:, 0] = sa * left[:, 1]
            left[:, -1] = sa * right[:, -2]
        # interior Gauss-Lobatto points of the inner cells
        iidx = np.arange(NG, NG + n)
        d = self._stencil(Up[0], Vt, iidx)
        u_m, u_p = self._linear_interior(d, iidx)
        # fluxes at the n+1 faces of the inner cells: u^- = right trace of the left
        # cell, u^+ = left trace of the right cell
        um = right[:, :-1]
        up = left[:, 1:]
        f = self.eq.flux
        fhat = 0.5 * (f(um, 0) + f(up, 0)) - 0.5 * a * (up - um)
        fl, fr = fhat[:, :-1], fhat[:, 1:]
        own_l, own_r = left[:, 1:-1], right[:, 1:-1]
        Fi = (f(own_l, 0) + f(own_r, 0)) / 12.0 + 5.0 * (f(u_m, 0) + f(u_p, 0)) / 12.0
        dxi = self._cell_dx(iidx)
        L = np.empty((2,) + fl.shape)
        L[0] = -(fr - fl) / dxi
        L[1] = -(fl + fr) / (2.0 * dxi) + Fi / dxi
        return L, T, H, Vt

    def pad_flags(self, T):
        """Flags of the padded grid: the mesh's flags, wrapped (periodic) or mirrored
        (transmissive / reflective) into the ghost layers; the outermost layer is
        unflagged (operator_padded clears it as well)."""
        n = self.n
        Tp = np.zeros(n + 2 * NG, dtype=bool)
        Tp[NG:NG + n] = T
        if self.bc == "periodic":
            Tp[:NG] = T[n - NG:]
            Tp[NG + n:] = T[:NG]
        else:
            Tp = self._mirror(Tp.astype(float)) > 0.5
        Tp[0] = Tp[-1] = False
        return Tp

    def operator(self, U, alpha=None, T_fixed=None):
        """Semi-discrete right-hand side L(U) of eq. odeH.

        Returns (L, info) with L shape (2, ncomp, n) and info = dict(alpha, T, H, limited)
        where T and H are the troubled and hybrid flags of the n cells and ``limited`` is
        U with the Step-1 modified first moments."""
        n = self.n
        Up = self.pad(U)
        a = self.alpha(U) if alpha is None else float(alpha)
        Tp = None if T_fixed is None else self.pad_flags(np.asarray(T_fixed, dtype=bool))
        L, T, H, Vt = self.operator_padded(Up, a, Tp, mirror=True)
        lim = U.copy()
        lim[1] = Vt[:, NG:NG + n]
        info = dict(alpha=a, T=T[NG:NG + n].astype(np.uint8), H=H[NG:NG + n].astype(np.uint8),
                    limited=lim)
        return L, info

    # ------------------------------------------------------------------ eq. RK
    def rk3_step(self, U, dt):
        """One TVD-RK3 step; returns (U^{n+1}, [info of the three stages])."""
        L0, i0 = self.operator(U)
        W0 = i0["limited"]
        U1 = W0 + dt * L0
        L1, i1 = self.operator(U1)
        W1 = i1["limited"]
        U2 = 0.75 * W0 + 0.25 * W1 + 0.25 * dt * L1
        L2, i2 = self.operator(U2)
        W2 = i2["limited"]
        U3 = W0 / 3.0 + 2.0 / 3.0 * W2 + 2.0 / 3.0 * dt * L2
        return U3, [i0, i1, i2]

    def run(self, U, T=None, dt=None, cfl=0.6, nsteps=None, weights_fn=None):
        """Advance to time T (last step clipped) with dt = cfl dx / alpha per step, or
        nsteps steps of a fixed dt.  weights_fn(step) -> (lim_w, rec_w) resets the linear
        weights before each step (the random-weights test of Section 3.1).
        Returns (U, t, steps, infos_of_last_step)."""
        t = 0.0
        k = 0
        infos = None
        while True:
            if nsteps is not None and k >= nsteps:
                break
            if nsteps is None and t >= T:
                break
            if weights_fn is not None:
                self.set_linear_weights(*weights_fn(k))
            h = dt if dt is not None else self.cfl_dt(U, cfl)
            if T is not None and t + h > T:
                h = T - t
            U, infos = self.rk3_step(U, h)
            t += h
            k += 1
        return U, t, k, infos
