"""Two-dimensional hybrid HWENO scheme (oracle; test infrastructure).

Implements, in the paper's order, one evaluation of the semi-discrete operator of
eq. ode2 and the TVD-RK3 update (Section 2.2, Steps 4-6):

  0. ghost cells (3 layers): periodic wrap, or at transmissive and reflective boundaries
     the even mirror (averages copied, the first moment normal to the boundary negated,
     the tangential one copied); a reflective wall also reverses the normal momentum.
     Such ghosts are mirror images of the cells they face in every respect (flags,
     limited moments, edge values), as in Scheme1D.  The double Mach reflection and
     forward-step problems (Examples 3.10, 3.11) have boundary data of their own
     (oracle/dmr.py, oracle/step.py)
  1. global Lax-Friedrichs speeds alpha (x) and beta (y): max over cells of |f'(u)|,
     |g'(u)| (Euler: |mu| + c, |nu| + c) at the cell averages of the stage input
  2. troubled cells T by the KXRCF indicator on the unmodified stage input (Remark 3);
     tc_mode 'none' -> no cell, 'all' -> every cell ("New HWENO", Section 3)
  3. Step 4: in troubled cells, vbar is replaced by the one-dimensional limiter value of
     the x-line (averages of I_{i-1,j}, I_ij, I_{i+1,j}, x-moments of I_{i-1,j},
     I_{i+1,j}) and wbar by that of the y-line; for Euler in the characteristic fields of
     the x- resp. y-direction at the cell's average.  The modified moments replace the
     stored ones in the Runge-Kutta combination (see rk3_step).
  4. Step 5: H = T somewhere in the 3x3 block S0 (Figure 1).  Edge Gauss points: HWENO
     (Step 5.1) when H, else the least-squares quartic p0 (Step 5.2); interior 3x3 Gauss
     points always p0 (Step 5.3).  HWENO weights: one set per cell (and for Euler per
     characteristic field and per direction: x-edge points use the x-direction fields,
     y-edge points the y-direction fields).
  5. Lax-Friedrichs fluxes at the edge Gauss points and the right-hand sides of eq. ode2
     with the edge rule of ng points (3 in the paper; 2 in the reduced variant) and the
     3x3 Gauss volume rule.

State layout: U has shape (3, ncomp, ny, nx): U[0] averages, U[1] x-moments (vbar),
U[2] y-moments (wbar); x is the fastest axis.
"""
import numpy as np

from . import dmr, exact, step
from .kxrcf import troubled_2d
from .physics import Equation
from .weno import nonlinear_weights, combine

NG = 3


class Scheme2D:
    def __init__(self, eq, nx, ny, x0=0.0, x1=1.0, y0=0.0, y1=1.0, bc=("periodic", "periodic"),
                 ng_edge=3, lim_w=(0.98, 0.01, 0.01), rec_w=(0.96, 0.01, 0.01, 0.01, 0.01),
                 eps=1e-6, tc_mode="kxrcf", step_corner=step.STEP, inflow=step.INFLOW):
        if isinstance(eq, str):
            eq = Equation(eq, 2)
        self.eq = eq
        self.nx, self.ny = int(nx), int(ny)
        self.x0, self.x1, self.y0, self.y1 = map(float, (x0, x1, y0, y1))
        self.dx = (self.x1 - self.x0) / self.nx
        self.dy = (self.y1 - self.y0) / self.ny
        if isinstance(bc, str):
            bc = (bc, bc)
        self.bc = tuple(bc)
        for b in self.bc:
            if b not in ("periodic", "transmissive", "reflective", "dmr", "step"):
                raise ValueError(b)
        if ("reflective" in self.bc or "dmr" in self.bc or "step" in self.bc) and eq.name != "euler":
            raise ValueError("reflective walls are defined for the Euler equations")
        self.dmr = "dmr" in self.bc
        if self.dmr and (self.bc != ("dmr", "dmr") or abs(self.dx - self.dy) > 1e-12 * self.dx):
            raise ValueError("the double Mach reflection boundaries apply to all four sides of a square-cell mesh")
        self.step = "step" in self.bc
        if self.step:
            if self.bc != ("step", "step") or abs(self.dx - self.dy) > 1e-12 * self.dx:
                raise ValueError("the forward-step boundaries apply to all four sides of a square-cell mesh")
            si, sj = step.corner_cells(self.x0, self.y0, self.dx, self.dy, step_corner)
            if not (3 <= sj and 2 * sj <= self.ny and sj <= si <= self.nx - 1):
                raise ValueError("step corner outside 3 <= sj, 2 sj <= ny, sj <= si < nx")
            self.step_ij = (si, sj)
            self.u_in = step.conserved(inflow, eq.gamma)
            jj, ii = np.meshgrid(np.arange(self.ny), np.arange(self.nx), indexing="ij")
            self.solid = (ii >= si) & (jj < sj)
            self._step_map = self._step_sources()
        self.ng = int(ng_edge)
        self.eps = float(eps)
        self.tc_mode = tc_mode
        self.set_linear_weights(lim_w, rec_w)
        # Step 4 (dimension by dimension): the 1D Step-1 operators
        L0, L1, L2 = exact.limiter_ops_1d()
        self.lim_C = [exact.to_float(C) for C in (L0, L1, L2)]
        self.lim_q = [np.array([float(x) for x in exact.first_moment_row_1d(C)]) for C in (L0, L1, L2)]
        self.lim_G = [exact.to_float(exact.gram_1d(len(C) - 1)) for C in (L0, L1, L2)]
        # Step 5 polynomials
        Cs = exact.recon_ops_2d()
        self.rec_C = [exact.to_float(C) for C in Cs]
        aspect = self.dy / self.dx
        self.rec_G = [exact.gram_2d(4, aspect)] + [exact.gram_2d(2, aspect)] * 4
        gx, gw = exact.gauss(self.ng)
        self.edge_nodes, self.edge_w = np.array(gx), np.array(gw)
        vx, vw = exact.gauss(3)
        self.vol_nodes, self.vol_w = np.array(vx), np.array(vw)
        # point sets (reference coordinates)
        self.pts = {
            "L": [(-0.5, e) for e in gx], "R": [(0.5, e) for e in gx],
            "B": [(e, -0.5) for e in gx], "T": [(e, 0.5) for e in gx],
            "I": [(a, b) for b in vx for a in vx],      # row-major: eta outer, xi inner
        }
        self.P = {k: [exact.point_values_2d(C, v) for C in Cs] for k, v in self.pts.items()}

    def set_linear_weights(self, lim_w, rec_w):
        if len(lim_w) != 3 or min(lim_w) <= 0.0 or abs(sum(lim_w) - 1.0) > 1e-14:
            raise ValueError("limiter linear weights: three positive numbers summing to one")
        if len(rec_w) != 5 or min(rec_w) <= 0.0 or abs(sum(rec_w) - 1.0) > 1e-14:
            raise ValueError("reconstruction linear weights: five positive numbers summing to one")
        self.lim_w = tuple(float(x) for x in lim_w)
        self.rec_w = tuple(float(x) for x in rec_w)

    # ------------------------------------------------------------------ ghost cells
    def _wall_signs(self, ncomp):
        """Per-component factors (x, y) that a reflective wall adds on top of the mirror:
        the normal momentum (rho u at an x wall, rho v at a y wall) is reversed.  Ones for
        periodic and transmissive boundaries."""
        cx, cy = np.ones(ncomp), np.ones(ncomp)
        if ncomp == 4:
            if self.bc[0] == "reflective":
                cx[1] = -1.0
            if self.bc[1] == "reflective":
                cy[2] = -1.0
        return cx, cy

    def pad(self, U, t=0.0):
        """Three ghost layers: periodic wrap, or the even mirror (averages copied, the first
        moment normal to the boundary negated, the tangential one copied) at transmissive
        and reflective boundaries; a reflective wall also reverses the normal momentum
        (that component's average and moments negated on top of the mirror).  With the
        double Mach reflection boundaries, the ghost cells of time t (pad_dmr)."""
        if self.dmr:
            return self.pad_dmr(U, t)
        if self.step:
            return self.pad_step(U)
        nx, ny = self.nx, self.ny
        Up = np.zeros(U.shape[:2] + (ny + 2 * NG, nx + 2 * NG), dtype=U.dtype)
        Up[:, :, NG:NG + ny, NG:NG + nx] = U
        cx, cy = self._wall_signs(U.shape[1])
        # x direction (rows NG..NG+ny)
        rows = slice(NG, NG + ny)
        if self.bc[0] == "periodic":
            Up[:, :, rows, :NG] = U[:, :, :, nx - NG:]
            Up[:, :, rows, NG + nx:] = U[:, :, :, :NG]
        else:
            for g in range(1, NG + 1):
                Up[:, :, rows, NG - g] = U[:, :, :, g - 1] * cx[:, None]
                Up[:, :, rows, NG + nx - 1 + g] = U[:, :, :, nx - g] * cx[:, None]
                Up[1, :, rows, NG - g] *= -1.0
                Up[1, :, rows, NG + nx - 1 + g] *= -1.0
        # y direction (all columns, including the x ghosts: corners)
        if self.bc[1] == "periodic":
            Up[:, :, :NG, :] = Up[:, :, ny:ny + NG, :]
            Up[:, :, NG + ny:, :] = Up[:, :, NG:2 * NG, :]
        else:
            for g in range(1, NG + 1):
                Up[:, :, NG - g, :] = Up[:, :, NG + g - 1, :] * cy[:, None]
                Up[:, :, NG + ny - 1 + g, :] = Up[:, :, NG + ny - g, :] * cy[:, None]
                Up[2, :, NG - g, :] *= -1.0
                Up[2, :, NG + ny - 1 + g, :] *= -1.0
        return Up

    # ------------------------------------------------------------------ double Mach reflection
    # Example 3.10 on [x0, x1] x [y0, y1] (the paper's [0, 4] x [0, 1]): prescribed ghost
    # cells hold the exact solution's moments at the stage's time (left side; top side;
    # bottom side left of the wall's start x = 1/6), the bottom side from x = 1/6 on is a
    # reflective wall and the right side an outflow (transmissive) boundary, both mirrors
    # as above.  Reading for the prescribed ghosts (the paper does not define one): they
    # are never troubled, and their trace on the boundary face is the exact state at the
    # face's Gauss points.
    def _dmr_layout(self):
        nx, ny = self.nx, self.ny
        NY, NX = ny + 2 * NG, nx + 2 * NG
        xc = self.x0 + (np.arange(NX) - NG + 0.5) * self.dx
        yc = self.y0 + (np.arange(NY) - NG + 0.5) * self.dy
        pres = np.zeros((NY, NX), dtype=bool)
        pres[:, :NG] = True
        pres[NG + ny:, :] = True
        pres[:NG, xc < dmr.X_WALL] = True
        wall = xc >= dmr.X_WALL
        return xc, yc, pres, wall

    def _dmr_mirror(self, A, sx, sy):
        """Mirrored ghosts of the double Mach reflection boundaries: the outflow columns on
        the right (factor sx) and the wall rows at the bottom (factor sy); prescribed
        positions are left as they are."""
        A = A.copy()
        nx, ny = self.nx, self.ny
        rows = slice(NG, NG + ny)
        _, _, _, wall = self._dmr_layout()
        for g in range(1, NG + 1):
            A[..., rows, NG + nx - 1 + g] = sx * A[..., rows, NG + nx - g]
        for g in range(1, NG + 1):
            A[..., NG - g, wall] = sy * A[..., NG + g - 1, wall]
        return A

    def pad_dmr(self, U, t):
        nx, ny = self.nx, self.ny
        Up = np.zeros(U.shape[:2] + (ny + 2 * NG, nx + 2 * NG), dtype=U.dtype)
        Up[:, :, NG:NG + ny, NG:NG + nx] = U
        rows = slice(NG, NG + ny)
        # outflow (right side): the transmissive mirror
        for g in range(1, NG + 1):
            Up[:, :, rows, NG + nx - 1 + g] = U[:, :, :, nx - g]
            Up[1, :, rows, NG + nx - 1 + g] *= -1.0
        # wall (bottom side from x = 1/6, over every column): the mirror with the y moments
        # negated and the normal momentum rho v reversed
        xc, yc, pres, wall = self._dmr_layout()
        for g in range(1, NG + 1):
            Up[:, :, NG - g, wall] = Up[:, :, NG + g - 1, wall]
            Up[2, :, NG - g, wall] *= -1.0
            Up[:, 2, NG - g, wall] *= -1.0
        for j, i in zip(*np.nonzero(pres)):
            Up[:, :, j, i] = dmr.cell_moments(xc[i], yc[j], self.dx, t)
        return Up

    def _dmr_pad_flags(self, T):
        nx, ny = self.nx, self.ny
        Tp = np.zeros((ny + 2 * NG, nx + 2 * NG), dtype=bool)
        Tp[NG:NG + ny, NG:NG + nx] = T
        Tp = self._dmr_mirror(Tp.astype(float), 1.0, 1.0) > 0.5
        _, _, pres, _ = self._dmr_layout()
        Tp[pres] = False
        return Tp

    def _dmr_edge_values(self, vals, t):
        """Edge values of the ghost cells next to the mesh: mirror images at the outflow
        and wall sides, the exact state at the Gauss points of the prescribed sides."""
        vals = {k: v.copy() for k, v in vals.items()}
        nx, ny = self.nx, self.ny
        e = self.edge_nodes
        xs = self.x0 + (np.arange(nx) + 0.5) * self.dx               # mesh column centres
        ys = self.y0 + (np.arange(ny) + 0.5) * self.dy
        ex = lambda X, Y: np.moveaxis(dmr.state_at(X, Y, t), 0, 1)   # (ng, 4, n)
        # outflow (right): the inner cell's value on the boundary face
        vals["L"][..., 1:ny + 1, nx + 1] = vals["R"][..., 1:ny + 1, nx]
        # prescribed left side: exact state at (x0, y_j + e_k dy)
        Y = ys[None, :] + e[:, None] * self.dy
        vals["R"][..., 1:ny + 1, 0] = ex(np.full_like(Y, self.x0), Y)
        # top: exact state at (x_i + e_k dx, y1)
        X = xs[None, :] + e[:, None] * self.dx
        vals["B"][..., ny + 1, 1:nx + 1] = ex(X, np.full_like(X, self.y1))
        # bottom: wall (mirror, normal momentum reversed) from x = 1/6, exact state before
        cy = np.array([1.0, 1.0, -1.0, 1.0])[None, :, None]
        wall = xs >= dmr.X_WALL
        exact = ex(X, np.full_like(X, self.y0))
        bottom = np.where(wall[None, None, :], cy * vals["B"][..., 1, 1:nx + 1], exact)
        vals["T"][..., 0, 1:nx + 1] = bottom
        return vals

    # ------------------------------------------------------------------ forward step
    # Example 3.11 (oracle/step.py): solid cells inside the step, inflow on the left,
    # outflow on the right, walls at the top, the bottom and on the step's faces.  Ghost
    # and solid positions follow the position rule, traces on faces between the fluid and
    # anything else the face rule.
    def _step_sources(self):
        """Source map of the padded grid: for every position, the padded indices (J, I) of
        its source cell, the factors of the x and y moments and of rho u and rho v, and
        whether it is prescribed (inflow)."""
        nx, ny = self.nx, self.ny
        si, sj = self.step_ij
        NY, NX = ny + 2 * NG, nx + 2 * NG
        J = np.zeros((NY, NX), dtype=int)
        I = np.zeros((NY, NX), dtype=int)
        fac = np.ones((4, NY, NX))
        pres = np.zeros((NY, NX), dtype=bool)
        for jp in range(NY):
            for ip in range(NX):
                i, j, sx, sy, fu, fv, pr = step.source(ip - NG, jp - NG, nx, ny, si, sj)
                J[jp, ip], I[jp, ip] = j + NG, i + NG
                fac[:, jp, ip] = (sx, sy, fu, fv)
                pres[jp, ip] = pr
        return J, I, fac, pres

    def _step_factors(self, ncomp, kind):
        """Per (component, position) factors of a padded array of the given kind: 'avg'
        (averages), 'x' / 'y' (x / y first moments)."""
        _, _, fac, _ = self._step_map
        cf = np.ones((ncomp,) + fac.shape[1:])
        cf[1] = fac[2]
        cf[2] = fac[3]
        if kind == "x":
            cf = cf * fac[0]
        elif kind == "y":
            cf = cf * fac[1]
        return cf

    def _step_fill(self, A, kind):
        """A padded array (ncomp, NY, NX) with every position replaced by its source's
        value (times its factors); prescribed positions: the inflow state's average, zero
        first moments."""
        J, I, _, pres = self._step_map
        out = A[:, J, I] * self._step_factors(A.shape[0], kind)
        out[:, pres] = self.u_in[:, None] if kind == "avg" else 0.0
        return out

    def pad_step(self, U):
        nx, ny = self.nx, self.ny
        Up = np.zeros(U.shape[:2] + (ny + 2 * NG, nx + 2 * NG), dtype=U.dtype)
        Up[:, :, NG:NG + ny, NG:NG + nx] = U
        return np.stack([self._step_fill(Up[m], kind) for m, kind in enumerate(("avg", "x", "y"))])

    def _step_flags(self, T):
        """Padded flags with every position replaced by its source's flag (prescribed:
        never troubled)."""
        J, I, _, pres = self._step_map
        out = T[J, I].copy()
        out[pres] = False
        return out

    def _fluid2(self):
        """Fluid mask of the margin-2 region (mesh cells and one ghost layer)."""
        F = np.zeros((self.ny + 2, self.nx + 2), dtype=bool)
        F[1:-1, 1:-1] = ~self.solid
        return F

    def _step_edge_values(self, vals):
        """Face rule: on each face between a fluid cell and a non-fluid position, the
        non-fluid side takes the fluid cell's trace (normal momentum reversed at a wall,
        unchanged at the outflow), or the inflow state on the left side."""
        vals = {k: v.copy() for k, v in vals.items()}
        F = self._fluid2()
        ny2, nx2 = F.shape
        nc = vals["L"].shape[1]
        # x faces between positions (J, I) and (J, I + 1) of the margin-2 region
        for J, I in zip(*np.nonzero(F[:, :-1] & ~F[:, 1:])):
            c = np.ones(nc)
            if I + 1 < nx2 - 1:                      # solid: the step's left face
                c[1] = -1.0
            vals["L"][:, :, J, I + 1] = c[None, :] * vals["R"][:, :, J, I]
        for J, I in zip(*np.nonzero(~F[:, :-1] & F[:, 1:])):
            if I == 0:                               # inflow side
                vals["R"][:, :, J, I] = self.u_in[None, :]
            else:
                c = np.ones(nc)
                c[1] = -1.0
                vals["R"][:, :, J, I] = c[None, :] * vals["L"][:, :, J, I + 1]
        # y faces between (J, I) and (J + 1, I): walls on every side
        cy = np.ones(nc)
        cy[2] = -1.0
        for J, I in zip(*np.nonzero(F[:-1, :] & ~F[1:, :])):
            vals["B"][:, :, J + 1, I] = cy[None, :] * vals["T"][:, :, J, I]
        for J, I in zip(*np.nonzero(~F[:-1, :] & F[1:, :])):
            vals["T"][:, :, J, I] = cy[None, :] * vals["B"][:, :, J + 1, I]
        return vals

    def mirror_ghosts(self, A, sx=1.0, sy=1.0):
        """Overwrites the transmissive / reflective ghost layers of a padded (..., NY, NX)
        array with the mirror images of the interior cells, in the order of pad(); sx / sy
        is the factor a value picks up in an x / y mirror (a number, or per component an
        array of shape (ncomp, 1) for arrays with a leading component axis).  Such a ghost
        is the mirror image of the cell it copies in every respect: state, troubled flag,
        limited moments and edge values (the flags are not the ones KXRCF would give on
        the mirrored stencil, where the copied velocity points the other way relative to
        the neighbours)."""
        A = A.copy()
        nx, ny = self.nx, self.ny
        rows = slice(NG, NG + ny)
        if self.bc[0] != "periodic":
            for g in range(1, NG + 1):
                A[..., rows, NG - g] = sx * A[..., rows, NG + g - 1]
                A[..., rows, NG + nx - 1 + g] = sx * A[..., rows, NG + nx - g]
        if self.bc[1] != "periodic":
            for g in range(1, NG + 1):
                A[..., NG - g, :] = sy * A[..., NG + g - 1, :]
                A[..., NG + ny - 1 + g, :] = sy * A[..., NG + ny - g, :]
        return A

    def _mirror_edge_values(self, vals):
        """Edge values of the transmissive / reflective ghost cells next to the mesh (vals
        arrays cover the mesh plus one ghost layer): each is the mirror image of the cell
        it copies, so the ghost's value on the boundary face equals the inner cell's value
        there (normal momentum reversed at a wall)."""
        vals = {k: v.copy() for k, v in vals.items()}
        nx, ny = self.nx, self.ny
        cx, cy = self._wall_signs(vals["L"].shape[1])
        cx, cy = cx[:, None], cy[:, None]
        if self.bc[0] != "periodic":
            vals["R"][..., 1:ny + 1, 0] = cx * vals["L"][..., 1:ny + 1, 1]
            vals["L"][..., 1:ny + 1, nx + 1] = cx * vals["R"][..., 1:ny + 1, nx]
        if self.bc[1] != "periodic":
            vals["T"][..., 0, 1:nx + 1] = cy * vals["B"][..., 1, 1:nx + 1]
            vals["B"][..., ny + 1, 1:nx + 1] = cy * vals["T"][..., ny, 1:nx + 1]
        return vals

    # ------------------------------------------------------------------ speeds
    def alphas(self, U):
        ub = U[0]
        if self.step:
            ub = ub[:, ~self.solid]                   # solid cells hold no flow
        return (float(np.max(self.eq.spectral_radius(ub, 0))),
                float(np.max(self.eq.spectral_radius(ub, 1))))

    def cfl_dt(self, U, cfl):
        ax, ay = self.alphas(U)
        return cfl / (ax / self.dx + ay / self.dy)

    # ------------------------------------------------------------------ helpers
    @staticmethod
    def _sl(A, r, dj=0, di=0):
        NY, NX = A.shape[-2:]
        return A[..., r + dj:NY - r + dj, r + di:NX - r + di]

    # ------------------------------------------------------------------ Step 4
    def _troubled(self, Up):
        NY, NX = Up.shape[-2:]
        T = np.zeros((NY, NX), dtype=bool)
        if self.tc_mode == "none":
            return T
        if self.tc_mode == "all":
            T[1:-1, 1:-1] = True
            return T
        s = self._sl
        velx = self.eq.velocity(s(Up[0], 1), 0)
        vely = self.eq.velocity(s(Up[0], 1), 1)
        comps = (0, 3) if self.eq.name == "euler" else (0,)
        t = np.zeros((NY - 2, NX - 2), dtype=bool)
        for c in comps:
            cell = lambda dj, di: (s(Up[0, c], 1, dj, di), s(Up[1, c], 1, dj, di), s(Up[2, c], 1, dj, di))
            t |= troubled_2d(cell(0, 0), cell(0, -1), cell(0, 1), cell(-1, 0), cell(1, 0),
                             velx, vely, self.dx, self.dy)
        T[1:-1, 1:-1] = t
        return T

    def _limit_scalar(self, d):
        cs = [C @ d for C in self.lim_C]
        betas = [np.einsum("ik,ij,jk->k", c, G, c) for c, G in zip(cs, self.lim_G)]
        qs = [q @ d for q in self.lim_q]
        w = nonlinear_weights(betas, self.lim_w, self.eps)
        return combine(w, self.lim_w, qs)

    def _limit(self, Up, T):
        """Modified first moments (Vt, Wt) on the padded grid (Step 4, Jacobi)."""
        Vt = Up[1].copy()
        Wt = Up[2].copy()
        jj, ii = np.nonzero(T)
        if jj.size == 0:
            return Vt, Wt
        ub, vb, wb = Up[0], Up[1], Up[2]
        # 1D stencil vectors (6, ncomp, k): u_{-1}, u_0, u_{+1}, m_{-1}, m_0, m_{+1}
        dx_line = np.stack([ub[:, jj, ii - 1], ub[:, jj, ii], ub[:, jj, ii + 1],
                            vb[:, jj, ii - 1], vb[:, jj, ii], vb[:, jj, ii + 1]])
        dy_line = np.stack([ub[:, jj - 1, ii], ub[:, jj, ii], ub[:, jj + 1, ii],
                            wb[:, jj - 1, ii], wb[:, jj, ii], wb[:, jj + 1, ii]])
        if self.eq.name != "euler":
            Vt[0, jj, ii] = self._limit_scalar(dx_line[:, 0])
            Wt[0, jj, ii] = self._limit_scalar(dy_line[:, 0])
            return Vt, Wt
        for d, line, out in ((0, dx_line, Vt), (1, dy_line, Wt)):
            Lm, Rm = self.eq.eigen_pair(ub[:, jj, ii], d)
            dc = np.einsum("kab,sbk->sak", Lm, line)
            nc = dc.shape[1]
            mc = self._limit_scalar(dc.reshape(6, -1)).reshape(nc, -1)
            out[:, jj, ii] = np.einsum("kab,bk->ak", Rm, mc)
        return Vt, Wt

    # ------------------------------------------------------------------ Step 5
    def _stencil27(self, ub, vb, wb, r):
        """Stencil data (27, ncomp, ...) of every cell at margin r of the padded grid:
        (u_1..u_9, v_1..v_9, w_1..w_9) with the labels of Figure 1."""
        out = []
        for A in (ub, vb, wb):
            for k in range(1, 10):
                a, b = exact.label_offset(k)
                out.append(self._sl(A, r, b, a))
        return np.stack(out)

    def _hweno_scalar(self, d, keys):
        """HWENO values (Step 5.1) of one field, d (27, k), at the point sets keys.
        Returns {key: (npts, k)}."""
        cs = [C @ d for C in self.rec_C]
        betas = [np.einsum("ik,ij,jk->k", c, G, c) for c, G in zip(cs, self.rec_G)]
        w = nonlinear_weights(betas, self.rec_w, self.eps)
        return {key: combine(w, self.rec_w, [P @ d for P in self.P[key]]) for key in keys}

    def _edge_values(self, Up, Vt, Wt, H):
        """Values at the four edges' Gauss points for every cell at margin 2.

        Returns dict key -> array (ng, ncomp, ny+2, nx+2)."""
        D = self._stencil27(Up[0], Vt, Wt, 2)                     # (27, nc, ny+2, nx+2)
        vals = {k: np.einsum("ps,scyx->pcyx", self.P[k][0], D) for k in "LRBT"}
        Hm = self._sl(H, 2)
        jj, ii = np.nonzero(Hm)
        if jj.size == 0:
            return vals, D
        dH = D[:, :, jj, ii]                                      # (27, nc, k)
        if self.eq.name != "euler":
            res = self._hweno_scalar(dH[:, 0], "LRBT")
            for k in "LRBT":
                vals[k][:, 0, jj, ii] = res[k]
            return vals, D
        ubar = self._sl(Up[0], 2)[:, jj, ii]
        for d, keys in ((0, "LR"), (1, "BT")):
            Lm, Rm = self.eq.eigen_pair(ubar, d)
            dc = np.einsum("kab,sbk->sak", Lm, dH)                # (27, nc, k)
            nc = dc.shape[1]
            res = self._hweno_scalar(dc.reshape(27, -1), keys)
            for key in keys:
                v = res[key].reshape(self.ng, nc, -1)
                vals[key][:, :, jj, ii] = np.einsum("kab,pbk->pak", Rm, v)
        return vals, D

    # ------------------------------------------------------------------ L(U)
    def operator_padded(self, Up, ax, ay, T_fixed=None, ghosts=False, t=0.0):
        """L at every cell of margin 3 of the padded state Up, given the Lax-Friedrichs
        speeds.  Returns (L, info) with info = dict(T, H, Vt, Wt) on that region.
        ghosts: Up is pad() of a mesh state at time t; its transmissive and reflective
        ghost cells are mirror images of the cells they copy in every respect (flags,
        limited moments, edge values), prescribed ones (double Mach reflection) are
        never troubled and take the exact state on the boundary face."""
        if T_fixed is None:
            T = self._troubled(Up)
        else:
            T = T_fixed
        if ghosts and self.dmr:
            T = self._dmr_mirror(T.astype(float), 1.0, 1.0) > 0.5
            T[self._dmr_layout()[2]] = False
        elif ghosts and self.step:
            T = self._step_flags(T)
        elif ghosts:
            T = self.mirror_ghosts(T)
        if ghosts:
            # the outermost layer has no neighbours; its flags are never used
            T[0, :] = T[-1, :] = False
            T[:, 0] = T[:, -1] = False
        Vt, Wt = self._limit(Up, T)
        if ghosts and self.dmr:
            cy = np.array([1.0, 1.0, -1.0, 1.0])[:, None]
            Vt = self._dmr_mirror(Vt, -1.0, cy)
            Wt = self._dmr_mirror(Wt, 1.0, -cy)
        elif ghosts and self.step:
            Vt = self._step_fill(Vt, "x")
            Wt = self._step_fill(Wt, "y")
        elif ghosts:
            cx, cy = self._wall_signs(Vt.shape[0])
            Vt = self.mirror_ghosts(Vt, sx=-cx[:, None], sy=cy[:, None])
            Wt = self.mirror_ghosts(Wt, sx=cx[:, None], sy=-cy[:, None])
        NY, NX = T.shape
        H = np.zeros_like(T)
        acc = np.zeros((NY - 2, NX - 2), dtype=bool)
        for dj in (-1, 0, 1):
            for di in (-1, 0, 1):
                acc |= T[1 + dj:NY - 1 + dj, 1 + di:NX - 1 + di]
        H[1:-1, 1:-1] = acc
        vals, D = self._edge_values(Up, Vt, Wt, H)
        if ghosts and self.dmr:
            vals = self._dmr_edge_values(vals, t)
        elif ghosts and self.step:
            vals = self._step_edge_values(vals)
        elif ghosts:
            vals = self._mirror_edge_values(vals)
        # interior Gauss points of the cells at margin 3
        Dint = D[:, :, 1:-1, 1:-1]
        vint = np.einsum("ps,scyx->pcyx", self.P["I"][0], Dint)  # (9, nc, ny, nx)
        f = self.eq.flux
        # x faces: between cell column c and c+1 of the margin-2 region, interior rows
        um = vals["R"][:, :, 1:-1, :-1]
        up = vals["L"][:, :, 1:-1, 1:]
        Fh = 0.5 * (f(np.moveaxis(um, 0, 1), 0) + f(np.moveaxis(up, 0, 1), 0)) \
            - 0.5 * ax * np.moveaxis(up - um, 0, 1)               # (nc, ng, ny, nx+1)
        # y faces
        um = vals["T"][:, :, :-1, 1:-1]
        up = vals["B"][:, :, 1:, 1:-1]
        Gh = 0.5 * (f(np.moveaxis(um, 0, 1), 1) + f(np.moveaxis(up, 0, 1), 1)) \
            - 0.5 * ay * np.moveaxis(up - um, 0, 1)               # (nc, ng, ny+1, nx)
        FL, FR = Fh[..., :-1], Fh[..., 1:]
        GB, GT = Gh[..., :-1, :], Gh[..., 1:, :]
        W = self.edge_w[None, :, None, None]
        nodes = self.edge_nodes[None, :, None, None]
        fint = f(np.moveaxis(vint, 0, 1), 0)                     # (nc, 9, ny, nx)
        gint = f(np.moveaxis(vint, 0, 1), 1)
        w2 = (self.vol_w[:, None] * self.vol_w[None, :]).ravel()[None, :, None, None]
        dx, dy = self.dx, self.dy
        L = np.empty((3,) + FL.shape[:1] + FL.shape[2:], dtype=FL.dtype)
        L[0] = -(W * (FR - FL)).sum(1) / dx - (W * (GT - GB)).sum(1) / dy
        L[1] = (-(W * (FL + FR)).sum(1) / (2.0 * dx) + (w2 * fint).sum(1) / dx
                - (W * nodes * (GT - GB)).sum(1) / dy)
        L[2] = (-(W * nodes * (FR - FL)).sum(1) / dx - (W * (GB + GT)).sum(1) / (2.0 * dy)
                + (w2 * gint).sum(1) / dy)
        info = dict(T=self._sl(T, 3).astype(np.uint8), H=self._sl(H, 3).astype(np.uint8),
                    Vt=self._sl(Vt, 3), Wt=self._sl(Wt, 3))
        return L, info

    def operator(self, U, alphas=None, T_fixed=None, t=0.0):
        """Semi-discrete right-hand side L(U) of eq. ode2 (t: the time of U, which only
        prescribed boundary data depend on); returns (L, info) with
        info = dict(alpha, T, H, limited)."""
        Up = self.pad(U, t)
        ax, ay = self.alphas(U) if alphas is None else alphas
        Tp = None
        if T_fixed is not None and self.dmr:
            Tp = self._dmr_pad_flags(np.asarray(T_fixed, dtype=bool))
        elif T_fixed is not None and self.step:
            Tp = np.zeros((self.ny + 2 * NG, self.nx + 2 * NG), dtype=bool)
            Tp[NG:NG + self.ny, NG:NG + self.nx] = np.asarray(T_fixed, dtype=bool) & ~self.solid
            Tp = self._step_flags(Tp)
        elif T_fixed is not None:
            Tp = self.pad(np.broadcast_to(T_fixed.astype(float), (3, 1) + T_fixed.shape))[0, 0] > 0.5
        if Tp is not None:
            # the outermost ghost layer has no neighbours: flags there are never used
            Tp[0, :] = Tp[-1, :] = False
            Tp[:, 0] = Tp[:, -1] = False
        L, info = self.operator_padded(Up, ax, ay, Tp, ghosts=True, t=t)
        lim = U.copy()
        lim[1] = info.pop("Vt")
        lim[2] = info.pop("Wt")
        if self.step:
            # solid cells are never updated: no right-hand side, flag or limiting there
            L[:, :, self.solid] = 0.0
            lim[:, :, self.solid] = U[:, :, self.solid]
            info["T"][self.solid] = 0
            info["H"][self.solid] = 0
        info["limited"] = lim
        info["alpha"] = (ax, ay)
        return L, info

    # ------------------------------------------------------------------ Step 6
    def rk3_step(self, U, dt, frozen=None, t=0.0):
        """One TVD-RK3 step from time t.  The limited stage state (modified first moments
        in troubled cells) enters the Runge-Kutta combination.  The stage inputs are those
        of times t, t + dt and t + dt/2 (for prescribed boundary data).  frozen: optional
        list of three (alphas, T) pairs fixing each stage's Lax-Friedrichs speeds and
        troubled flags (the frozen-flag map that the adjoint differentiates).  Returns
        (U^{n+1}, infos)."""
        fz = frozen if frozen is not None else [(None, None)] * 3
        L0, i0 = self.operator(U, alphas=fz[0][0], T_fixed=fz[0][1], t=t)
        W0 = i0["limited"]
        U1 = W0 + dt * L0
        L1, i1 = self.operator(U1, alphas=fz[1][0], T_fixed=fz[1][1], t=t + dt)
        W1 = i1["limited"]
        U2 = 0.75 * W0 + 0.25 * W1 + 0.25 * dt * L1
        L2, i2 = self.operator(U2, alphas=fz[2][0], T_fixed=fz[2][1], t=t + 0.5 * dt)
        W2 = i2["limited"]
        U3 = W0 / 3.0 + 2.0 / 3.0 * W2 + 2.0 / 3.0 * dt * L2
        if self.step:
            U3[:, :, self.solid] = U[:, :, self.solid]    # solid cells keep their values
        return U3, [i0, i1, i2]

    def run(self, U, T=None, dt=None, cfl=0.6, nsteps=None, weights_fn=None):
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
            U, infos = self.rk3_step(U, h, t=t)
            t += h
            k += 1
        return U, t, k, infos
