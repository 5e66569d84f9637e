"""Flux functions, wave speeds and characteristic eigenvectors (oracle; test infrastructure).

Equations (Section 2 and Section 3 of the paper):
* linear advection  u_t + a u_x (+ b u_y) = 0            (eq. EQ / EQ2 with f = a u, g = b u)
* Burgers           u_t + (u^2/2)_x (+ (u^2/2)_y) = 0    (eqs. 1dbugers, 2dbugers)
* Euler, gamma-law  eqs. euler1 (1D: rho, rho*mu, E) and euler2 (2D: rho, rho*mu, rho*nu, E)

A state array has the conserved components on axis 0.

Characteristic fields (Remarks 2 and 4): right eigenvectors of the flux Jacobian in the
textbook normalisation below, evaluated at the cell-average state of the cell being
limited or reconstructed; the left eigenvectors are the exact matrix inverse (computed
here with numpy.linalg.inv, deliberately not a closed form).
  1D:      R = [[1, 1, 1], [u-c, u, u+c], [H-u c, u^2/2, H+u c]]
  2D, x:   columns (1, u-c, v, H-u c), (1, u, v, q2/2), (0, 0, 1, v), (1, u+c, v, H+u c)
  2D, y:   columns (1, u, v-c, H-v c), (1, u, v, q2/2), (0, 1, 0, u), (1, u, v+c, H+v c)
with H = (E + p)/rho, c = sqrt(gamma p / rho), q2 = u^2 + v^2.

Pins (tests/test_oracle_physics.py): A R = R Lambda with A the flux Jacobian obtained by
complex-step differentiation of the flux functions, and L R = I.
"""
import numpy as np


class Equation:
    """Conservation law: name in {'advection', 'burgers', 'euler'}."""

    def __init__(self, name, dim, adv=(1.0, 1.0), gamma=1.4):
        if name not in ("advection", "burgers", "euler"):
            raise ValueError(name)
        self.name = name
        self.dim = dim
        self.adv = tuple(float(a) for a in adv)
        self.gamma = float(gamma)
        self.ncomp = (dim + 2) if name == "euler" else 1

    # ---------------------------------------------------------------- fluxes
    def flux(self, U, d):
        """Physical flux in direction d (0 = x: f, 1 = y: g) of the point state U."""
        if self.name == "advection":
            return self.adv[d] * U
        if self.name == "burgers":
            return 0.5 * U * U
        g = self.gamma
        rho = U[0]
        mom = U[1:1 + self.dim]
        E = U[1 + self.dim]
        kin = sum(m * m for m in mom) / (2.0 * rho)
        p = (g - 1.0) * (E - kin)
        vel_d = mom[d] / rho
        out = [mom[d]]
        for k in range(self.dim):
            out.append(mom[k] * vel_d + (p if k == d else 0.0))
        out.append(vel_d * (E + p))
        return np.stack(out)

    def pressure(self, U):
        rho = U[0]
        mom = U[1:1 + self.dim]
        E = U[1 + self.dim]
        return (self.gamma - 1.0) * (E - sum(m * m for m in mom) / (2.0 * rho))

    # ---------------------------------------------------------------- wave speeds
    def spectral_radius(self, Ubar, d):
        """|f'(u)| (scalar) or |velocity_d| + c (Euler) at cell-average states."""
        if self.name == "advection":
            return np.full(np.shape(Ubar[0]), abs(self.adv[d]))
        if self.name == "burgers":
            return np.abs(Ubar[0])
        rho = Ubar[0]
        p = self.pressure(Ubar)
        c = np.sqrt(self.gamma * p / rho)
        return np.abs(Ubar[1 + d] / rho) + c

    def velocity(self, Ubar, d):
        """Velocity used by the troubled-cell indicator (Remarks 1, 3): f'(u) or g'(u) for
        a scalar law, the fluid velocity for Euler, at cell-average states."""
        if self.name == "advection":
            return np.full(np.shape(Ubar[0]), self.adv[d])
        if self.name == "burgers":
            return np.array(Ubar[0], dtype=float)
        return Ubar[1 + d] / Ubar[0]

    # ---------------------------------------------------------------- eigenvectors
    def right_eigenvectors(self, ubar, d):
        """Right eigenvector matrices at cell-average states.

        ubar: shape (ncomp,) or (ncomp, k).  Returns (ncomp, ncomp) or (k, ncomp, ncomp)
        with the eigenvectors as columns."""
        ubar = np.asarray(ubar)
        single = ubar.ndim == 1
        if single:
            ubar = ubar[:, None]
        g = self.gamma
        rho = ubar[0]
        one = np.ones_like(rho)
        zero = np.zeros_like(rho)
        if self.dim == 1:
            u = ubar[1] / rho
            E = ubar[2]
            p = (g - 1.0) * (E - 0.5 * rho * u * u)
            c = np.sqrt(g * p / rho)
            H = (E + p) / rho
            rows = [[one, one, one],
                    [u - c, u, u + c],
                    [H - u * c, 0.5 * u * u, H + u * c]]
        else:
            u = ubar[1] / rho
            v = ubar[2] / rho
            E = ubar[3]
            q2 = u * u + v * v
            p = (g - 1.0) * (E - 0.5 * rho * q2)
            c = np.sqrt(g * p / rho)
            H = (E + p) / rho
            if d == 0:
                rows = [[one, one, zero, one],
                        [u - c, u, zero, u + c],
                        [v, v, one, v],
                        [H - u * c, 0.5 * q2, v, H + u * c]]
            else:
                rows = [[one, one, zero, one],
                        [u, u, one, u],
                        [v - c, v, zero, v + c],
                        [H - v * c, 0.5 * q2, u, H + v * c]]
        R = np.moveaxis(np.array(rows), -1, 0)
        return R[0] if single else R

    def eigen_pair(self, ubar, d):
        """(L, R) with L = inverse of R, batched like right_eigenvectors."""
        R = self.right_eigenvectors(ubar, d)
        return np.linalg.inv(R), R

    def eigenvalues(self, ubar, d):
        g = self.gamma
        rho = ubar[0]
        mom = [ubar[1 + k] for k in range(self.dim)]
        E = ubar[1 + self.dim]
        q2 = sum((m / rho) ** 2 for m in mom)
        p = (g - 1.0) * (E - 0.5 * rho * q2)
        c = np.sqrt(g * p / rho)
        un = mom[d] / rho
        if self.dim == 1:
            return np.array([un - c, un, un + c])
        return np.array([un - c, un, un, un + c])
