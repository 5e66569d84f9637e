"""Exact solution of the Riemann problem of the 1D Euler equations (oracle; test
infrastructure, imported only by the tests).

The shock tests of Section 3.2 compare the scheme's density with the exact solution; for
the Lax problem (Example 3.6) that solution is the self-similar solution of a Riemann
problem for a gamma-law gas.  It is written out here from the textbook theory of that
problem (two nonlinear waves, each a shock or a rarefaction, around a contact; the star
pressure is the root of a monotone function):

* f_K(p) (K = L, R) is the velocity change across the K wave that takes the state K to
  pressure p: for p > p_K a shock, (p - p_K) sqrt(A_K / (p + B_K)) with
  A_K = 2 / ((gamma + 1) rho_K), B_K = p_K (gamma - 1)/(gamma + 1); otherwise a
  rarefaction, 2 c_K / (gamma - 1) ((p / p_K)^((gamma - 1)/(2 gamma)) - 1).
* p* solves f_L(p) + f_R(p) + u_R - u_L = 0 (f_L + f_R increases with p; the root is
  bracketed and found by Brent's method), u* = (u_L + u_R + f_R(p*) - f_L(p*)) / 2.
* the solution at x/t follows from the wave speeds: a shock moves at
  u_K -+ c_K sqrt((gamma + 1)/(2 gamma) p*/p_K + (gamma - 1)/(2 gamma)) and leaves the
  density rho_K (p*/p_K + m) / (m p*/p_K + 1), m = (gamma - 1)/(gamma + 1); a rarefaction
  spans u_K -+ c_K to u* -+ c*_K with c*_K = c_K (p*/p_K)^((gamma - 1)/(2 gamma)), leaves
  rho_K (p*/p_K)^(1/gamma), and inside it the state is isentropic with the Riemann
  invariant u +- 2c/(gamma - 1) of the K side.

Pins (tests/test_oracle_shock_suite.py): the star states of two textbook Riemann problems
(Sod's shock tube and the symmetric double rarefaction), the Rankine-Hugoniot conditions
across the computed shocks, isentropy and the Riemann invariant across the computed
rarefactions, mirror symmetry, and a uniform state.
"""
import math

import numpy as np
from scipy.optimize import brentq


class RiemannExact:
    """Exact solution of the Riemann problem (rho, u, p)_L | (rho, u, p)_R at x = x0."""

    def __init__(self, left, right, gamma=1.4, x0=0.0):
        self.g = float(gamma)
        self.x0 = float(x0)
        self.L = tuple(float(v) for v in left)
        self.R = tuple(float(v) for v in right)
        g = self.g
        rl, ul, pl = self.L
        rr, ur, pr = self.R
        self.cl = math.sqrt(g * pl / rl)
        self.cr = math.sqrt(g * pr / rr)
        if 2.0 * (self.cl + self.cr) / (g - 1.0) <= ur - ul:
            raise ValueError("the data generate a vacuum")
        F = lambda p: self._f(p, rl, pl, self.cl) + self._f(p, rr, pr, self.cr) + ur - ul
        lo, hi = 1e-14 * min(pl, pr), max(pl, pr)
        while F(hi) < 0.0:
            hi *= 2.0
        self.ps = brentq(F, lo, hi, xtol=1e-15 * hi, rtol=4 * np.finfo(float).eps, maxiter=500)
        self.us = 0.5 * (ul + ur + self._f(self.ps, rr, pr, self.cr) - self._f(self.ps, rl, pl, self.cl))
        m = (g - 1.0) / (g + 1.0)
        self.rho_star = []
        for (rk, uk, pk) in (self.L, self.R):
            q = self.ps / pk
            self.rho_star.append(rk * (q + m) / (m * q + 1.0) if q > 1.0 else rk * q ** (1.0 / g))

    def _f(self, p, rk, pk, ck):
        g = self.g
        if p > pk:
            A = 2.0 / ((g + 1.0) * rk)
            B = pk * (g - 1.0) / (g + 1.0)
            return (p - pk) * math.sqrt(A / (p + B))
        return 2.0 * ck / (g - 1.0) * ((p / pk) ** ((g - 1.0) / (2.0 * g)) - 1.0)

    def _side(self, s, rk, uk, pk, ck, sign, rho_star):
        """State at similarity coordinate s on the K side of the contact; sign = -1 for the
        left wave (moving left relative to the gas), +1 for the right one."""
        g = self.g
        q = self.ps / pk
        if q > 1.0:   # shock
            S = uk + sign * ck * math.sqrt((g + 1.0) / (2.0 * g) * q + (g - 1.0) / (2.0 * g))
            outside = s < S if sign < 0 else s > S
            return (rk, uk, pk) if outside else (rho_star, self.us, self.ps)
        head = uk + sign * ck
        cs = ck * q ** ((g - 1.0) / (2.0 * g))
        tail = self.us + sign * cs
        if (s < head) if sign < 0 else (s > head):
            return (rk, uk, pk)
        if (s > tail) if sign < 0 else (s < tail):
            return (rho_star, self.us, self.ps)
        # inside the fan: u + sign c = s (the fan's own characteristic family), and
        # u - sign 2c/(g-1) keeps its value on the K side
        c = (2.0 / (g + 1.0)) * (ck - sign * 0.5 * (g - 1.0) * (uk - s))
        u = s - sign * c
        rho = rk * (c / ck) ** (2.0 / (g - 1.0))
        p = pk * (c / ck) ** (2.0 * g / (g - 1.0))
        return (rho, u, p)

    def sample(self, x, t):
        """Primitive variables (rho, u, p), each shaped like x, at time t > 0."""
        x = np.asarray(x, dtype=float)
        out = np.empty((3,) + x.shape)
        for idx, xv in np.ndenumerate(x):
            s = (xv - self.x0) / t
            if s <= self.us:
                st = self._side(s, *self.L, self.cl, -1.0, self.rho_star[0])
            else:
                st = self._side(s, *self.R, self.cr, +1.0, self.rho_star[1])
            out[(slice(None),) + idx] = st
        return out

    def cell_averages(self, x0, x1, n, t, per_cell=400):
        """Cell averages of rho, u, p over n uniform cells of [x0, x1] (midpoint rule with
        per_cell points per cell: exact inside the constant regions, O(1/per_cell) of a
        jump in the few cells a discontinuity crosses)."""
        dx = (x1 - x0) / n
        pts = x0 + dx * (np.arange(n)[:, None] + (np.arange(per_cell)[None, :] + 0.5) / per_cell)
        return self.sample(pts, t).mean(axis=-1)
