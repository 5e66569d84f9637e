"""Double Mach reflection (Example 3.10) boundary data (oracle; test infrastructure).

The problem: a Mach 10 shock in a gamma = 1.4 gas meets a reflecting wall at 60 degrees.
The wall lies along y = 0 from x = 1/6; the shock crosses it there at t = 0 and runs into
gas at rest, (rho, u, v, p) = (1.4, 0, 0, 1); behind it (rho, u, v, p) =
(8, 8.25 cos 30deg, -8.25 sin 30deg, 116.5).  The shock line at time t is
    x = 1/6 + (y + 20 t) / sqrt(3)
(its speed normal to itself is 10).  Boundaries of [0, 4] x [0, 1]: the exact post-shock
state at x = 0 and along y = 0 for x < 1/6, a reflecting wall along y = 0 for x >= 1/6,
the exact moving shock along y = 1, outflow at x = 4.

Prescribed ghost cells hold the moments of this exact solution: the cell average and the
first moments (1/|I|) int u (x - x_c)/dx and (1/|I|) int u (y - y_c)/dy over the cell, of a
piecewise-constant state split by the shock line.  They are computed exactly by clipping
the cell (a square in reference coordinates) with the half-plane behind the shock and
integrating 1, xi and eta over the clipped polygon.  Values at boundary Gauss points are
the exact state there.
"""
import math

import numpy as np

GAMMA = 1.4
SQ3 = math.sqrt(3.0)
X_WALL = 1.0 / 6.0
POST = (8.0, 8.25 * math.cos(math.pi / 6.0), -8.25 * math.sin(math.pi / 6.0), 116.5)
PRE = (1.4, 0.0, 0.0, 1.0)


def conserved(state, gamma=GAMMA):
    rho, u, v, p = state
    return np.array([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])


U_POST = conserved(POST)
U_PRE = conserved(PRE)


def shock_offset(t):
    """c(t) with the post-shock region {x - y / sqrt(3) < c(t)}."""
    return X_WALL + 20.0 * t / SQ3


def state_at(x, y, t):
    """Exact conserved state at points (arrays) at time t: shape (4,) + x.shape."""
    post = (np.asarray(x) - np.asarray(y) / SQ3) < shock_offset(t)
    return np.where(post[None], U_POST.reshape((4,) + (1,) * np.ndim(post)),
                    U_PRE.reshape((4,) + (1,) * np.ndim(post)))


def clip_square(a, b, d):
    """Vertices of the part of the reference square [-1/2, 1/2]^2 where a xi + b eta < d
    (Sutherland-Hodgman against one half-plane), counter-clockwise."""
    sq = [(-0.5, -0.5), (0.5, -0.5), (0.5, 0.5), (-0.5, 0.5)]
    out = []
    for i in range(4):
        p, q = sq[i], sq[(i + 1) % 4]
        fp = a * p[0] + b * p[1] - d
        fq = a * q[0] + b * q[1] - d
        if fp < 0.0:
            out.append(p)
        if (fp < 0.0) != (fq < 0.0):
            s = fp / (fp - fq)
            out.append((p[0] + s * (q[0] - p[0]), p[1] + s * (q[1] - p[1])))
    return out


def polygon_moments(poly):
    """(area, int xi, int eta) of a simple polygon by the shoelace formulas."""
    A = Sx = Sy = 0.0
    n = len(poly)
    for i in range(n):
        x0, y0 = poly[i]
        x1, y1 = poly[(i + 1) % n]
        cr = x0 * y1 - x1 * y0
        A += cr
        Sx += (x0 + x1) * cr
        Sy += (y0 + y1) * cr
    return A / 2.0, Sx / 6.0, Sy / 6.0


def cell_moments(xc, yc, h, t):
    """Moments (3, 4) = (average, x moment, y moment) of each conserved component of the
    exact solution over the square cell of centre (xc, yc) and side h."""
    # x - y/sqrt3 < c  <=>  xi - eta/sqrt3 < (c - xc + yc/sqrt3)/h  in reference coordinates
    d = (shock_offset(t) - xc + yc / SQ3) / h
    poly = clip_square(1.0, -1.0 / SQ3, d)
    A, Mx, My = polygon_moments(poly) if len(poly) >= 3 else (0.0, 0.0, 0.0)
    jump = U_POST - U_PRE
    return np.stack([U_PRE + A * jump, Mx * jump, My * jump])
