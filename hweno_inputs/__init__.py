"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module only builds initial states: it draws the seeded parameters of each workload
and projects the resulting initial function onto the scheme's unknowns (cell averages and
first moments, the initial conditions stated below eq. odeH and eq. ode2).  It contains
none of the scheme's arithmetic and imports neither the oracle nor the GPU package.

Projection: per cell (or per piece of a cell split at the breakpoints of a
piecewise-defined function), Gauss-Legendre quadrature with ``nq`` points per direction
in reference coordinates xi = (x - x_i)/dx in [-1/2, 1/2]:
    ubar = int u dxi,   vbar = int u xi dxi   (and wbar = int u eta in 2D).

Workloads (arrays are float64, shape (2, ncomp, n) in 1D and (3, ncomp, ny, nx) in 2D,
moment index first: 0 = averages, 1 = x first moments, 2 = y first moments):

* advection_1d(seed, n)      u0 = 1 + sum_{k=1..3} a_k sin(k pi x + phi_k) on [0, 2],
                             a_k ~ U[-0.5, 0.5], phi_k ~ U[0, 2 pi)
* euler_riemann_1d(seed, n)  2-4 piecewise-constant states separated at sorted U[0.1, 0.9]
                             breakpoints on [0, 1]; rho_s ~ U[0.1, 1], u_s ~ U[-1, 1],
                             p_s ~ U[0.1, 1]; density rho_s (1 + 0.2 sin(k x)), k ~ U{5..20}
* euler_shock_vortex_2d(seed, n)  [0, 1]^2: planar shock of seeded normal angle and pressure
                             ratio U[2, 10] (post-shock state by Rankine-Hugoniot) with an
                             isentropic vortex of strength U[1, 5] and radius 0.05 superposed
* euler_wall_state(nx, ny, seed)  2D Euler cell averages with an oblique jump that meets
                             all four sides, flow towards the sides and seeded first
                             moments of size 0.01 (troubled cells along every side)
* euler_dmr_state(nx, ny, h, seed)  the double Mach reflection's initial state on a small
                             mesh of cell size h, with jump bands along the left and right
                             sides and seeded first-moment noise of size 0.002
* euler_step_state(nx, ny, si, sj, seed)  the same kind of data on a forward-step mesh:
                             jumps in bands along the channel's sides and the step's two
                             faces, solid cells at the Mach 3 free stream
* batch_sizes(seed, count)   instance sizes log-uniform in [256, 8192]
* non-uniform 1D meshes: stretched_faces(n, x0, x1, amp) (x = s + amp sin(2 pi s)/(2 pi)),
  random_faces(seed, n, x0, x1, ratio) (cell sizes U[1, ratio], rng(6000 + seed)), and
  project_1d_faces(func, faces) (averages and first moments on those cells)
* burgers_modes_2d(seed, n)  u0 = 0.5 + 0.25 sum_{m=1..4} a_m sin(pi (k_m x + l_m y)/2 + phi_m)
                             on [0, 4]^2, (k_m, l_m) in {0,1,2}^2 \\ {0}, sum |a_m| = 1
* paper examples 3.1-3.4 (smooth accuracy tests of Section 3.1) and the initial states of
  the 1D shock tests of Section 3.2 (Examples 3.5-3.8; 3.5 and 3.9 reuse the initial
  states of 3.1 and 3.3 up to a later final time)
* example_3_10(nx, ny)       double Mach reflection on [0, 4] x [0, 1]: a Mach 10 shock
                             through (1/6, 0) at 60 degrees to the x axis, projected exactly
                             (each cell split by the shock line)
* example_3_11(nx, ny)       forward step on [0, 3] x [0, 1]: the Mach 3 free stream
                             (rho, u, v, p) = (1.4, 3, 0, 1) in every cell (the cells inside
                             the step included; they are never updated)
"""
import math

import numpy as np

GAMMA = 1.4


def gauss_legendre_ref(nq):
    """Nodes and weights of the nq-point Gauss-Legendre rule on [-1/2, 1/2]."""
    x, w = np.polynomial.legendre.leggauss(nq)
    return 0.5 * x, 0.5 * w


def project_1d(func, x0, x1, n, breakpoints=(), nq=10):
    """Cell averages and first moments of func (vectorised, returns (ncomp, npts)).

    Cells that contain a breakpoint are integrated piece by piece."""
    dx = (x1 - x0) / n
    xs, ws = gauss_legendre_ref(nq)
    centres = x0 + (np.arange(n) + 0.5) * dx
    # plain cells
    pts = centres[None, :] + dx * xs[:, None]          # (nq, n)
    vals = np.asarray(func(pts.ravel())).reshape(-1, nq, n)
    avg = np.einsum("q,cqn->cn", ws, vals)
    mom = np.einsum("q,cqn->cn", ws * xs, vals)
    # cells split by breakpoints
    bps = sorted(float(b) for b in breakpoints)
    for i in sorted({int((b - x0) // dx) for b in bps if x0 < b < x1}):
        a = -0.5
        cuts = [((b - x0) / dx - i - 0.5) for b in bps if x0 + i * dx < b < x0 + (i + 1) * dx]
        a_list = [a] + cuts
        b_list = cuts + [0.5]
        acc0 = 0.0
        acc1 = 0.0
        for lo, hi in zip(a_list, b_list):
            h = hi - lo
            xi = lo + h * (xs + 0.5)
            # sample strictly inside the piece
            v = np.asarray(func(centres[i] + dx * xi)).reshape(-1, nq)
            acc0 = acc0 + h * (v @ ws)
            acc1 = acc1 + h * (v @ (ws * xi))
        avg[:, i] = acc0
        mom[:, i] = acc1
    return np.stack([avg, mom])


def project_1d_faces(func, faces, nq=10):
    """Cell averages and first moments of func on the mesh with the given face
    coordinates: per cell, (1/dx_i) int u dx and (1/dx_i) int u (x - x_i)/dx_i dx by nq-point
    Gauss-Legendre (func vectorised, returns (ncomp, npts))."""
    faces = np.asarray(faces, dtype=float)
    dx = np.diff(faces)
    centres = 0.5 * (faces[1:] + faces[:-1])
    xs, ws = gauss_legendre_ref(nq)
    pts = centres[None, :] + dx[None, :] * xs[:, None]
    vals = np.asarray(func(pts.ravel())).reshape(-1, nq, len(dx))
    return np.stack([np.einsum("q,cqn->cn", ws, vals), np.einsum("q,cqn->cn", ws * xs, vals)])


def stretched_faces(n, x0, x1, amp=0.3):
    """Faces of a smoothly stretched mesh: x(s) = s + amp sin(2 pi s) / (2 pi) on [0, 1]
    mapped to [x0, x1] (cell sizes vary smoothly by a factor (1 + amp) / (1 - amp), and
    periodically, so the mesh suits periodic problems)."""
    s = np.linspace(0.0, 1.0, n + 1)
    return x0 + (x1 - x0) * (s + amp * np.sin(2.0 * np.pi * s) / (2.0 * np.pi))


def random_faces(seed, n, x0, x1, ratio=3.0):
    """Faces of a mesh with independent cell sizes drawn from U[1, ratio] (rng(6000 + seed)),
    scaled to fill [x0, x1]."""
    w = np.random.default_rng(6000 + seed).uniform(1.0, ratio, n)
    return x0 + (x1 - x0) * np.concatenate([[0.0], np.cumsum(w) / w.sum()])


def project_2d(func, x0, x1, y0, y1, nx, ny, nq=5, chunk_rows=64):
    """Cell averages and x/y first moments of func(x, y) -> (ncomp, ...) over a uniform
    nx x ny mesh, with an nq x nq Gauss-Legendre rule per cell."""
    dx = (x1 - x0) / nx
    dy = (y1 - y0) / ny
    xs, ws = gauss_legendre_ref(nq)
    xc = x0 + (np.arange(nx) + 0.5) * dx
    out = None
    for r0 in range(0, ny, chunk_rows):
        r1 = min(ny, r0 + chunk_rows)
        yc = y0 + (np.arange(r0, r1) + 0.5) * dy
        X = xc[None, None, None, :] + dx * xs[None, :, None, None]   # (1, qx, 1, nx)
        Y = yc[None, None, :, None] + dy * xs[:, None, None, None]   # (qy, 1, r, 1)
        X, Y = np.broadcast_arrays(X, Y)                             # (qy, qx, r, nx)
        v = np.asarray(func(X, Y))                                   # (c, qy, qx, r, nx)
        if out is None:
            out = np.zeros((3, v.shape[0], ny, nx))
        w2 = ws[:, None] * ws[None, :]
        out[0, :, r0:r1] = np.einsum("yx,cyxrn->crn", w2, v)
        out[1, :, r0:r1] = np.einsum("yx,cyxrn->crn", w2 * xs[None, :], v)
        out[2, :, r0:r1] = np.einsum("yx,cyxrn->crn", w2 * xs[:, None], v)
    return out


def primitive_to_conserved(rho, vel, p, gamma=GAMMA):
    """Conserved components (rho, momenta..., E) from density, velocity list, pressure."""
    kin = 0.5 * rho * sum(u * u for u in vel)
    return np.stack([rho] + [rho * u for u in vel] + [p / (gamma - 1.0) + kin])


# ------------------------------------------------------------------------------ 1D


def advection_1d(seed=0, n=160):
    rng = np.random.default_rng(1000 + seed)
    a = rng.uniform(-0.5, 0.5, 3)
    phi = rng.uniform(0.0, 2.0 * math.pi, 3)

    def u0(x):
        x = np.asarray(x, dtype=float)
        return (1.0 + sum(a[k] * np.sin((k + 1) * math.pi * x + phi[k]) for k in range(3)))[None]

    return project_1d(u0, 0.0, 2.0, n), dict(a=a, phi=phi, func=u0, x0=0.0, x1=2.0)


def euler_riemann_params(rng):
    nstates = int(rng.integers(2, 5))
    bps = np.sort(rng.uniform(0.1, 0.9, nstates - 1))
    states = [(rng.uniform(0.1, 1.0), rng.uniform(-1.0, 1.0), rng.uniform(0.1, 1.0))
              for _ in range(nstates)]
    k = int(rng.integers(5, 21))
    return bps, states, k


def euler_riemann_func(bps, states, k, gamma=GAMMA):
    def u0(x):
        x = np.asarray(x, dtype=float)
        idx = np.searchsorted(bps, x, side="right")
        rho_s = np.array([s[0] for s in states])[idx]
        u_s = np.array([s[1] for s in states])[idx]
        p_s = np.array([s[2] for s in states])[idx]
        rho = rho_s * (1.0 + 0.2 * np.sin(k * x))
        return primitive_to_conserved(rho, [u_s], p_s, gamma)
    return u0


def euler_riemann_1d(seed=0, n=2000, rng=None):
    if rng is None:
        rng = np.random.default_rng(2000 + seed)
    bps, states, k = euler_riemann_params(rng)
    u0 = euler_riemann_func(bps, states, k)
    U = project_1d(u0, 0.0, 1.0, n, breakpoints=bps)
    return U, dict(breakpoints=bps, states=states, k=k, func=u0, x0=0.0, x1=1.0)


def batch_sizes(seed=0, count=512, lo=256, hi=8192):
    ss = np.random.SeedSequence(4000 + seed)
    children = ss.spawn(count + 1)
    rng = np.random.default_rng(children[0])
    sizes = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), count))).astype(np.int64)
    return sizes, children[1:]


def batch_euler_1d(seed=0, count=512, lo=256, hi=8192):
    """Independent 1D Euler instances on [0, 1] (transmissive), each drawn with the
    piecewise-constant generator from its own child seed.  Returns (list of U, sizes)."""
    sizes, children = batch_sizes(seed, count, lo, hi)
    Us = []
    for nb, ch in zip(sizes, children):
        U, _ = euler_riemann_1d(n=int(nb), rng=np.random.default_rng(ch))
        Us.append(U)
    return Us, sizes


# ------------------------------------------------------------------------------ 2D


def euler_shock_vortex_params(seed):
    rng = np.random.default_rng(3000 + seed)
    theta = rng.uniform(0.0, 2.0 * math.pi)
    ratio = rng.uniform(2.0, 10.0)
    strength = rng.uniform(1.0, 5.0)
    centre = rng.uniform(0.25, 0.75, 2)
    return dict(theta=theta, ratio=ratio, strength=strength, centre=centre, radius=0.05)


def euler_shock_vortex_func(prm, gamma=GAMMA):
    g = gamma
    nx_, ny_ = math.cos(prm["theta"]), math.sin(prm["theta"])
    ps = prm["ratio"]
    rho2 = ((g + 1.0) * ps + g - 1.0) / ((g - 1.0) * ps + g + 1.0)
    c1 = math.sqrt(g)
    S = c1 * math.sqrt((g + 1.0) * (ps - 1.0) / (2.0 * g) + 1.0)
    u2 = S * (1.0 - 1.0 / rho2)
    eps_v = prm["strength"]
    xv, yv = prm["centre"]
    R = prm["radius"]

    def u0(x, y):
        pre = (nx_ * (x - 0.5) + ny_ * (y - 0.5)) > 0.0
        rho_b = np.where(pre, 1.0, rho2)
        p_b = np.where(pre, 1.0, ps)
        ub = np.where(pre, 0.0, u2 * nx_)
        vb = np.where(pre, 0.0, u2 * ny_)
        r2 = ((x - xv) ** 2 + (y - yv) ** 2) / (R * R)
        amp = eps_v / (2.0 * math.pi) * np.exp(0.5 * (1.0 - r2))
        du = -amp * (y - yv) / R
        dv = amp * (x - xv) / R
        dT = -(g - 1.0) * eps_v ** 2 / (8.0 * g * math.pi ** 2) * np.exp(1.0 - r2)
        Tb = p_b / rho_b
        T = Tb + dT
        rho = rho_b * (T / Tb) ** (1.0 / (g - 1.0))
        p = rho * T
        return primitive_to_conserved(rho, [ub + du, vb + dv], p, g)

    return u0


def euler_shock_vortex_2d(seed=0, n=1024, nq=5):
    prm = euler_shock_vortex_params(seed)
    u0 = euler_shock_vortex_func(prm)
    U = project_2d(u0, 0.0, 1.0, 0.0, 1.0, n, n, nq=nq)
    return U, dict(prm, func=u0)


def euler_wall_state(nx, ny, seed=0):
    """2D Euler data for meshes with walls: density and pressure jump across the line
    x + 0.7 y = 0.6 and near the right and top sides, velocities pointing at the nearest
    side, first moments drawn N(0, 0.01^2) (cell-centre coordinates of the unit square)."""
    rng = np.random.default_rng(seed)
    xc, yc = (np.arange(nx) + 0.5) / nx, (np.arange(ny) + 0.5) / ny
    X, Y = np.meshgrid(xc, yc)
    front = (X + 0.7 * Y < 0.6) | (X > 0.93) | (Y > 0.9)
    rho = 1.0 + 0.5 * front
    u = 0.4 * np.where(X < 0.5, -1.0, 1.0) + 0.1 * np.sin(3.0 * Y)
    v = 0.3 * np.where(Y < 0.5, -1.0, 1.0) + 0.1 * np.cos(2.0 * X)
    p = 1.0 + 0.8 * front
    U = np.zeros((3, 4, ny, nx))
    U[0] = primitive_to_conserved(rho, [u, v], p)
    U[1:] = 0.01 * rng.normal(size=(2, 4, ny, nx))
    return U


def euler_step_state(nx, ny, si, sj, seed=0):
    """2D Euler data for a forward-step mesh of nx x ny cells whose solid cells are
    i >= si, j < sj (they hold the Mach 3 free stream): density and pressure jump in bands
    one and a half cells wide along part of every side of the fluid -- the lower half of the
    inflow side, the upper half of the exit, the left half of the top wall, the channel
    floor, the step's left face and the right half of its top face -- so that troubled and
    linear cells both meet every kind of boundary; velocity to the right with a vertical
    component towards the nearest wall; first moments drawn N(0, 0.002^2)."""
    rng = np.random.default_rng(seed)
    i, j = np.meshgrid(np.arange(nx) + 0.5, np.arange(ny) + 0.5)
    solid = (i > si) & (j < sj)
    band = (((i < 1.5) & (j < 0.5 * ny)) | ((i > nx - 1.5) & (j > 0.5 * (ny + sj)))
            | ((j > ny - 1.5) & (i < 0.5 * nx)) | ((j < 1.5) & (i < si))
            | ((np.abs(i - si) < 1.5) & (j < sj + 1.0))
            | ((np.abs(j - sj) < 1.5) & (i > 0.5 * (si + nx))))
    rho = 1.0 + 0.5 * band
    u = 0.6 + 0.02 * np.sin(0.5 * j)
    v = np.where(j > 0.5 * (ny + sj), 0.2, -0.2)
    p = 1.0 + 0.8 * band
    U = np.zeros((3, 4, ny, nx))
    U[0] = primitive_to_conserved(rho, [u, v], p)
    U[1:] = 0.002 * rng.normal(size=(2, 4, ny, nx))
    m = int(solid.sum())
    U[0][:, solid] = primitive_to_conserved(np.full(m, 1.4), [np.full(m, 3.0), np.zeros(m)], np.ones(m))
    U[1:, :, solid] = 0.0
    return U


def burgers_modes_params(seed):
    rng = np.random.default_rng(seed)
    choices = [(k, l) for k in range(3) for l in range(3) if (k, l) != (0, 0)]
    idx = rng.integers(0, len(choices), 4)
    kl = [choices[i] for i in idx]
    a = rng.uniform(-1.0, 1.0, 4)
    a = a / np.sum(np.abs(a))
    phi = rng.uniform(0.0, 2.0 * math.pi, 4)
    return kl, a, phi


def burgers_modes_func(kl, a, phi):
    def u0(x, y):
        s = sum(a[m] * np.sin(math.pi * (kl[m][0] * x + kl[m][1] * y) / 2.0 + phi[m])
                for m in range(4))
        return (0.5 + 0.25 * s)[None]
    return u0


def burgers_modes_2d(seed=0, n=256, target=False, nq=5):
    kl, a, phi = burgers_modes_params((5100 if target else 5000) + seed)
    u0 = burgers_modes_func(kl, a, phi)
    return project_2d(u0, 0.0, 4.0, 0.0, 4.0, n, n, nq=nq), dict(kl=kl, a=a, phi=phi, func=u0)


# ------------------------------------------------------------------------------ paper examples


def example_3_1(n):
    """Burgers, u0 = 0.5 + sin(pi x) on [0, 2], periodic."""
    f = lambda x: (0.5 + np.sin(math.pi * np.asarray(x)))[None]
    return project_1d(f, 0.0, 2.0, n)


def example_3_2(n, x1=2.0):
    """Euler density wave rho = 1 + 0.2 sin(pi x), velocity 1, pressure 1, periodic."""
    def f(x):
        x = np.asarray(x, dtype=float)
        rho = 1.0 + 0.2 * np.sin(math.pi * x)
        return primitive_to_conserved(rho, [np.ones_like(x)], np.ones_like(x))
    return project_1d(f, 0.0, x1, n)


def example_3_3(n):
    """2D Burgers, u0 = 0.5 + sin(pi (x + y)/2) on [0, 4]^2, periodic."""
    f = lambda x, y: (0.5 + np.sin(math.pi * (x + y) / 2.0))[None]
    return project_2d(f, 0.0, 4.0, 0.0, 4.0, n, n, nq=6)


def example_3_4(n):
    """2D Euler density wave rho = 1 + 0.2 sin(pi (x + y)), velocity (1, 1), pressure 1,
    on [0, 2]^2, periodic."""
    def f(x, y):
        rho = 1.0 + 0.2 * np.sin(math.pi * (x + y))
        one = np.ones_like(x)
        return primitive_to_conserved(rho, [one, one], one)
    return project_2d(f, 0.0, 2.0, 0.0, 2.0, n, n, nq=6)


def example_3_6(n):
    """Lax problem on [-0.5, 0.5] (transmissive): (rho, u, p) = (0.445, 0.698, 3.528) for
    x < 0 and (0.5, 0, 0.571) for x >= 0, gamma = 1.4."""
    left, right = (0.445, 0.698, 3.528), (0.5, 0.0, 0.571)

    def f(x):
        x = np.asarray(x, dtype=float)
        st = [np.where(x < 0.0, a, b) for a, b in zip(left, right)]
        return primitive_to_conserved(st[0], [st[1]], st[2])
    return project_1d(f, -0.5, 0.5, n, breakpoints=(0.0,))


def example_3_7(n):
    """Shu-Osher problem on [-5, 5] (transmissive): (rho, u, p) = (3.857143, 2.629369,
    10.333333) for x < -4 and (1 + 0.2 sin(5 x), 0, 1) for x >= -4, gamma = 1.4."""
    def f(x):
        x = np.asarray(x, dtype=float)
        post = x < -4.0
        rho = np.where(post, 3.857143, 1.0 + 0.2 * np.sin(5.0 * x))
        u = np.where(post, 2.629369, 0.0)
        p = np.where(post, 10.333333, 1.0)
        return primitive_to_conserved(rho, [u], p)
    return project_1d(f, -5.0, 5.0, n, breakpoints=(-4.0,))


def example_3_8(n):
    """Interaction of two blast waves on [0, 1] (reflective walls): rho = 1, u = 0 and
    p = 1000 for x < 0.1, 0.01 for 0.1 < x < 0.9, 100 for x > 0.9, gamma = 1.4."""
    def f(x):
        x = np.asarray(x, dtype=float)
        p = np.where(x < 0.1, 1000.0, np.where(x < 0.9, 0.01, 100.0))
        one = np.ones_like(x)
        return primitive_to_conserved(one, [0.0 * one], p)
    return project_1d(f, 0.0, 1.0, n, breakpoints=(0.1, 0.9))


# ------------------------------------------------------------------------------ Example 3.10


def _halfplane_square_moments(d, a, b):
    """(area, int xi, int eta) of {a xi + b eta < d} within [-1/2, 1/2]^2: the square's
    vertices inside the half-plane plus its crossings of the edges, in order, integrated by
    the shoelace formulas."""
    sq = [(-0.5, -0.5), (0.5, -0.5), (0.5, 0.5), (-0.5, 0.5)]
    poly = []
    for i in range(4):
        (x0, y0), (x1, y1) = sq[i], sq[(i + 1) % 4]
        f0, f1 = a * x0 + b * y0 - d, a * x1 + b * y1 - d
        if f0 < 0.0:
            poly.append((x0, y0))
        if (f0 < 0.0) != (f1 < 0.0):
            s = f0 / (f0 - f1)
            poly.append((x0 + s * (x1 - x0), y0 + s * (y1 - y0)))
    if len(poly) < 3:
        return 0.0, 0.0, 0.0
    A = Sx = Sy = 0.0
    for i in range(len(poly)):
        (x0, y0), (x1, y1) = poly[i], poly[(i + 1) % len(poly)]
        cr = x0 * y1 - x1 * y0
        A += cr
        Sx += (x0 + x1) * cr
        Sy += (y0 + y1) * cr
    return A / 2.0, Sx / 6.0, Sy / 6.0


def example_3_10(nx=1920, ny=480, h=None):
    """Double Mach reflection on [0, 4] x [0, 1] (square cells): behind the Mach 10 shock
    x < 1/6 + y/sqrt(3), (rho, u, v, p) = (8, 8.25 cos 30deg, -8.25 sin 30deg, 116.5); ahead
    of it the gas at rest, (1.4, 0, 0, 1).  Cells the shock line crosses take the exact
    area-weighted moments.  h: the cell size of a mesh of [0, nx h] x [0, ny h] instead."""
    if h is None:
        h = 4.0 / nx
        if abs(h - 1.0 / ny) > 1e-12 * h:
            raise ValueError("the double Mach reflection mesh needs square cells (nx = 4 ny)")
    post = primitive_to_conserved(np.array(8.0), [np.array(8.25 * math.cos(math.pi / 6)),
                                                  np.array(-8.25 * math.sin(math.pi / 6))], np.array(116.5))
    pre = primitive_to_conserved(np.array(1.4), [np.array(0.0), np.array(0.0)], np.array(1.0))
    post, pre = np.asarray(post, dtype=float), np.asarray(pre, dtype=float)
    s3 = math.sqrt(3.0)
    xc = (np.arange(nx) + 0.5) * h
    yc = (np.arange(ny) + 0.5) * h
    U = np.zeros((3, 4, ny, nx))
    U[0] = pre[:, None, None]
    X, Y = np.meshgrid(xc, yc)
    d = (1.0 / 6.0 - X + Y / s3) / h            # behind the shock: xi - eta/sqrt3 < d
    lim = 0.5 + 0.5 / s3
    U[0][:, d >= lim] = post[:, None]
    for j, i in zip(*np.nonzero(np.abs(d) < lim)):
        A, Mx, My = _halfplane_square_moments(d[j, i], 1.0, -1.0 / s3)
        U[0, :, j, i] = pre + A * (post - pre)
        U[1, :, j, i] = Mx * (post - pre)
        U[2, :, j, i] = My * (post - pre)
    return U


def euler_dmr_state(nx, ny, h, seed=0):
    """2D Euler data for a small double Mach reflection mesh of [0, nx h] x [0, ny h]: the
    initial state of example_3_10 on it, with density and pressure raised by 30 % and the
    x velocity by 0.5 in bands one and a half cells wide along the left and right sides,
    and first moments perturbed by N(0, 0.002^2) (troubled cells then meet the prescribed,
    wall and outflow sides)."""
    rng = np.random.default_rng(seed)
    U = example_3_10(nx, ny, h=h)
    i = np.arange(nx) + 0.5
    band = (i < 1.5) | (i > nx - 1.5)
    rho = U[0, 0]
    vel = [U[0, 1] / rho, U[0, 2] / rho]
    p = (GAMMA - 1.0) * (U[0, 3] - 0.5 * rho * (vel[0] ** 2 + vel[1] ** 2))
    f = np.where(band[None, :], 1.3, 1.0)
    vel[0] = vel[0] + np.where(band[None, :], 0.5, 0.0)
    U[0] = primitive_to_conserved(rho * f, vel, p * f)
    U[1:] += 0.002 * rng.normal(size=(2, 4, ny, nx))
    return U


# ------------------------------------------------------------------------------ Example 3.11
def example_3_11(nx=960, ny=320, gamma=GAMMA):
    """Forward step: the uniform Mach 3 state (rho, u, v, p) = (1.4, 3, 0, 1) as averages,
    zero first moments, in every cell of the nx x ny mesh of [0, 3] x [0, 1]."""
    rho, u, v, p = 1.4, 3.0, 0.0, 1.0
    state = np.array([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])
    U = np.zeros((3, 4, ny, nx))
    U[0] = state[:, None, None]
    return U
