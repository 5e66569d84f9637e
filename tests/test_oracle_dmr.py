"""Double Mach reflection boundaries (Example 3.10) in the oracle (CPU only).

* The exact cut-cell moments the prescribed ghost cells hold (oracle/dmr.py) are the
  limits of brute-force midpoint sums over each cell (error falling like 1/n with n^2
  samples), and take the closed-form values where the shock misses the cell or halves it.
* Away from the shock, the exact solution is uniform and the scheme must keep it so to
  round-off: one step from the exact initial state leaves every cell whose stencil (with
  the prescribed, wall and outflow ghosts around it) holds a single state unchanged.  This
  involves each boundary side: the inflow at x = 0 and the top side behind the shock
  (post-shock gas), the top side ahead of it and the wall at rest from x = 1/6 (gas at
  rest), and the outflow side.  A wrong state, side, sign or time in the boundary data
  breaks it.
* The shock moves at its exact speed: along the top row of cells, where the boundary data
  drive it, the density crosses the mean of its two states within one and a half cells of
  the exact shock position after ten steps.
(At these coarse meshes the first steps of the Mach 10 problem need the 3-point edge rule
and 96 rows: 24 or 48 rows with the 2-point rule produce negative pressure in the first
stage, with any boundary treatment.)
* The operator with its own flags passed back reproduces the free operator bit for bit.
"""
import math

import numpy as np
import pytest

import hweno_inputs as hi
from oracle import dmr
from oracle.scheme2d import NG, Scheme2D


def brute(xc, yc, h, t, n):
    s = (np.arange(n) + 0.5) / n - 0.5
    XI, ET = np.meshgrid(s, s)
    U = dmr.state_at(xc + h * XI, yc + h * ET, t)
    return np.stack([U.mean(axis=(1, 2)), (U * XI).mean(axis=(1, 2)), (U * ET).mean(axis=(1, 2))])


@pytest.mark.parametrize("cell", [(0.0005, 0.0, 0.3), (0.3, 0.012, -0.45), (0.99, 0.15, 0.1)])
def test_cut_cell_moments_are_the_limit_of_midpoint_sums(cell):
    yc, t, off = cell                 # a cell the shock line crosses, off cells from centre
    h = 1.0 / 480
    xc = dmr.shock_offset(t) + yc / math.sqrt(3.0) + off * h
    m = dmr.cell_moments(xc, yc, h, t)
    assert 0.0 < np.abs(m[1]).max()
    errs = [np.abs(brute(xc, yc, h, t, n) - m).max() / np.abs(m).max() for n in (100, 200, 400)]
    assert 0.0 < errs[0] < 1e-2
    assert errs[2] < errs[0] / 2.5, errs          # first-order convergence to the exact value


def test_cut_cell_moments_closed_forms():
    h = 0.01
    # entirely behind / ahead of the shock: the state itself, zero first moments
    assert np.array_equal(dmr.cell_moments(0.01, 0.5, h, 0.0), np.stack([dmr.U_POST, 0 * dmr.U_POST, 0 * dmr.U_POST]))
    assert np.array_equal(dmr.cell_moments(3.0, 0.5, h, 0.0), np.stack([dmr.U_PRE, 0 * dmr.U_PRE, 0 * dmr.U_PRE]))
    # the shock through the centre halves the cell (point symmetry): the mean of the states
    t = 0.05
    yc = 0.4
    xc = dmr.shock_offset(t) + yc / math.sqrt(3.0)
    m = dmr.cell_moments(xc, yc, h, t)
    assert np.allclose(m[0], 0.5 * (dmr.U_POST + dmr.U_PRE), rtol=1e-15)
    # the post-shock half lies left of the line: negative x moment, and the line's slope
    # (x - y/sqrt3 = c) puts it towards positive y
    assert (m[1][0] < 0.0) and (m[2][0] > 0.0)


def dmr_scheme(ny=96, ng=3):
    return Scheme2D("euler", 4 * ny, ny, 0.0, 4.0, 0.0, 1.0, bc="dmr", ng_edge=ng, tc_mode="kxrcf")


def test_uniform_regions_stay_exact_after_one_step():
    ny = 96
    h = 1.0 / ny
    o = dmr_scheme(ny)
    U0 = hi.example_3_10(4 * ny, ny)
    dt = o.cfl_dt(U0, 0.6)
    U1, _ = o.rk3_step(U0, dt, t=0.0)
    xc = (np.arange(4 * ny) + 0.5) * h
    yc = (np.arange(ny) + 0.5) * h
    X, Y = np.meshgrid(xc, yc)
    # A stage's operator at a cell reads cells up to three away (in both directions at
    # once), so a step's result up to nine.  Distance from the shock line in cells along x:
    # nine cells diagonally away cover 9 (1 + 1/sqrt3) < 15 of it, plus the shock's travel.
    dist = np.abs(X - Y / math.sqrt(3.0) - dmr.shock_offset(0.0)) / h
    far = dist > 15.0 + 20.0 * dt / math.sqrt(3.0) / h
    # the wall starts at x = 1/6 = 16 cells: the corner region is not uniform either
    far &= ~((X < 1.0 / 6 + 10 * h) & (Y < 10 * h))
    scale = np.abs(U0).reshape(3, 4, -1).max(axis=2)[:, :, None, None]
    change = np.abs(U1 - U0) / np.maximum(scale, 1e-300)
    assert change[:, :, far].max() < 1e-13
    # every side is represented among the unchanged cells
    assert far[:, 0].any() and far[-1, :].any() and far[0, -1] and far[-1, -1] and far[0, 60]


def test_shock_moves_at_its_exact_speed():
    ny = 96
    h = 1.0 / ny
    o = dmr_scheme(ny)
    U = hi.example_3_10(4 * ny, ny)
    t = 0.0
    for _ in range(10):
        dt = o.cfl_dt(U, 0.6)
        U, _ = o.rk3_step(U, dt, t=t)
        t += dt
    rho = U[0, 0, -1]                                # top row of cells
    xc = (np.arange(4 * ny) + 0.5) * h
    mid = 0.5 * (8.0 + 1.4)
    k = np.nonzero((rho[:-1] > mid) & (rho[1:] <= mid))[0][-1]
    x_num = xc[k] + h * (rho[k] - mid) / (rho[k] - rho[k + 1])
    x_exact = dmr.shock_offset(t) + (1.0 - 0.5 * h) / math.sqrt(3.0)
    assert abs(x_num - x_exact) < 1.5 * h, (x_num, x_exact, t)


def test_fixed_flags_reproduce_the_free_operator_dmr():
    ny = 96
    o = dmr_scheme(ny)
    U0 = hi.example_3_10(4 * ny, ny)
    U, _ = o.rk3_step(U0, o.cfl_dt(U0, 0.6), t=0.0)
    t = 0.01
    L, info = o.operator(U, t=t)
    T = info["T"].astype(bool)
    assert T[:3].any() and T[-3:].any()
    L2, info2 = o.operator(U, T_fixed=T, t=t)
    assert np.array_equal(L, L2) and np.array_equal(info["limited"], info2["limited"])
