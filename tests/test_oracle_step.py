"""Forward-step boundaries (Example 3.11) in the oracle (CPU only).

oracle/step.py states the reading (position rule for stencil data at ghost and solid
positions, face rule for traces on faces between the fluid and anything else).  Pins:

* gas at rest stays at rest to round-off, next to the step's corner included;
* one step from the Mach 3 free stream changes only cells within reach of the step:
  the inflow, the outflow and the channel walls keep a uniform stream parallel to them
  exactly as it is (a wrong state at the inflow, a reversed u at the outflow or at a
  channel wall would change the cells along that side);
* walls let no mass or energy through: a pressure pulse at the step's corner, in gas at
  rest, leaves the totals over the fluid cells unchanged to round-off over three steps
  (the fluxes through the step's faces and the channel walls vanish; a missing momentum
  reversal at a wall would move mass through it);
* away from the corner each face of the step is the reflective wall of a rectangular
  mesh (pinned in tests/test_oracle_boundaries.py to the mirror-extended periodic
  problem): the operator next to the step's top face and next to its left face equals
  that of a rectangle with walls on the same lines, on the cells that only see that wall;
* the operator with its own flags passed back reproduces the free operator bit for bit,
  with troubled cells along every wall.
"""
import numpy as np
import pytest

import hweno_inputs as hi
from oracle import step
from oracle.scheme2d import Scheme2D

REST = (1.0, 0.0, 0.0, 1.0)


def scheme(nx=60, ny=20, ng=3, corner=step.STEP, inflow=step.INFLOW):
    return Scheme2D("euler", nx, ny, 0.0, 3.0, 0.0, 1.0, bc="step", ng_edge=ng, tc_mode="kxrcf",
                    step_corner=corner, inflow=inflow)


def uniform(o, state):
    U = np.zeros((3, 4, o.ny, o.nx))
    U[0] = step.conserved(state)[:, None, None]
    return U


def centres(o):
    xc = o.x0 + (np.arange(o.nx) + 0.5) * o.dx
    yc = o.y0 + (np.arange(o.ny) + 0.5) * o.dy
    return np.meshgrid(xc, yc)


def pulse(o, x, y, r, amp, vel=0.0):
    """Gas at rest (rho = 1, p = 1) with a smooth pressure pulse of relative height amp and
    a velocity (vel, vel / 2) of the same Gaussian shape (cell averages by 4 x 4 Gauss
    points, first moments zero)."""
    X, Y = centres(o)
    g, w = np.polynomial.legendre.leggauss(4)
    avg = np.zeros((4,) + X.shape)
    for a, wa in zip(g, w):
        for b, wb in zip(g, w):
            xx, yy = X + 0.5 * a * o.dx, Y + 0.5 * b * o.dy
            e = np.exp(-((xx - x) ** 2 + (yy - y) ** 2) / r ** 2)
            u, v, p = vel * e, 0.5 * vel * e, 1.0 + amp * e
            avg += 0.25 * wa * wb * np.stack([np.ones_like(u), u, v, p / 0.4 + 0.5 * (u * u + v * v)])
    U = np.zeros((3, 4, o.ny, o.nx))
    U[0] = avg
    return U


def test_rest_stays_at_rest():
    o = scheme(inflow=REST)
    U = uniform(o, REST)
    L, info = o.operator(U)
    assert np.abs(L).max() < 1e-12 * np.abs(U).max()
    assert info["T"].sum() == 0


def test_free_stream_changes_only_near_the_step():
    o = scheme(120, 40)
    si, sj = o.step_ij
    U = hi.example_3_11(120, 40)
    dt = o.cfl_dt(U, 0.6)
    U1, _ = o.rk3_step(U, dt)
    change = np.abs(U1 - U).max(axis=(0, 1)) / np.abs(U).max()
    jj, ii = np.meshgrid(np.arange(o.ny), np.arange(o.nx), indexing="ij")
    # a step reads nine cells in each direction (three stages of a three-cell reach)
    near = (ii >= si - 10) & (jj < sj + 10)
    assert change[~near].max() < 1e-14
    assert change[~o.solid & near].max() > 1e-3            # the flow meets the step
    # every side of the channel is among the unchanged cells
    far = ~near
    assert far[:, 0].all() and far[:, -1][sj + 10:].all() and far[-1].all() and far[0, :si - 10].all()
    # solid cells keep their values
    assert np.array_equal(U1[:, :, o.solid], U[:, :, o.solid])


def test_walls_let_no_mass_or_energy_through():
    # the corner in the middle of a 120 x 40 mesh, so that in three steps nothing reaches
    # the inflow or the outflow (60 cells away): the pulse (radius 2 cells) rounds to the
    # rest state from 13 cells on, and a step reads at most 12 cells
    o = scheme(120, 40, corner=(1.5, 0.5), inflow=REST)
    U = pulse(o, 1.5, 0.5, 0.05, 0.5, vel=0.5)
    fluid = ~o.solid
    m0, e0 = U[0, 0][fluid].sum(), U[0, 3][fluid].sum()
    for _ in range(3):
        U, infos = o.rk3_step(U, o.cfl_dt(U, 0.6))
    # nothing but round-off at the inflow and outflow columns
    U0 = pulse(o, 1.5, 0.5, 0.05, 0.5, vel=0.5)
    assert np.abs(U - U0)[..., [0, -1]].max() < 1e-14 * np.abs(U0).max()
    m1, e1 = U[0, 0][fluid].sum(), U[0, 3][fluid].sum()
    assert abs(m1 - m0) < 1e-13 * m0 and abs(e1 - e0) < 1e-13 * e0
    # momentum is not conserved (the walls push back)
    assert abs(U[0, 1][fluid].sum() - U0[0, 1][fluid].sum()) > 1e-6


def compare_with_rectangle(o, U, rect, sub, cells):
    """L of the step scheme o on U against that of the rectangle scheme rect on U's
    sub-array sub = (rows, cols), on the cells (rows, cols) of the sub-array."""
    ax, ay = o.alphas(U)
    L, info = o.operator(U, alphas=(ax, ay))
    Us = U[:, :, sub[0], sub[1]]
    Lr, infor = rect.operator(Us, alphas=(ax, ay))
    Ls = L[:, :, sub[0], sub[1]]
    a = Ls[:, :, cells[0], cells[1]]
    b = Lr[:, :, cells[0], cells[1]]
    assert np.abs(b).max() > 1.0
    assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max()
    assert np.array_equal(info["T"][sub[0], sub[1]][cells[0], cells[1]], infor["T"][cells[0], cells[1]])


def test_top_face_is_a_rectangular_wall():
    # 120 x 40 on [0, 3] x [0, 1]: step corner at cell (24, 8); a pulse on the top face at
    # x = 2, compared on the channel [1.5, 2.5] x [0.2, 1] (40 x 32 cells) with walls
    o = scheme(120, 40, inflow=REST)
    U = pulse(o, 2.0, 0.2, 0.05, 2.0, vel=-0.5)
    rect = Scheme2D("euler", 40, 32, 1.5, 2.5, 0.2, 1.0, bc="reflective", ng_edge=3, tc_mode="kxrcf")
    sub = (slice(8, 40), slice(60, 100))
    # cells more than three columns from the rectangle's side walls
    cells = (slice(0, 32), slice(4, 36))
    compare_with_rectangle(o, U, rect, sub, cells)


def test_left_face_is_a_rectangular_wall():
    # a taller step (corner at (0.6, 0.5): cell (24, 20)); a pulse on the left face at
    # y = 0.25, compared on [0.1, 0.6] x [0, 0.5] (20 x 20 cells) with walls
    o = scheme(120, 40, corner=(0.6, 0.5), inflow=REST)
    U = pulse(o, 0.6, 0.25, 0.05, 2.0, vel=0.5)
    rect = Scheme2D("euler", 20, 20, 0.1, 0.6, 0.0, 0.5, bc="reflective", ng_edge=3, tc_mode="kxrcf")
    sub = (slice(0, 20), slice(4, 24))
    # cells more than three from the rectangle's left side and its top side (which the
    # step's corner and the open channel replace)
    cells = (slice(0, 17), slice(4, 20))
    compare_with_rectangle(o, U, rect, sub, cells)


@pytest.mark.parametrize("ng", [2, 3])
def test_fixed_flags_reproduce_the_free_operator_step(ng):
    o = scheme(120, 40, ng=ng)
    U = hi.example_3_11(120, 40)
    t = 0.0
    for _ in range(12):
        dt = o.cfl_dt(U, 0.6)
        U, infos = o.rk3_step(U, dt, t=t)
        t += dt
    L, info = o.operator(U)
    T = info["T"].astype(bool)
    si, sj = o.step_ij
    assert T[:sj, si - 3:si].any()                         # along the step's left face
    L2, info2 = o.operator(U, T_fixed=T)
    assert np.array_equal(L, L2) and np.array_equal(info["limited"], info2["limited"])
    assert np.array_equal(info["H"], info2["H"])


def test_sources_of_stencil_positions_lie_within_two_cells():
    """Every position outside the fluid that a fluid cell's 3 x 3 stencil reads takes its
    values from a fluid cell at most two cells away in x and one in y (two in x only where a
    one-cell-wide step reaches the exit), over every corner the configuration admits on
    meshes up to 16 x 16.  The reverse mode's gathers look for a cell's mirror positions in
    the 5 x 5 window around it on this account."""
    worst = (0, 0)
    for nx in range(7, 17):
        for ny in range(7, 17):
            for sj in range(3, ny // 2 + 1):
                for si in range(sj, nx):
                    def fluid(i, j):
                        return 0 <= i < nx and 0 <= j < ny and not (i >= si and j < sj)
                    for i in range(-1, nx + 1):
                        for j in range(-1, ny + 1):
                            if fluid(i, j) or not any(fluid(i + a, j + b) for a in (-1, 0, 1)
                                                      for b in (-1, 0, 1)):
                                continue
                            x, y, *_, pres = step.source(i, j, nx, ny, si, sj)
                            if pres:
                                continue
                            assert fluid(x, y)
                            worst = (max(worst[0], abs(x - i)), max(worst[1], abs(y - j)))
    assert worst == (2, 1), worst
