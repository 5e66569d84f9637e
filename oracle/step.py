"""Forward-facing step (Example 3.11) boundary data (oracle; test infrastructure).

The problem: a Mach 3 flow, (rho, u, v, p) = (1.4, 3, 0, 1), enters a channel [0, 3] x [0, 1]
from the left; a step of height 0.2 stands 0.6 from the entrance and runs to the exit.
Walls (top and bottom of the channel, the step's two faces) reflect, the left side is an
inflow of the free-stream state and the right side an outflow.

On a uniform mesh of the rectangle whose faces include the step's corner, the cells inside
the step are solid: they belong to the mesh arrays but are never updated.  The paper gives
no boundary treatment on moments.  The reading:

* position rule -- everything a stencil reads at a position outside the fluid (a ghost
  beyond the rectangle or a solid cell) is taken from one fluid cell, its source: beyond
  the left side the prescribed free-stream moments (average = the state, first moments
  zero, never troubled); beyond the right side the even mirror (outflow); beyond the top
  and bottom the wall mirror (rho v reversed); a solid position is then mirrored across
  the step face it lies closer to -- the left face x = x_s (rho u reversed) or the top
  face y = y_s (rho v reversed) -- and across both (a point reflection through the
  corner) when it lies on the diagonal.  The source's flag, limited moments and values
  all come with it, with the first moment normal to each mirror negated and the normal
  momentum reversed at each wall mirror.
* face rule -- at a face between a fluid cell and a non-fluid position, the non-fluid
  side's trace at each Gauss point is the fluid cell's own trace there, with the normal
  momentum reversed at a wall (zero mass and energy flux through every wall) and as it
  is at the outflow; at the inflow side it is the free-stream state.  (Away from the
  step's corner the position rule gives the same traces; the face rule also fixes the
  two faces of the corner cell, which faces two walls.)
"""
import math

import numpy as np

GAMMA = 1.4
INFLOW = (1.4, 3.0, 0.0, 1.0)          # rho, u, v, p of the Mach 3 free stream
STEP = (0.6, 0.2)                      # the step's corner on [0, 3] x [0, 1]


def conserved(state, gamma=GAMMA):
    rho, u, v, p = state
    return np.array([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])


def corner_cells(x0, y0, dx, dy, step=STEP):
    """Cell indices (si, sj) of the step's corner: solid cells are i >= si and j < sj.
    The corner must lie on cell faces."""
    a, b = (step[0] - x0) / dx, (step[1] - y0) / dy
    si, sj = int(round(a)), int(round(b))
    if abs(a - si) > 1e-9 or abs(b - sj) > 1e-9:
        raise ValueError("the step's corner must lie on cell faces")
    return si, sj


def source(i, j, nx, ny, si, sj):
    """Position rule for the position (i, j) (cell indices, possibly outside the mesh):
    returns (i', j', sx, sy, fu, fv, prescribed), the fluid cell whose values the position
    takes, the factors of its x and y first moments (-1 for each mirror across a vertical
    or horizontal line) and of rho u and rho v (-1 for each wall that reverses them)."""
    if i < 0:
        return 0, min(max(j, 0), ny - 1), 1.0, 1.0, 1.0, 1.0, True
    sx = sy = fu = fv = 1.0
    if i >= nx:                         # outflow: the even mirror
        i, sx = 2 * nx - 1 - i, -1.0
    if j < 0:                           # bottom wall
        j, sy, fv = -1 - j, -1.0, -1.0
    elif j >= ny:                       # top wall
        j, sy, fv = 2 * ny - 1 - j, -1.0, -1.0
    if i >= si and j < sj:              # inside the step
        a, b = i - si, sj - 1 - j       # cells from the left face, from the top face
        if a <= b:
            i, sx, fu = 2 * si - 1 - i, -sx, -fu
        if b <= a:
            j, sy, fv = 2 * sj - 1 - j, -sy, -fv
    return i, j, sx, sy, fu, fv, False


def mach(state=INFLOW, gamma=GAMMA):
    rho, u, v, p = state
    return math.hypot(u, v) / math.sqrt(gamma * p / rho)
