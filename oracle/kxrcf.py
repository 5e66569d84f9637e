"""KXRCF troubled-cell indicator (oracle; test infrastructure).

The paper names the indicator of Krivodonova et al. (Step 1, Step 4, Remarks 1 and 3) but
defers its formula to other work.  Reading adopted here (Krivodonova et al.'s published
form applied to the P1 polynomial that a cell's moments define):

* P1 polynomial of cell K in reference coordinates: u_K = ubar + 12 vbar xi (+ 12 wbar eta);
  its mean trace on the left/right face is ubar -/+ 6 vbar, on the bottom/top face
  ubar -/+ 6 wbar.
* inflow faces: the velocity (f'(u), g'(u) for a scalar law; the fluid velocity for
  Euler) is taken at the cell average; a face is inflow when velocity . n_e < 0.
* I_K = | sum_{inflow e} |e| (m_e(u_K) - m_e(u_nb)) |
        / ( h^{(k+1)/2} |dK^-| max_K |u_K| ),  k = 1, h = half the cell diameter,
  |e| = face length (1 per face in 1D), |dK^-| = total inflow face length,
  max_K |u_K| = |ubar| + 6|vbar| (+ 6|wbar|).
* troubled iff numerator > denominator (no division; a cell with no inflow face is
  never troubled).  For Euler the indicator runs on density and on energy; a cell is
  troubled when either fires.

Parity unpinned: the constants of this reading are not fixed by the paper, so only the
qualitative facts are pinned (smooth data raises no flag; a jump raises flags at the
jump), and GPU results are compared against this function for identical flags.
"""
import numpy as np


def indicator_margin_1d(ub, vb, ub_l, vb_l, ub_r, vb_r, vel, dx):
    """Returns (numerator, denominator) of the 1D indicator for arrays of cells.

    ub, vb: average and first moment of the cell; *_l / *_r of its left/right neighbour;
    vel: indicator velocity at the cell average."""
    h = 0.5 * dx
    left_in = vel > 0.0     # left face normal -1: inflow iff vel > 0
    right_in = vel < 0.0    # right face normal +1: inflow iff vel < 0
    jump_l = (ub - 6.0 * vb) - (ub_l + 6.0 * vb_l)
    jump_r = (ub + 6.0 * vb) - (ub_r - 6.0 * vb_r)
    num = np.abs(np.where(left_in, jump_l, 0.0) + np.where(right_in, jump_r, 0.0))
    length = np.where(left_in, 1.0, 0.0) + np.where(right_in, 1.0, 0.0)
    norm = np.abs(ub) + 6.0 * np.abs(vb)
    den = h * length * norm
    return num, den


def troubled_1d(ub, vb, ub_l, vb_l, ub_r, vb_r, vel, dx):
    num, den = indicator_margin_1d(ub, vb, ub_l, vb_l, ub_r, vb_r, vel, dx)
    has_inflow = (vel != 0.0)
    return has_inflow & (num > den)


def indicator_margin_2d(c, l, r, b, t, velx, vely, dx, dy):
    """Returns (numerator, denominator) of the 2D indicator.

    c, l, r, b, t: tuples (ubar, vbar, wbar) of the cell and its left, right, bottom, top
    neighbours; velx, vely: indicator velocity at the cell average."""
    ub, vb, wb = c
    h = 0.5 * np.sqrt(dx * dx + dy * dy)
    l_in = velx > 0.0
    r_in = velx < 0.0
    b_in = vely > 0.0
    t_in = vely < 0.0
    jl = (ub - 6.0 * vb) - (l[0] + 6.0 * l[1])
    jr = (ub + 6.0 * vb) - (r[0] - 6.0 * r[1])
    jb = (ub - 6.0 * wb) - (b[0] + 6.0 * b[2])
    jt = (ub + 6.0 * wb) - (t[0] - 6.0 * t[2])
    s = (np.where(l_in, dy * jl, 0.0) + np.where(r_in, dy * jr, 0.0)
         + np.where(b_in, dx * jb, 0.0) + np.where(t_in, dx * jt, 0.0))
    num = np.abs(s)
    length = (np.where(l_in, dy, 0.0) + np.where(r_in, dy, 0.0)
              + np.where(b_in, dx, 0.0) + np.where(t_in, dx, 0.0))
    norm = np.abs(ub) + 6.0 * np.abs(vb) + 6.0 * np.abs(wb)
    den = h * length * norm
    return num, den


def troubled_2d(c, l, r, b, t, velx, vely, dx, dy):
    num, den = indicator_margin_2d(c, l, r, b, t, velx, vely, dx, dy)
    has_inflow = (velx != 0.0) | (vely != 0.0)
    return has_inflow & (num > den)
