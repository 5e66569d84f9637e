"""Shared parity helpers of the GPU tests: tolerances, error norms, the oracle's step with
given troubled flags, and the rounding-tie test for troubled-cell decisions.

Tolerances
* TOL: one operator evaluation, every stored array within max|gpu - oracle| / max|oracle|;
  after time stepping, the same bound per field, a field being a conserved component
  represented by its moments, i.e. the piecewise-linear function ubar + 12 vbar xi
  (+ 12 wbar eta), compared in the sup norm.
* ARRAY_BACKSTOP: each stored array after time stepping.  First moments are O(dx)
  quantities whose round-off is set by the averages; the oracle run on the mirror image
  of a problem (the same arithmetic in another summation order) differs from the oracle
  by up to 7.2e-13 per array after the 800 steps of the 1D advection workload
  (tests/test_oracle_spread.py), so the backstop is that spread times about 14.
"""
import numpy as np

from oracle import kxrcf
from oracle.scheme1d import Scheme1D

TOL = 1e-12
ARRAY_BACKSTOP = 1e-11


def array_err(a, b):
    """max over stored arrays of max|a-b| / max|b| (absolute when the array is zero)."""
    a = np.asarray(a).reshape(a.shape[0] * a.shape[1], -1)
    b = np.asarray(b).reshape(b.shape[0] * b.shape[1], -1)
    worst = 0.0
    for x, y in zip(a, b):
        scale = np.abs(y).max()
        e = np.abs(x - y).max() / (scale if scale > 0 else 1.0)
        worst = max(worst, e)
    return worst


def p1_field_err(a, b):
    """max over conserved components of the relative sup-norm error of the piecewise-linear
    field ubar + 12 vbar xi (+ 12 wbar eta) defined by the moments."""
    a, b = np.asarray(a), np.asarray(b)
    worst = 0.0
    for c in range(a.shape[1]):
        d = np.abs(a[0, c] - b[0, c]) + sum(6.0 * np.abs(a[m, c] - b[m, c]) for m in range(1, a.shape[0]))
        n = np.abs(b[0, c]) + sum(6.0 * np.abs(b[m, c]) for m in range(1, b.shape[0]))
        worst = max(worst, d.max() / n.max())
    return worst


def check_run(U, Uo, what=""):
    fe, ae = p1_field_err(U, Uo), array_err(U, Uo)
    print(f"{what}: field error {fe:.3e}, array error {ae:.3e}")
    assert fe < TOL, (what, fe)
    assert ae < ARRAY_BACKSTOP, (what, ae)


def rk3_with_flags(o, U, dt, Ts):
    """The oracle's TVD-RK3 step (eq. RK) with the troubled flags of each stage given.
    Returns (U^{n+1}, infos, the three stage inputs)."""
    L0, i0 = o.operator(U, T_fixed=Ts[0])
    W0 = i0["limited"]
    S1 = W0 + dt * L0
    L1, i1 = o.operator(S1, T_fixed=Ts[1])
    S2 = 0.75 * W0 + 0.25 * i1["limited"] + 0.25 * dt * L1
    L2, i2 = o.operator(S2, T_fixed=Ts[2])
    return W0 / 3.0 + 2.0 / 3.0 * i2["limited"] + 2.0 / 3.0 * dt * L2, [i0, i1, i2], [U, S1, S2]


TIE = 1e-12


def _decisions_1d(o, Up, k, comps, vel):
    """(troubled, near threshold) of padded cell k for indicator velocity vel."""
    fired = near = False
    for c in comps:
        a, m = Up[0, c], Up[1, c]
        num, den = kxrcf.indicator_margin_1d(a[k:k + 1], m[k:k + 1], a[k - 1:k], m[k - 1:k],
                                             a[k + 1:k + 2], m[k + 1:k + 2], np.array([vel]),
                                             o._cell_dx(np.array([k])))
        fired |= bool(vel != 0.0 and num[0] > den[0])
        near |= bool(vel != 0.0 and abs(num[0] - den[0]) <= TIE * den[0])
    return fired, near


def _decisions_2d(o, Up, j, i, comps, vx, vy):
    fired = near = False
    for c in comps:
        def at(dj, di):
            return tuple(Up[mm, c, j + dj:j + dj + 1, i + di:i + di + 1] for mm in range(3))
        num, den = kxrcf.indicator_margin_2d(at(0, 0), at(0, -1), at(0, 1), at(-1, 0), at(1, 0),
                                             np.array([[vx]]), np.array([[vy]]), o.dx, o.dy)
        inflow = vx != 0.0 or vy != 0.0
        fired |= bool(inflow and num.item() > den.item())
        near |= bool(inflow and abs(num.item() - den.item()) <= TIE * den.item())
    return fired, near


def is_tie(o, S, cell, t=0.0):
    """Whether the troubled-cell decision of cell (index, or (j, i) in 2D) on the stage
    input S is decided by rounding: some indicator variable sits at the threshold up to
    TIE, or the indicator velocity (a component of it in 2D) is zero up to TIE times the
    largest wave speed and the decision changes with its sign (the velocity only selects
    the inflow faces)."""
    comps = (0, o.eq.ncomp - 1) if o.eq.name == "euler" else (0,)
    Up = o.pad(S) if isinstance(o, Scheme1D) else o.pad(S, t)
    if isinstance(o, Scheme1D):
        k = cell + 3
        vel = float(o.eq.velocity(Up[0][:, k:k + 1], 0)[0])
        fired, near = _decisions_1d(o, Up, k, comps, vel)
        if near:
            return True
        if abs(vel) <= TIE * o.alpha(S):
            return len({_decisions_1d(o, Up, k, comps, v)[0] for v in (1.0, -1.0, 0.0)}) > 1
        return False
    j, i = cell[0] + 3, cell[1] + 3
    U0 = Up[0][:, j:j + 1, i:i + 1]
    vx, vy = float(o.eq.velocity(U0, 0).item()), float(o.eq.velocity(U0, 1).item())
    fired, near = _decisions_2d(o, Up, j, i, comps, vx, vy)
    if near:
        return True
    ax, ay = o.alphas(S)
    xs = (1.0, -1.0, 0.0) if abs(vx) <= TIE * ax else (vx,)
    ys = (1.0, -1.0, 0.0) if abs(vy) <= TIE * ay else (vy,)
    return len({_decisions_2d(o, Up, j, i, comps, a, b)[0] for a in xs for b in ys}) > 1


def differing_flags_are_ties(o, stages, gpu_T, times=None):
    """For each stage, the cells where the GPU's flags differ from the oracle's own
    decision on the stage input the GPU's flags lead to must all be rounding ties.
    times: the stage inputs' times (2D time-dependent boundary data).  Returns the number
    of such cells per stage."""
    counts = []
    for st in range(len(stages)):
        t = 0.0 if times is None else times[st]
        own = (o.operator(stages[st])[1]["T"] if isinstance(o, Scheme1D)
               else o.operator(stages[st], t=t)[1]["T"])
        cells = list(zip(*np.nonzero(gpu_T[st] != own)))
        for cell in cells:
            cell = int(cell[0]) if len(cell) == 1 else (int(cell[0]), int(cell[1]))
            assert is_tie(o, stages[st], cell, t), (st, cell)
        counts.append(len(cells))
    return counts
