"""Pins of the KXRCF troubled-cell indicator (oracle/kxrcf.py; CPU only).

The paper names the indicator (Step 1, Step 4, Remarks 1 and 3) but prints no formula;
the reading is Krivodonova et al.'s form on the P1 polynomial u_K = ubar + 12 vbar xi
(+ 12 wbar eta) with k = 1.  What its mathematics fixes, independently of any code:

* on the cell moments of smooth data (exact projections) the jump of the P1 traces
  across a face is O(h^3) -- the projection errors of the two cells agree to leading
  order at their common face, where the even second Legendre polynomial takes the same
  value from both sides -- and the normalisation h^{(k+1)/2} |dK^-| |u_K| is O(h), so
  I_K falls like h^2 under refinement; a wrong trace factor (jump O(h), I_K = O(1)) or
  normalisation exponent (k = 2: order 1.5) breaks this;
* across a jump of size J the numerator stays J, so I_K grows like 1/h; for a jump from
  1 to 2 on the inflow face of a cell with zero first moment, I_K = 1/dx exactly in 1D and
  1/(h |u_K|) with h = half the cell diagonal in 2D;
* only inflow faces count: a jump on a cell's outflow face alone raises no flag there,
  and reversing the velocity moves the flag to the other side of the jump;
* for Euler a cell is troubled when the density or the energy indicator fires;
* at exactly I_K = 1 the cell is not troubled (strict inequality).
"""
import numpy as np
import pytest

import hweno_inputs as hi
from oracle import kxrcf
from oracle.physics import Equation
from oracle.scheme1d import Scheme1D
from oracle.scheme2d import Scheme2D


def ratio_1d(U, vel, dx):
    """I_K of every interior cell of a periodic 1D scalar state (2, 1, n)."""
    ub, vb = U[0, 0], U[1, 0]
    num, den = kxrcf.indicator_margin_1d(ub, vb, np.roll(ub, 1), np.roll(vb, 1), np.roll(ub, -1),
                                         np.roll(vb, -1), np.full_like(ub, vel), dx)
    return num / den


def ratio_2d(U, velx, vely, dx, dy):
    def cell(dj, di):
        return tuple(np.roll(np.roll(U[m, 0], -dj, axis=0), -di, axis=1) for m in range(3))
    one = np.ones_like(U[0, 0])
    num, den = kxrcf.indicator_margin_2d(cell(0, 0), cell(0, -1), cell(0, 1), cell(-1, 0), cell(1, 0),
                                         velx * one, vely * one, dx, dy)
    return num / den


def smooth_1d(n):
    return np.stack(hi.project_1d(lambda x: np.array([1.5 + np.sin(2 * np.pi * x)]), 0.0, 1.0, n))


def smooth_2d(n):
    f = lambda x, y: np.array([1.5 + np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y)])
    return np.stack(hi.project_2d(f, 0.0, 1.0, 0.0, 1.0, n, n, nq=6))


def test_smooth_indicator_falls_like_h_squared_1d():
    ns = [40, 80, 160, 320]
    worst = [ratio_1d(smooth_1d(n), 1.0, 1.0 / n).max() for n in ns]
    orders = np.log2(np.array(worst[:-1]) / np.array(worst[1:]))
    assert np.all(np.abs(orders - 2.0) < 0.05), (worst, orders)
    assert worst[0] < 1.0    # smooth data: no flag already on the coarsest mesh


def test_smooth_indicator_falls_like_h_squared_2d():
    ns = [16, 32, 64, 128]
    worst = [ratio_2d(smooth_2d(n), 0.7, 0.4, 1.0 / n, 1.0 / n).max() for n in ns]
    orders = np.log2(np.array(worst[:-1]) / np.array(worst[1:]))
    assert np.all(np.abs(orders - 2.0) < 0.1), (worst, orders)


def step_1d(n, xj=0.5):
    x = (np.arange(n) + 0.5) / n
    U = np.zeros((2, 1, n))
    U[0, 0] = np.where(x < xj, 1.0, 2.0)
    return U


@pytest.mark.parametrize("n", [20, 40, 80])
def test_jump_indicator_grows_like_inverse_h_1d(n):
    U = step_1d(n)
    r = ratio_1d(U, 1.0, 1.0 / n)
    j = n // 2                       # first cell right of the jump: inflow face on the jump
    assert r[j] == pytest.approx(n, rel=1e-14)      # I_K = 1/dx exactly
    others = np.delete(r, [j, 0])    # cell 0 sees the periodic wrap's jump from 2 to 1
    assert np.all(others == 0.0)
    o = Scheme1D(Equation("advection", 1, adv=(1.0,)), n, 0.0, 1.0, tc_mode="kxrcf")
    _, info = o.operator(U)
    assert set(np.nonzero(info["T"])[0]) == {0, j}


def test_jump_indicator_closed_form_2d():
    n = 32
    dx = dy = 1.0 / n
    xc = (np.arange(n) + 0.5) / n
    X, _ = np.meshgrid(xc, xc)
    U = np.zeros((3, 1, n, n))
    U[0, 0] = np.where(X < 0.5, 1.0, 2.0)
    r = ratio_2d(U, 1.0, 0.0, dx, dy)
    h = 0.5 * np.hypot(dx, dy)
    assert np.allclose(r[:, n // 2], 1.0 / (h * 2.0), rtol=1e-14)
    assert np.all(r[:, 1:n // 2] == 0.0) and np.all(r[:, n // 2 + 1:] == 0.0)
    # a diagonal velocity adds the bottom face, with zero jump: the numerator keeps the
    # left face's dy J, the denominator gains the bottom face's length dx
    r2 = ratio_2d(U, 1.0, 1.0, dx, dy)
    assert np.allclose(r2[:, n // 2], dy * 1.0 / (h * (dx + dy) * 2.0), rtol=1e-14)
    o = Scheme2D(Equation("advection", 2, adv=(1.0, 0.0)), n, n, tc_mode="kxrcf", ng_edge=3)
    _, info = o.operator(U)
    assert set(np.nonzero(info["T"].any(axis=0))[0]) == {0, n // 2}


def test_outflow_jump_raises_no_flag():
    n = 40
    U = step_1d(n)
    j = n // 2
    r_pos = ratio_1d(U, 1.0, 1.0 / n)
    r_neg = ratio_1d(U, -1.0, 1.0 / n)
    # velocity > 0: the cell left of the jump has it on its right (outflow) face
    assert r_pos[j - 1] == 0.0 and r_pos[j] > 1.0
    # velocity < 0: the flag moves to the cell left of the jump
    assert r_neg[j] == 0.0 and r_neg[j - 1] > 1.0
    # zero velocity: no inflow face anywhere, so no flag
    assert not kxrcf.troubled_1d(U[0, 0][1:-1], U[1, 0][1:-1], U[0, 0][:-2], U[1, 0][:-2],
                                 U[0, 0][2:], U[1, 0][2:], np.zeros(n - 2), 1.0 / n).any()


def euler_pair(rho, u, p):
    """Two-state 1D Euler data (left state for x < 1/2), zero first moments."""
    n = 20
    x = (np.arange(n) + 0.5) / n
    prim = [np.where(x < 0.5, a, b) for a, b in (rho, u, p)]
    U = np.zeros((2, 3, n))
    U[0] = hi.primitive_to_conserved(prim[0], [prim[1]], prim[2])
    return U


def indicators_at(U, i):
    """(density fires, energy fires) for cell i of a transmissive 1D Euler state."""
    o = Scheme1D("euler", U.shape[-1], bc="transmissive", tc_mode="kxrcf")
    Up = o.pad(U)
    k = i + 3
    vel = o.eq.velocity(Up[0][:, k:k + 1], 0)
    fires = []
    for c in (0, 2):
        t = kxrcf.troubled_1d(Up[0, c, k:k + 1], Up[1, c, k:k + 1], Up[0, c, k - 1:k], Up[1, c, k - 1:k],
                              Up[0, c, k + 1:k + 2], Up[1, c, k + 1:k + 2], vel, o.dx)
        fires.append(bool(t[0]))
    _, info = o.operator(U)
    return tuple(fires), bool(info["T"][i])


def test_euler_fires_on_density_or_energy():
    j = 10
    # contact at almost no speed: density jumps, energy jumps by rho u^2/2 only
    (rho_f, e_f), T = indicators_at(euler_pair((1.0, 0.2), (1e-3, 1e-3), (1.0, 1.0)), j)
    assert rho_f and not e_f and T
    # pressure jump at constant density: only the energy indicator fires
    (rho_f, e_f), T = indicators_at(euler_pair((1.0, 1.0), (0.5, 0.5), (1.0, 0.3)), j)
    assert not rho_f and e_f and T
    # both constant: no flag
    (rho_f, e_f), T = indicators_at(euler_pair((1.0, 1.0), (0.5, 0.5), (1.0, 1.0)), j)
    assert not rho_f and not e_f and not T


def test_threshold_is_strict():
    dx = 0.25                        # den = (dx/2) * 1 * |ubar| = 0.125 for ubar = 1
    ub, vb = np.array([1.0]), np.array([0.0])
    at = kxrcf.troubled_1d(ub, vb, np.array([0.875]), vb, ub, vb, np.array([1.0]), dx)
    above = kxrcf.troubled_1d(ub, vb, np.array([0.875 - 2.0 ** -50]), vb, ub, vb, np.array([1.0]), dx)
    num, den = kxrcf.indicator_margin_1d(ub, vb, np.array([0.875]), vb, ub, vb, np.array([1.0]), dx)
    assert num[0] == den[0] == 0.125
    assert not at[0] and above[0]
