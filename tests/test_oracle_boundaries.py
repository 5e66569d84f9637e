"""Boundary reading of the oracle (CPU only): one rule for transmissive and reflective
boundaries in one and two dimensions.

The paper defines no boundary treatment for the first moments.  The reading taken: a
ghost cell is the mirror image of the cell it faces in every respect -- its stored
moments (average copied, normal first moment negated; a wall also reverses the normal
momentum), its troubled flag, its limited moments and its traces on the boundary face.

* The troubled flags decide everything downstream of Step 1 / Step 4, so the operator
  with its own flags passed back in (the fixed-flag path the adjoint and the lockstep
  recomputation use) must reproduce the free operator bit for bit, on states whose
  troubled cells sit within three cells of every wall.
* Ghost flags are the mirror images of the flags of the inner cells, and the outermost
  ghost layer (which has a neighbour on one side only) is never flagged.
* A reflective wall is a true symmetry of the Euler equations, so the scheme on the walled
  mesh equals the periodic scheme on the mirror-extended mesh, with mirrored troubled sets
  (pinned in test_oracle_shock_suite.py for 1D; here for 2D walls in x, in y and in both
  directions, where the extension is the four-fold mirror image).
"""
import numpy as np
import pytest

import hweno_inputs as hi
from oracle.scheme1d import NG as NG1, Scheme1D
from oracle.scheme2d import NG as NG2, Scheme2D


def walls_state_1d(n=40, seed=0):
    """1D Euler data with jumps one and two cells from each end, flow towards the walls
    near both ends, and small seeded first moments."""
    x = (np.arange(n) + 0.5) / n
    rho = np.where(x < 2.04 / n, 1.0, np.where(x < 0.5, 0.3, np.where(x < 1 - 1.96 / n, 0.8, 0.2)))
    u = np.where(x < 0.5, 0.7, -0.6)
    p = np.where(x < 1.04 / n, 1.0, np.where(x < 1 - 0.96 / n, 0.4, 0.1))
    U = np.zeros((2, 3, n))
    U[0] = hi.primitive_to_conserved(rho, [u], p)
    U[1] = 1e-4 * np.random.default_rng(seed).normal(size=(3, n))
    return U


def walls_state_2d(n=24, seed=0):
    """2D Euler data with a frame of denser gas two cells wide along every wall, a
    diagonal jump, inflow from every wall and small seeded first moments."""
    xc = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(xc, xc)
    edge = (X < 2.0 / n) | (X > 1 - 2.0 / n) | (Y < 2.0 / n) | (Y > 1 - 2.0 / n)
    rho = 1.0 + 0.5 * edge + 0.3 * (X + Y > 1)
    u = 0.5 * np.where(X < 0.5, 1.0, -1.0)
    v = 0.4 * np.where(Y < 0.5, 1.0, -1.0)
    p = 1.0 + 0.4 * ((X < 1.0 / n) | (Y > 1 - 1.0 / n))
    U = np.zeros((3, 4, n, n))
    U[0] = hi.primitive_to_conserved(rho, [u, v], p)
    U[1:] = 1e-4 * np.random.default_rng(seed).normal(size=(2, 4, n, n))
    return U


@pytest.mark.parametrize("bc", ["periodic", "transmissive", "reflective"])
def test_fixed_flags_reproduce_the_free_operator_1d(bc):
    U = walls_state_1d()
    o = Scheme1D("euler", U.shape[-1], bc=bc, tc_mode="kxrcf")
    L, info = o.operator(U)
    T = info["T"].astype(bool)
    assert T[:3].any() and T[-3:].any(), np.nonzero(T)
    L2, info2 = o.operator(U, T_fixed=T)
    assert np.array_equal(L, L2)
    assert np.array_equal(info["limited"], info2["limited"])
    assert np.array_equal(info["H"], info2["H"])
    # the step built on the fixed flags is the free step as well
    dt = o.cfl_dt(U, 0.6)
    A, ia = o.rk3_step(U, dt)
    L0, j0 = o.operator(U, T_fixed=ia[0]["T"])
    W0 = j0["limited"]
    L1, j1 = o.operator(W0 + dt * L0, T_fixed=ia[1]["T"])
    L2_, j2 = o.operator(0.75 * W0 + 0.25 * j1["limited"] + 0.25 * dt * L1, T_fixed=ia[2]["T"])
    B = W0 / 3.0 + 2.0 / 3.0 * j2["limited"] + 2.0 / 3.0 * dt * L2_
    assert np.array_equal(A, B)


@pytest.mark.parametrize("bc", ["periodic", "transmissive", "reflective", ("reflective", "transmissive")])
def test_fixed_flags_reproduce_the_free_operator_2d(bc):
    U = walls_state_2d()
    n = U.shape[-1]
    o = Scheme2D("euler", n, n, bc=bc, ng_edge=2, tc_mode="kxrcf")
    L, info = o.operator(U)
    T = info["T"].astype(bool)
    for side in (T[:3], T[-3:], T[:, :3], T[:, -3:]):
        assert side.any()
    L2, info2 = o.operator(U, T_fixed=T)
    assert np.array_equal(L, L2)
    assert np.array_equal(info["limited"], info2["limited"])
    assert np.array_equal(info["H"], info2["H"])


@pytest.mark.parametrize("bc", ["transmissive", "reflective"])
def test_ghost_flags_and_limited_moments_are_mirror_images_1d(bc):
    U = walls_state_1d()
    n = U.shape[-1]
    o = Scheme1D("euler", n, bc=bc, tc_mode="kxrcf")
    Up = o.pad(U)
    L, T, H, Vt = o.operator_padded(Up, o.alpha(U), mirror=True)
    sm = np.array([-1.0, 1.0 if bc == "reflective" else -1.0, -1.0])
    for g in range(1, NG1):
        assert T[NG1 - g] == T[NG1 + g - 1] and T[NG1 + n - 1 + g] == T[NG1 + n - g]
        assert np.array_equal(Vt[:, NG1 - g], sm * Vt[:, NG1 + g - 1])
        assert np.array_equal(Vt[:, NG1 + n - 1 + g], sm * Vt[:, NG1 + n - g])
    assert not T[0] and not T[-1]
    # the mirrored cells next to the walls are troubled, so the rule is exercised
    assert T[NG1] or T[NG1 + 1]


def test_transmissive_boundary_flux_has_no_jump_term_1d():
    """With the boundary face carrying one state on both sides, the Lax-Friedrichs flux
    there is the physical flux of the inner cell's trace, whatever the speed alpha: the
    average's right-hand side of the cell next to each wall depends on alpha only through
    its inner face."""
    U = walls_state_1d()
    n = U.shape[-1]
    o = Scheme1D("euler", n, bc="transmissive", tc_mode="kxrcf")
    a = o.alpha(U)
    L1, _ = o.operator(U, alpha=a)
    L2, _ = o.operator(U, alpha=2.0 * a)
    # cell 0: doubling alpha adds (alpha/2) (u^+ - u^-)/dx from its inner face only
    Up = o.pad(U)
    _, T, H, Vt = o.operator_padded(Up, a, mirror=True)
    left, right = o._traces(Up, Vt, H, np.arange(NG1 - 1, NG1 + n + 1))
    scale = np.abs(L1[0]).max()
    for cell, (up, um) in ((0, (left[:, 2], right[:, 1])), (n - 1, (left[:, n], right[:, n - 1]))):
        sgn = 1.0 if cell == 0 else -1.0        # the inner face is the right / left face
        expect = sgn * 0.5 * a * (up - um) / o.dx
        got = L2[0, :, cell] - L1[0, :, cell]
        assert np.abs(got - expect).max() <= 1e-12 * scale, (cell, got, expect)
        assert np.abs(expect).max() > 1e-6 * scale   # the inner face does have a jump


def wall_state_2d(n=16, seed=3):
    """2D Euler data with an oblique density and pressure jump, a velocity field that is
    not symmetric about any wall, and small seeded first moments."""
    xc = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(xc, xc)
    front = X + 0.7 * Y < 0.6
    rho = 1.0 + 0.5 * front
    u = 0.3 * np.sin(3.0 * X) + 0.1
    v = -0.2 * np.cos(2.0 * Y) + 0.1
    p = 1.0 + 0.8 * front
    U = np.zeros((3, 4, n, n))
    U[0] = hi.primitive_to_conserved(rho, [u, v], p)
    U[1:] = 0.01 * np.random.default_rng(seed).normal(size=(2, 4, n, n))
    return U


def mirror_extend_2d(U, axis):
    """The state on the doubled domain whose second half is U and whose first half is its
    mirror image across the low wall of the given axis (0: x, 1: y): averages and
    tangential moments even, normal moments odd, the normal momentum reversed."""
    ax = -1 if axis == 0 else -2
    M = np.concatenate([np.flip(U, axis=ax), U], axis=ax).copy()
    n = U.shape[ax]
    half = (slice(None), slice(None)) + ((slice(None), slice(0, n)) if axis == 0 else (slice(0, n), slice(None)))
    sign = np.ones((3, 4))
    sign[1 + axis, :] *= -1.0      # the normal first moment
    sign[:, 1 + axis] *= -1.0      # the normal momentum
    M[half] *= sign[:, :, None, None]
    return M


@pytest.mark.parametrize("walls", ["x", "y", "xy"])
def test_reflective_walls_equal_the_mirror_extended_periodic_problem_2d(walls):
    n = 16
    U = wall_state_2d(n)
    bc = ("reflective" if "x" in walls else "periodic", "reflective" if "y" in walls else "periodic")
    o = Scheme2D("euler", n, n, bc=bc, ng_edge=2, tc_mode="kxrcf")
    M = U
    nxp, nyp, x0, y0 = n, n, 0.0, 0.0
    if "x" in walls:
        M, nxp, x0 = mirror_extend_2d(M, 0), 2 * n, -1.0
    if "y" in walls:
        M, nyp, y0 = mirror_extend_2d(M, 1), 2 * n, -1.0
    p = Scheme2D("euler", nxp, nyp, x0, 1.0, y0, 1.0, bc="periodic", ng_edge=2, tc_mode="kxrcf")
    sx = slice(nxp - n, nxp)
    sy = slice(nyp - n, nyp)
    dt = 0.5 * o.cfl_dt(U, 0.6)
    A, B = U, M
    flagged = 0
    for k in range(6):
        A, ia = o.rk3_step(A, dt)
        B, ib = p.rk3_step(B, dt)
        assert np.abs(A - B[:, :, sy, sx]).max() <= 1e-13 * np.abs(A).max(), k
        for st in range(3):
            Tp = ib[st]["T"]
            assert np.array_equal(ia[st]["T"], Tp[sy, sx]), (k, st)
            if "x" in walls:
                assert np.array_equal(ia[st]["T"][:, ::-1], Tp[sy, :n]), (k, st)
            if "y" in walls:
                assert np.array_equal(ia[st]["T"][::-1, :], Tp[:n, sx]), (k, st)
            flagged += int(ia[st]["T"].sum())
    assert flagged > 0
