"""How far two valid summation orders of the oracle's own arithmetic drift apart (CPU).

The scheme commutes with the reflection x -> -x (averages mirrored, first moments mirrored
and negated, the advection speed reversed), so running the oracle on the mirror image of
a problem and mirroring back evaluates the same mathematics with every stencil sum taken
in the opposite order.  On the 1D advection workload (N = 160, 800 steps of dt = 0.0025
to T = 2) the two runs differ by a few 1e-13 per stored array -- the round-off floor of
any second implementation, the GPU's included.  The per-array backstop of the GPU parity
tests (tests/parity.py) is set about fourteen times above this spread.
"""
import numpy as np

import hweno_inputs as hi
from oracle.physics import Equation
from oracle.scheme1d import Scheme1D

from parity import ARRAY_BACKSTOP, array_err


def mirror(U):
    M = U[:, :, ::-1].copy()
    M[1] *= -1.0
    return M


def test_mirror_image_spread_of_the_oracle():
    U0, _ = hi.advection_1d(0, 160)
    o = Scheme1D(Equation("advection", 1, adv=(1.0,)), 160, 0.0, 2.0, tc_mode="none")
    r = Scheme1D(Equation("advection", 1, adv=(-1.0,)), 160, 0.0, 2.0, tc_mode="none")
    A, _, _, _ = o.run(U0, nsteps=800, dt=0.0025)
    B, _, _, _ = r.run(mirror(U0), nsteps=800, dt=0.0025)
    spread = array_err(mirror(B), A)
    print(f"mirror-image spread after 800 steps: {spread:.3e}")
    assert 1e-14 < spread < 2e-12
    assert 5.0 * spread < ARRAY_BACKSTOP < 50.0 * spread
