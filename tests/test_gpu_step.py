"""GPU parity on the forward-facing step (Example 3.11): the HIP library's inflow, outflow,
wall and step boundaries against the oracle's (tests/test_oracle_step.py pins the oracle).

* Operator: 120 x 40 mesh of [0, 3] x [0, 1] (the paper's 960 x 320 at an eighth of the
  resolution), both edge rules, the paper's step and a taller one further downstream,
  from the free stream and from the oracle's state after fifteen steps: L, the limited
  state, flags and hybrid masks on the whole mesh (solid cells: zero, the stored state, no
  flags).
* Lockstep: ten steps, each started on the GPU from the oracle's state; flags of every
  stage identical except proven rounding ties (tests/parity.py), 1e-12 per field; the
  solid cells keep their values bit for bit.
* Full size: 960 x 320 to T = 4 on the GPU (3-point edge rule, CFL 0.6): finite, positive
  density and pressure, the free stream still entering at the left; and one operator
  evaluation of the final state against the oracle on the whole mesh.
"""
import numpy as np
import pytest

import hweno_inputs as hi
from oracle.scheme2d import Scheme2D

from parity import TOL, array_err, differing_flags_are_ties, p1_field_err, rk3_with_flags

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hw():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2002_08816_amd as hw
    return hw


def pair(hw, nx, ny, ng, corner=(0.6, 0.2)):
    s = hw.Solver(2, nx, ny, domain=(0.0, 3.0, 0.0, 1.0), eq="euler", ng_edge=ng, tc_mode="kxrcf",
                  bc="step", step=corner)
    o = Scheme2D("euler", nx, ny, 0.0, 3.0, 0.0, 1.0, bc="step", ng_edge=ng, tc_mode="kxrcf",
                 step_corner=corner)
    return s, o


def evolved(o, U, nsteps):
    for _ in range(nsteps):
        U, _ = o.rk3_step(U, o.cfl_dt(U, 0.6))
    return U


def check_operator(s, o, V):
    s.set_state(V)
    L, W = s.apply_operator(V)
    T, H = s.flags(0)
    Lo, info = o.operator(V)
    if differing_flags_are_ties(o, [V], [T])[0]:
        Lo, info = o.operator(V, T_fixed=T)
    assert np.array_equal(T, info["T"]) and np.array_equal(H, info["H"])
    assert not T[o.solid].any() and not H[o.solid].any()
    assert np.array_equal(L[:, :, o.solid], 0 * L[:, :, o.solid])
    assert np.array_equal(W[:, :, o.solid], V[:, :, o.solid])
    print(f"troubled {int(T.sum())}, hybrid {int(H.sum())}: L {array_err(L, Lo):.3e}, "
          f"limited {array_err(W, info['limited']):.3e}")
    assert array_err(L, Lo) < TOL
    assert array_err(W, info["limited"]) < TOL
    return T


@pytest.mark.parametrize("ng", [2, 3])
@pytest.mark.parametrize("corner", [(0.6, 0.2), (1.5, 0.5)])
def test_step_operator(hw, ng, corner):
    nx, ny = 120, 40
    s, o = pair(hw, nx, ny, ng, corner)
    s.flag_export(True)
    # the evolved state comes from the 3-point edge rule for both edge rules
    o3 = o if ng == 3 else Scheme2D("euler", nx, ny, 0.0, 3.0, 0.0, 1.0, bc="step", ng_edge=3,
                                    tc_mode="kxrcf", step_corner=corner)
    U0 = hi.example_3_11(nx, ny)
    U1 = evolved(o3, U0, 15)
    check_operator(s, o, U0)
    T = check_operator(s, o, U1)
    assert T.sum() > 0
    s.close()


def test_step_lockstep(hw):
    nx, ny = 120, 40
    s, o = pair(hw, nx, ny, 3)
    s.flag_export(True)
    U = evolved(o, hi.example_3_11(nx, ny), 15)
    worst, ties = 0.0, 0
    for k in range(10):
        dt = o.cfl_dt(U, 0.6)
        s.set_state(U)
        s.step(dt)
        G, _ = s.get_state()
        flags = [s.flags(st) for st in range(3)]
        ref, infos = o.rk3_step(U, dt)
        if any(not np.array_equal(flags[st][0], infos[st]["T"]) for st in range(3)):
            Ts = [f[0] for f in flags]
            ref, infos, stages = rk3_with_flags(o, U, dt, Ts)
            ties += sum(differing_flags_are_ties(o, stages, Ts))
        for st in range(3):
            assert np.array_equal(flags[st][0], infos[st]["T"]), (k, st)
            assert np.array_equal(flags[st][1], infos[st]["H"]), (k, st)
        assert np.array_equal(G[:, :, o.solid], U[:, :, o.solid])
        e = p1_field_err(G, ref)
        worst = max(worst, e)
        assert e < TOL, (k, e)
        U = ref
    print(f"step lockstep: worst field error {worst:.3e}, rounding ties {ties}")
    s.close()


def test_step_full_size(hw):
    nx, ny, T = 960, 320, 4.0
    s, o = pair(hw, nx, ny, 3)
    U0 = hi.example_3_11(nx, ny)
    s.set_state(U0)
    steps, t = s.run(T)
    U, t = s.get_state()
    assert abs(t - T) < 1e-12 and steps > 5000
    fluid = ~o.solid
    rho = U[0, 0]
    p = 0.4 * (U[0, 3] - 0.5 * (U[0, 1] ** 2 + U[0, 2] ** 2) / rho)
    assert np.isfinite(U).all() and rho[fluid].min() > 0.0 and p[fluid].min() > 0.0
    assert np.array_equal(U[:, :, o.solid], U0[:, :, o.solid])
    # the supersonic inflow: the first column still holds the free stream's density
    assert np.abs(rho[:, 0] - 1.4).max() < 1e-6
    print(f"forward step 960x320: {steps} steps to T = {T}; density in "
          f"[{rho[fluid].min():.3f}, {rho[fluid].max():.3f}]")
    # one operator evaluation of the final state on the whole mesh
    s.flag_export(True)
    check_operator(s, o, U)
    s.close()
