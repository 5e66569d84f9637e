"""GPU parity on the double Mach reflection problem (Example 3.10): the HIP library's
prescribed, wall and outflow boundaries against the oracle's (tests/test_oracle_dmr.py pins
the oracle).

* Operator: 384 x 96 mesh of [0, 4] x [0, 1] (the paper's 1920 x 480 at a fifth of the
  resolution), both edge rules, from the exact initial state at t = 0 and from the oracle's
  state after three steps (3-point edge rule) at its time: L, the limited state, flags
  and hybrid masks; also 360 x 90, whose last row and column of 16 x 16 tiles are partial
  (tile positions beyond the two ghost layers, in the padding).
* Lockstep: ten steps, each started on the GPU from the oracle's state and time; flags of
  every stage identical except proven rounding ties (tests/parity.py), 1e-12 per field.
* Full size: 1920 x 480 to T = 0.2 on the GPU (CFL 0.6): finite, positive density and
  pressure; the shock along the top row within two cells of its exact position; and one
  operator evaluation of the final state against the oracle on the whole mesh.
"""
import math

import numpy as np
import pytest

import hweno_inputs as hi
from oracle import dmr
from oracle.scheme2d import Scheme2D

from parity import TOL, array_err, differing_flags_are_ties, p1_field_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hw():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2002_08816_amd as hw
    return hw


def pair(hw, ny, ng):
    kw = dict(domain=(0.0, 4.0, 0.0, 1.0), eq="euler", ng_edge=ng, tc_mode="kxrcf", bc="dmr")
    s = hw.Solver(2, 4 * ny, ny, **kw)
    o = Scheme2D("euler", 4 * ny, ny, 0.0, 4.0, 0.0, 1.0, bc="dmr", ng_edge=ng, tc_mode="kxrcf")
    return s, o


@pytest.mark.parametrize("ng, ny", [(2, 96), (3, 96), (3, 90)])
def test_dmr_operator(hw, ng, ny):
    s, o = pair(hw, ny, ng)
    s.flag_export(True)
    U = hi.example_3_10(4 * ny, ny)
    # the evolved state comes from the 3-point edge rule: at this resolution the first
    # steps of the Mach 10 problem with the 2-point rule lose positivity
    o3 = o if ng == 3 else Scheme2D("euler", 4 * ny, ny, 0.0, 4.0, 0.0, 1.0, bc="dmr", ng_edge=3, tc_mode="kxrcf")
    Uo, t = U, 0.0
    for k in range(3):
        dt = o3.cfl_dt(Uo, 0.6)
        Uo, _ = o3.rk3_step(Uo, dt, t=t)
        t += dt
    for V, tv in ((U, 0.0), (Uo, t)):
        s.set_state(V)
        s.set_time(tv)
        L, W = s.apply_operator(V)
        T, H = s.flags(0)
        Lo, info = o.operator(V, t=tv)
        if differing_flags_are_ties(o, [V], [T], [tv])[0]:
            Lo, info = o.operator(V, T_fixed=T, t=tv)
        assert np.array_equal(T, info["T"]) and np.array_equal(H, info["H"])
        assert T.sum() > 0
        print(f"t = {tv:.5f}: L {array_err(L, Lo):.3e}, limited {array_err(W, info['limited']):.3e}")
        assert array_err(L, Lo) < TOL
        assert array_err(W, info["limited"]) < TOL
    s.close()


def test_dmr_lockstep(hw):
    ny = 96
    s, o = pair(hw, ny, 3)
    s.flag_export(True)
    U, t, worst, ties = hi.example_3_10(4 * ny, ny), 0.0, 0.0, 0
    for k in range(10):
        dt = o.cfl_dt(U, 0.6)
        s.set_state(U)
        s.set_time(t)
        s.step(dt)
        G, tg = s.get_state()
        assert abs(tg - (t + dt)) <= 1e-15 * (t + dt)
        flags = [s.flags(st) for st in range(3)]
        ref, infos = o.rk3_step(U, dt, t=t)
        if any(not np.array_equal(flags[st][0], infos[st]["T"]) for st in range(3)):
            Ts = [f[0] for f in flags]
            ref, infos, stages = dmr_rk3_with_flags(o, U, dt, t, Ts)
            ties += sum(differing_flags_are_ties(o, stages, Ts, [t, t + dt, t + 0.5 * dt]))
        for st in range(3):
            assert np.array_equal(flags[st][0], infos[st]["T"]), (k, st)
            assert np.array_equal(flags[st][1], infos[st]["H"]), (k, st)
        e = p1_field_err(G, ref)
        worst = max(worst, e)
        assert e < TOL, (k, e)
        U, t = ref, t + dt
    print(f"dmr lockstep: worst field error {worst:.3e}, rounding ties {ties}")
    s.close()


def dmr_rk3_with_flags(o, U, dt, t, Ts):
    """The oracle's step with given flags at the stage times of a step from t."""
    L0, i0 = o.operator(U, T_fixed=Ts[0], t=t)
    W0 = i0["limited"]
    S1 = W0 + dt * L0
    L1, i1 = o.operator(S1, T_fixed=Ts[1], t=t + dt)
    S2 = 0.75 * W0 + 0.25 * i1["limited"] + 0.25 * dt * L1
    L2, i2 = o.operator(S2, T_fixed=Ts[2], t=t + 0.5 * dt)
    return W0 / 3.0 + 2.0 / 3.0 * i2["limited"] + 2.0 / 3.0 * dt * L2, [i0, i1, i2], [U, S1, S2]


def test_dmr_full_size(hw):
    ny, T = 480, 0.2
    s, o = pair(hw, ny, 3)
    s.set_state(hi.example_3_10(4 * ny, ny))
    steps, t = s.run(T)
    U, t = s.get_state()
    assert abs(t - T) < 1e-12 and steps > 1000
    rho = U[0, 0]
    p = 0.4 * (U[0, 3] - 0.5 * (U[0, 1] ** 2 + U[0, 2] ** 2) / rho)
    assert np.isfinite(U).all() and rho.min() > 0.0 and p.min() > 0.0
    h = 1.0 / ny
    top = rho[-1]
    mid = 0.5 * (8.0 + 1.4)
    k = np.nonzero((top[:-1] > mid) & (top[1:] <= mid))[0][-1]
    xc = (np.arange(4 * ny) + 0.5) * h
    x_num = xc[k] + h * (top[k] - mid) / (top[k] - top[k + 1])
    x_exact = dmr.shock_offset(T) + (1.0 - 0.5 * h) / math.sqrt(3.0)
    print(f"dmr 1920x480: {steps} steps, top-row shock at {x_num:.4f} (exact {x_exact:.4f})")
    assert abs(x_num - x_exact) < 2.0 * h
    # one operator evaluation of the final state on the whole mesh
    s.flag_export(True)
    L, W = s.apply_operator(U)
    Tf, Hf = s.flags(0)
    Lo, info = o.operator(U, t=t)
    if differing_flags_are_ties(o, [U], [Tf], [t])[0]:
        Lo, info = o.operator(U, T_fixed=Tf, t=t)
    assert np.array_equal(Tf, info["T"]) and np.array_equal(Hf, info["H"])
    print(f"final operator: L {array_err(L, Lo):.3e}, troubled {int(Tf.sum())}, hybrid {int(Hf.sum())}")
    assert array_err(L, Lo) < TOL and array_err(W, info["limited"]) < TOL
    s.close()
