"""GPU parity of the one-dimensional scheme on meshes of cells of different sizes
(hw_set_mesh_1d) against the oracle's Scheme1DNU, through the C ABI.

* one operator evaluation on random meshes (cell sizes U[1, 3]), every boundary condition
  and troubled-cell mode: every stored array of L and of the limited state within
  max|gpu - oracle| / max|oracle| <= 1e-12 (tests/parity.py), flags and masks identical;
* equal cells through the same entry point give the uniform path's operator (1e-13);
* a lockstep run of the seeded Riemann data on a stretched mesh (every step from the
  oracle's state; fields within 1e-12, flags identical up to proven rounding ties);
* fifth-order convergence of smooth advection on the stretched mesh, GPU alone;
* a batch of instances of different sizes, each on its own random mesh: every instance
  after 40 CFL steps equals the same instance run alone (the single-instance path is the
  one pinned against the oracle above), and faces = None returns to the uniform meshes;
* rejections: 2D handles, faces that are not increasing, launch forms on such a mesh.
"""
import math

import numpy as np
import pytest

import hweno_inputs as hi
from oracle.mesh1d import Scheme1DNU
from oracle.physics import Equation

from parity import TOL, array_err
from test_gpu_shock_suite import lockstep

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hw():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2002_08816_amd as hw
    return hw


def riemann_on(faces, seed):
    prm = hi.euler_riemann_params(np.random.default_rng(2000 + seed))
    return hi.project_1d_faces(hi.euler_riemann_func(*prm), faces)


@pytest.mark.parametrize("bc", ["periodic", "transmissive", "reflective"])
@pytest.mark.parametrize("tc", ["kxrcf", "all", "none"])
def test_nonuniform_operator_matches_the_oracle(hw, bc, tc):
    n = 300                                   # two 256-cell tiles, the second ragged
    faces = hi.random_faces(1, n, 0.0, 1.0, ratio=3.0)
    print(f"non-uniform operator euler n={n} bc={bc} tc={tc}", flush=True)
    U = riemann_on(faces, 4)
    s = hw.Solver(1, n, domain=(faces[0], faces[-1]), eq="euler", bc=bc, tc_mode=tc)
    s.set_mesh(faces)
    s.flag_export(True)
    L, W = s.apply_operator(U)
    T, H = s.flags(0)
    o = Scheme1DNU("euler", faces, bc=bc, tc_mode=tc)
    Lo, info = o.operator(U)
    assert np.array_equal(T, info["T"]) and np.array_equal(H, info["H"])
    if tc == "kxrcf":
        assert 0 < T.sum() < n
    e = max(array_err(L, Lo), array_err(W, info["limited"]))
    print(f"  max array error {e:.3e}")
    assert e < TOL, e
    s.close()


@pytest.mark.parametrize("eq", ["burgers", "advection"])
def test_nonuniform_scalar_operator_matches_the_oracle(hw, eq):
    n = 260
    faces = hi.stretched_faces(n, 0.0, 2.0, amp=0.4)
    _, prm = hi.advection_1d(2, 8)
    U = hi.project_1d_faces(prm["func"], faces)
    U[1] += 0.03 * np.random.default_rng(5).normal(size=U[1].shape)   # flags some cells
    s = hw.Solver(1, n, domain=(0.0, 2.0), eq=eq, bc="periodic", tc_mode="kxrcf")
    s.set_mesh(faces)
    s.flag_export(True)
    L, W = s.apply_operator(U)
    T, _ = s.flags(0)
    o = Scheme1DNU(Equation(eq, 1, adv=(1.0,)), faces, bc="periodic", tc_mode="kxrcf")
    Lo, info = o.operator(U)
    assert np.array_equal(T, info["T"]) and T.any()
    e = max(array_err(L, Lo), array_err(W, info["limited"]))
    print(f"{eq}: max array error {e:.3e}")
    assert e < TOL, e
    s.close()


def test_equal_cells_equal_the_uniform_path(hw):
    n = 400
    U, _ = hi.euler_riemann_1d(seed=2, n=n)
    s = hw.Solver(1, n, eq="euler", bc="transmissive", tc_mode="kxrcf")
    L0, W0 = s.apply_operator(U)
    s.set_mesh(np.linspace(0.0, 1.0, n + 1))
    L1, W1 = s.apply_operator(U)
    s.set_mesh(None)
    L2, _ = s.apply_operator(U)
    assert np.array_equal(L0, L2)
    e = max(array_err(L1, L0), array_err(W1, W0))
    print(f"equal cells: {e:.3e}")
    assert e < 1e-13, e
    s.close()


def test_nonuniform_lockstep_run(hw):
    n, T = 400, 0.1
    faces = hi.stretched_faces(n, 0.0, 1.0, amp=0.3)
    U0 = riemann_on(faces, 3)
    s = hw.Solver(1, n, eq="euler", bc="transmissive", tc_mode="kxrcf")
    s.set_mesh(faces)
    s.flag_export(True)
    o = Scheme1DNU("euler", faces, bc="transmissive", tc_mode="kxrcf")
    counts = lockstep(s, o, U0, T, "non-uniform Riemann")
    assert counts.sum() > 0
    s.close()


def test_fifth_order_on_the_gpu(hw):
    ns = (40, 80, 160)
    _, prm = hi.advection_1d(0, 8)
    errs = []
    for n in ns:
        faces = hi.stretched_faces(n, 0.0, 2.0, amp=0.3)
        U0 = hi.project_1d_faces(prm["func"], faces)
        s = hw.Solver(1, n, domain=(0.0, 2.0), eq="advection", adv=(1.0, 1.0), bc="periodic",
                      tc_mode="none")
        s.set_mesh(faces)
        h = np.diff(faces).min()
        h0 = np.diff(hi.stretched_faces(ns[0], 0.0, 2.0, amp=0.3)).min()
        dt = 0.5 * h * (h / h0) ** (2.0 / 3.0)
        nsteps = int(math.ceil(2.0 / dt - 1e-9))
        s.set_state(U0)
        s.steps(nsteps, 2.0 / nsteps)
        U, _ = s.get_state()
        e = np.abs(U[0, 0] - U0[0, 0])
        errs.append((e.mean(), e.max()))
        s.close()
    o = [(math.log(errs[i][0] / errs[i + 1][0]) / math.log(2.0),
          math.log(errs[i][1] / errs[i + 1][1]) / math.log(2.0)) for i in range(2)]
    print("errors", errs, "orders", o)
    assert o[-1][0] >= 4.7 and o[-1][1] >= 4.7


def test_nonuniform_batch_matches_single_instances(hw):
    sizes = np.array([300, 513, 256, 700, 97])
    faces = [hi.random_faces(10 + b, int(n), 0.0, 1.0 + 0.25 * b, ratio=3.0) for b, n in enumerate(sizes)]
    Us = [riemann_on(f, 20 + b) for b, f in enumerate(faces)]
    nsteps = 40
    print(f"non-uniform batch {list(sizes)}, {nsteps} CFL steps", flush=True)
    bs = hw.BatchSolver(sizes, eq="euler", bc="transmissive", tc_mode="kxrcf")
    bs.set_meshes(faces)
    bs.set_states(Us)
    bs.steps(nsteps)
    got = bs.get_states()
    tb, sb = bs.times()
    for b, (f, n) in enumerate(zip(faces, sizes)):
        s = hw.Solver(1, int(n), domain=(f[0], f[-1]), eq="euler", bc="transmissive", tc_mode="kxrcf")
        s.set_mesh(f)
        s.set_state(Us[b])
        s.steps(nsteps)
        U, t = s.get_state()
        e = np.abs(got[b] - U).max() / np.abs(U).max()
        print(f"  instance {b} (n={n}): t = {t:.6f}, batch t = {tb[b]:.6f}, max rel diff {e:.2e}")
        assert abs(tb[b] - t) <= 1e-14 * t
        assert e <= 1e-13, (b, e)
        s.close()
    # back to the uniform meshes of the configuration (unit intervals)
    bs.set_meshes(None)
    Uu = [riemann_on(np.linspace(0.0, 1.0, int(n) + 1), 30 + b) for b, n in enumerate(sizes)]
    bs.set_states(Uu)
    bs.steps(3)
    ref = hw.BatchSolver(sizes, eq="euler", bc="transmissive", tc_mode="kxrcf")
    ref.set_states(Uu)
    ref.steps(3)
    for a, c in zip(bs.get_states(), ref.get_states()):
        assert np.array_equal(a, c)
    assert np.array_equal(bs.times()[0], ref.times()[0])
    bs.close()
    ref.close()


def test_mesh_rejections(hw):
    from paper_2002_08816_amd import capi
    s = hw.Solver(2, 16, 16, eq="burgers")
    with pytest.raises(capi.HWError) as ei:
        capi.hw_set_mesh_1d(s.h, np.linspace(0.0, 1.0, 17))
    assert ei.value.status == capi.HW_EINVAL
    s.close()
    b = hw.BatchSolver(np.array([64, 80]), eq="euler", bc="transmissive", tc_mode="kxrcf")
    with pytest.raises(ValueError):
        b.set_meshes([np.linspace(0.0, 1.0, 65)])              # one array per instance
    f = [np.linspace(0.0, 1.0, 65), np.linspace(0.0, 2.0, 81)]
    f[1][40] = f[1][39]
    with pytest.raises(capi.HWError) as ei:
        b.set_meshes(f)
    assert ei.value.status == capi.HW_EINVAL
    b.set_meshes([np.linspace(0.0, 1.0, 65), np.linspace(0.0, 2.0, 81)])
    with pytest.raises(capi.HWError) as ei:
        b.tune()
    assert ei.value.status == capi.HW_EINVAL
    b.close()
    s = hw.Solver(1, 32, eq="euler", bc="transmissive")
    f = np.linspace(0.0, 1.0, 33)
    f[10] = f[9]
    with pytest.raises(capi.HWError) as ei:
        s.set_mesh(f)
    assert ei.value.status == capi.HW_EINVAL
    s.set_mesh(np.linspace(0.0, 1.0, 33))
    with pytest.raises(capi.HWError) as ei:
        capi.hw_batch_set_form(s.h, 128, 0, 0)
    assert ei.value.status == capi.HW_EINVAL
    s.set_mesh(None)
    s.close()
