"""The no-allocation operator (hw_apply_operator_noalloc) against the handle's operator
(hw_apply_operator), through the C ABI: the same kernels on the same input, so the
results must be identical, for two calls in a row on one GPU (the second on a smaller
mesh, so it runs on what the first left in the shared scratch array), with troubled-cell
detection on.  Also: a mesh beyond the scratch limit is rejected before any GPU work."""
import ctypes

import numpy as np
import pytest

import hweno_inputs as hi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hw():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2002_08816_amd as hw
    return hw


def handle_operator(hw, cfg, U):
    """(L, limited) from a handle created for cfg, through hw_apply_operator."""
    import torch
    from paper_2002_08816_amd import capi
    ts, st = hw.solver.new_stream()
    h = capi.hw_create(cfg, st)
    try:
        with torch.cuda.stream(ts):
            d_in = torch.from_numpy(U).cuda()
            d_L = torch.empty_like(d_in)
            d_W = torch.empty_like(d_in)
            capi.hw_apply_operator(h, d_in.data_ptr(), d_L.data_ptr(), d_W.data_ptr())
            L, W = d_L.cpu().numpy(), d_W.cpu().numpy()
        ts.synchronize()
    finally:
        capi.hw_destroy(h)
    return L, W


def noalloc_operator(cfg, U, ts, st):
    import torch
    from paper_2002_08816_amd import capi
    with torch.cuda.stream(ts):
        d_in = torch.from_numpy(U).cuda()
        d_L = torch.full_like(d_in, float("nan"))
        d_W = torch.full_like(d_in, float("nan"))
        capi.hw_apply_operator_noalloc(cfg, d_in.data_ptr(), d_L.data_ptr(), d_W.data_ptr(), st)
        L, W = d_L.cpu().numpy(), d_W.cpu().numpy()
    ts.synchronize()
    return L, W


@pytest.mark.parametrize("eq,ng,tc", [("euler", 2, "kxrcf"), ("euler", 3, "all"), ("burgers", 3, "kxrcf")])
def test_noalloc_operator_matches_the_handle_operator(hw, eq, ng, tc):
    from paper_2002_08816_amd.solver import make_config, new_stream
    ts, st = new_stream()
    # Euler with two edge points first runs the largest square mesh the scratch holds
    first = 448 if (eq, ng) == ("euler", 2) else 160
    for n, seed, bc in ((first, 0, "periodic"), (72, 1, "transmissive")):
        if eq == "euler":
            U, _ = hi.euler_shock_vortex_2d(seed, n)
            bcs = ("periodic", bc)
        else:
            U, _ = hi.burgers_modes_2d(seed, n)
            bcs = (bc, bc)
        U = np.ascontiguousarray(U)
        cfg = make_config(2, n, n, eq=eq, ng_edge=ng, tc_mode=tc, bc=bcs,
                          domain=(0.0, 1.0, 0.0, 1.0) if eq == "euler" else (0.0, 4.0, 0.0, 4.0))
        print(f"case {eq} ng={ng} tc={tc} n={n} bc={bcs}", flush=True)
        L0, W0 = handle_operator(hw, cfg, U)
        L1, W1 = noalloc_operator(cfg, U, ts, st)
        assert np.isfinite(L1).all() and np.isfinite(W1).all()
        assert np.array_equal(L0, L1) and np.array_equal(W0, W1), (n, np.abs(L0 - L1).max())


def test_noalloc_rejects_meshes_beyond_the_scratch(hw):
    from paper_2002_08816_amd import capi
    from paper_2002_08816_amd.solver import make_config
    cfg = make_config(2, 1024, 1024, eq="euler", ng_edge=2, tc_mode="kxrcf")
    with pytest.raises(capi.HWError) as e:
        capi.hw_apply_operator_noalloc(cfg, 1, 1, None, None)
    assert e.value.status == capi.HW_EINVAL and "scratch" in str(e.value)
    cfg1 = make_config(1, 64, eq="euler")
    with pytest.raises(capi.HWError):
        capi.hw_apply_operator_noalloc(cfg1, 1, 1, None, None)
