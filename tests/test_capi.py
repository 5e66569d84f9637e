"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every function
declared in include/hweno.h with the binding's signature table, fills the paper's
defaults, and rejects invalid configurations before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hweno.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_]+\s*\*?\s*(hw_[a-z_0-9]+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_abi():
    names = declared_functions()
    for must in ("hw_create", "hw_destroy", "hw_set_state", "hw_get_state", "hw_step", "hw_run",
                 "hw_apply_operator", "hw_batch_create", "hw_batch_steps", "hw_batch_tune"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2002_08816_amd import capi
    lib = ctypes.CDLL(capi.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert name in capi.SIGNATURES, name
    assert set(capi.SIGNATURES) == set(declared_functions())


def test_config_defaults_follow_the_paper():
    from paper_2002_08816_amd import capi
    c1 = capi.hw_config_default(1)
    assert c1.dim == 1 and c1.eps == 1e-6 and c1.cfl == 0.6 and c1.gamma_gas == 1.4
    assert list(c1.lim_w) == [0.98, 0.01, 0.01]
    assert list(c1.rec_w)[:3] == [0.98, 0.01, 0.01]
    c2 = capi.hw_config_default(2)
    assert list(c2.rec_w) == [0.96, 0.01, 0.01, 0.01, 0.01]
    assert c2.ng_edge == 3 and c2.tc_mode == capi.HW_TC_KXRCF
    # Example 3.11: step corner (0.6, 0.2), Mach 3 inflow (rho, u, v, p) = (1.4, 3, 0, 1)
    assert (c2.step_x, c2.step_y) == (0.6, 0.2) and list(c2.inflow) == [1.4, 3.0, 0.0, 1.0]


def _bad(mutate, dim=2):
    from paper_2002_08816_amd import capi
    cfg = capi.hw_config_default(dim)
    cfg.nx = 16
    cfg.ny = 16 if dim == 2 else 1
    mutate(cfg)
    with pytest.raises(capi.HWError) as ei:
        capi.hw_create(cfg, None)
    assert ei.value.status == capi.HW_EINVAL
    return str(ei.value)


def test_invalid_configurations_are_rejected():
    assert "sum to 1" in _bad(lambda c: c.lim_w.__setitem__(0, 0.5))
    assert "positive" in _bad(lambda c: c.rec_w.__setitem__(1, -0.01))
    assert "7 cells" in _bad(lambda c: setattr(c, "nx", 6))
    assert "ng_edge" in _bad(lambda c: setattr(c, "ng_edge", 4))
    assert "square" in _bad(lambda c: setattr(c, "y1", 2.0))
    assert "dim" in _bad(lambda c: setattr(c, "dim", 3))
    assert "eps" in _bad(lambda c: setattr(c, "eps", 0.0))
    assert "cfl" in _bad(lambda c: setattr(c, "cfl", -1.0))
    assert "gamma" in _bad(lambda c: setattr(c, "gamma_gas", 1.0))
    assert "empty" in _bad(lambda c: setattr(c, "x1", 0.0), dim=1)
    assert "boundary" in _bad(lambda c: setattr(c, "bc_x", 5))
    # double Mach reflection boundaries: 2D Euler, both directions
    assert "double Mach" in _bad(lambda c: setattr(c, "bc_x", 3))
    assert "double Mach" in _bad(lambda c: setattr(c, "bc_y", 3), dim=2)
    # reflective walls: Euler only (1D and 2D)
    from paper_2002_08816_amd import capi

    # forward step: 2D Euler, both directions, the corner on cell faces with room around it
    def step(**kw):
        def m(c):
            c.bc_x = c.bc_y = capi.HW_BC_STEP
            c.x1, c.y1 = 3.0, 1.0
            c.nx, c.ny = 60, 20
            for k, v in kw.items():
                if k == "inflow":
                    for i in range(4):
                        c.inflow[i] = v[i]
                else:
                    setattr(c, k, v)
        return m
    assert "forward-step" in _bad(lambda c: setattr(c, "bc_x", capi.HW_BC_STEP))
    assert "forward-step" in _bad(step(eq=capi.HW_BURGERS))
    assert "cell faces" in _bad(step(step_x=0.61))
    assert "corner cells" in _bad(step(step_y=0.1))          # sj = 2 < 3
    assert "corner cells" in _bad(step(step_y=0.6))          # 2 sj > ny
    assert "corner cells" in _bad(step(step_x=0.1))          # si < sj
    assert "corner cells" in _bad(step(step_x=3.0))          # si = nx
    assert "inflow" in _bad(step(inflow=(1.4, 3.0, 0.0, -1.0)))

    def refl(eq):
        def m(c):
            c.bc_x = capi.HW_BC_REFLECTIVE
            c.eq = eq
        return m
    assert "reflective" in _bad(refl(capi.HW_BURGERS), dim=2)
    assert "reflective" in _bad(refl(capi.HW_BURGERS), dim=1)
    assert "reflective" in _bad(refl(capi.HW_ADVECTION), dim=1)


def test_batch_rejects_bad_instances():
    from paper_2002_08816_amd import capi
    cfg = capi.hw_config_default(1)
    with pytest.raises(capi.HWError) as ei:
        capi.hw_batch_create(cfg, [32, 5, 64])
    assert ei.value.status == capi.HW_EINVAL and "instance 1" in str(ei.value)
    cfg2 = capi.hw_config_default(2)
    cfg2.nx = cfg2.ny = 16
    with pytest.raises(capi.HWError):
        capi.hw_batch_create(cfg2, [32])


def test_status_strings():
    from paper_2002_08816_amd import capi
    assert capi.hw_status_string(capi.HW_ENONFINITE).startswith("non-finite")
    assert capi.hw_status_string(99) == "unknown status"


def test_product_path_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2002_08816_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
