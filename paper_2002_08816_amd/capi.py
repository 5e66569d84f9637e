"""ctypes binding of the C ABI declared in include/hweno.h (argument marshalling only).

Every function here has the name of the C entry point it forwards to.  The library is
loaded from this package's directory; importing this module on a machine where it has not
been built raises an ImportError (there is no fallback path)."""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhweno.so")

c_int, c_long, c_double, c_void_p, c_char_p = (ctypes.c_int, ctypes.c_long, ctypes.c_double,
                                               ctypes.c_void_p, ctypes.c_char_p)
P_double = ctypes.POINTER(ctypes.c_double)
P_int = ctypes.POINTER(ctypes.c_int)
P_long = ctypes.POINTER(ctypes.c_long)
P_uchar = ctypes.POINTER(ctypes.c_ubyte)

HW_OK, HW_EINVAL, HW_ENOMEM, HW_EDEVICE, HW_ENONFINITE, HW_ESTATE = range(6)
HW_ADVECTION, HW_BURGERS, HW_EULER = range(3)
HW_BC_PERIODIC, HW_BC_TRANSMISSIVE, HW_BC_REFLECTIVE, HW_BC_DMR, HW_BC_STEP = range(5)
HW_TC_KXRCF, HW_TC_NONE, HW_TC_ALL = range(3)


class hw_config(ctypes.Structure):
    _fields_ = [("dim", c_int), ("nx", c_int), ("ny", c_int),
                ("x0", c_double), ("x1", c_double), ("y0", c_double), ("y1", c_double),
                ("eq", c_int), ("adv", c_double * 2), ("gamma_gas", c_double),
                ("bc_x", c_int), ("bc_y", c_int), ("ng_edge", c_int),
                ("lim_w", c_double * 3), ("rec_w", c_double * 5),
                ("eps", c_double), ("cfl", c_double), ("tc_mode", c_int),
                ("step_x", c_double), ("step_y", c_double), ("inflow", c_double * 4)]


# name -> (restype, argtypes), in the order of include/hweno.h
SIGNATURES = {
    "hw_config_default": (None, [ctypes.POINTER(hw_config), c_int]),
    "hw_create": (c_int, [ctypes.POINTER(hw_config), c_void_p, ctypes.POINTER(c_void_p)]),
    "hw_batch_create": (c_int, [ctypes.POINTER(hw_config), c_int, P_int, P_double, P_double,
                                c_void_p, ctypes.POINTER(c_void_p)]),
    "hw_destroy": (c_int, [c_void_p]),
    "hw_get_sizes": (c_int, [c_void_p, P_long, P_int, P_int]),
    "hw_set_state": (c_int, [c_void_p, P_double, P_double, P_double]),
    "hw_get_state": (c_int, [c_void_p, P_double, P_double, P_double, P_double]),
    "hw_set_state_device": (c_int, [c_void_p, c_void_p]),
    "hw_get_state_device": (c_int, [c_void_p, c_void_p]),
    "hw_step": (c_int, [c_void_p, c_double]),
    "hw_steps": (c_int, [c_void_p, c_int, c_double]),
    "hw_run": (c_int, [c_void_p, c_double, c_long, P_long, P_double]),
    "hw_apply_operator": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "hw_set_linear_weights": (c_int, [c_void_p, P_double, P_double]),
    "hw_set_flag_export": (c_int, [c_void_p, c_int]),
    "hw_get_flags": (c_int, [c_void_p, c_int, P_uchar, P_uchar]),
    "hw_get_time": (c_int, [c_void_p, P_double, P_long]),
    "hw_set_time": (c_int, [c_void_p, c_double]),
    "hw_set_mesh_1d": (c_int, [c_void_p, P_double]),
    "hw_get_stats": (c_int, [c_void_p, P_double, P_long, P_long]),
    "hw_profile_steps": (c_int, [c_void_p, c_int, c_double, P_double, P_double, P_double]),
    "hw_batch_steps": (c_int, [c_void_p, c_int, c_int]),
    "hw_batch_tune": (c_int, [c_void_p, P_int]),
    "hw_batch_set_form": (c_int, [c_void_p, c_int, c_int, c_int]),
    "hw_apply_operator_adjoint": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "hw_forward_ckpt": (c_int, [c_void_p, c_int, c_double, c_int]),
    "hw_adjoint": (c_int, [c_void_p, c_void_p, c_void_p]),
    "hw_apply_operator_noalloc": (c_int, [ctypes.POINTER(hw_config), c_void_p, c_void_p, c_void_p, c_void_p]),
    "hw_last_error": (c_char_p, [c_void_p]),
    "hw_status_string": (c_char_p, [c_int]),
}


def _load():
    # torch ships its own HIP runtime (same soname as the system one).  Loading torch
    # first makes the library bind to that runtime, so device pointers and streams from
    # torch are the library's own; loading the library first would put two runtimes in
    # the process.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                          "(python -m paper_2002_08816_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


class HWError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{_lib.hw_status_string(status).decode()}: {message}")
        self.status = status


def _check(status, handle=None):
    if status != HW_OK:
        raise HWError(status, (_lib.hw_last_error(handle) or b"").decode())
    return status


# ---------------------------------------------------------------- forwarding functions
def hw_config_default(dim):
    cfg = hw_config()
    _lib.hw_config_default(ctypes.byref(cfg), int(dim))
    return cfg


def hw_create(cfg, stream=None):
    out = c_void_p()
    _check(_lib.hw_create(ctypes.byref(cfg), stream, ctypes.byref(out)))
    return out


def hw_batch_create(cfg, nx, x0=None, x1=None, stream=None):
    n = len(nx)
    arr_nx = (c_int * n)(*[int(v) for v in nx])
    a0 = (c_double * n)(*x0) if x0 is not None else None
    a1 = (c_double * n)(*x1) if x1 is not None else None
    out = c_void_p()
    _check(_lib.hw_batch_create(ctypes.byref(cfg), n, arr_nx, a0, a1, stream, ctypes.byref(out)))
    return out


def hw_destroy(h):
    _check(_lib.hw_destroy(h))


def hw_get_sizes(h):
    cells, nc, nm = c_long(), c_int(), c_int()
    _check(_lib.hw_get_sizes(h, ctypes.byref(cells), ctypes.byref(nc), ctypes.byref(nm)), h)
    return cells.value, nc.value, nm.value


def _dptr(a):
    return a.ctypes.data_as(P_double) if a is not None else None


def hw_set_state(h, avg, mx, my=None):
    _check(_lib.hw_set_state(h, _dptr(avg), _dptr(mx), _dptr(my)), h)


def hw_get_state(h, avg, mx, my=None):
    t = c_double()
    _check(_lib.hw_get_state(h, _dptr(avg), _dptr(mx), _dptr(my), ctypes.byref(t)), h)
    return t.value


def hw_set_state_device(h, dptr):
    _check(_lib.hw_set_state_device(h, c_void_p(dptr)), h)


def hw_get_state_device(h, dptr):
    _check(_lib.hw_get_state_device(h, c_void_p(dptr)), h)


def hw_step(h, dt=0.0):
    return _check(_lib.hw_step(h, float(dt)), h)


def hw_steps(h, nsteps, dt=0.0):
    _check(_lib.hw_steps(h, int(nsteps), float(dt)), h)


def hw_run(h, T, max_steps=10 ** 9):
    steps, t = c_long(), c_double()
    _check(_lib.hw_run(h, float(T), int(max_steps), ctypes.byref(steps), ctypes.byref(t)), h)
    return steps.value, t.value


def hw_apply_operator(h, d_in, d_L, d_lim=None):
    _check(_lib.hw_apply_operator(h, c_void_p(d_in), c_void_p(d_L),
                                  c_void_p(d_lim) if d_lim else None), h)


def hw_set_linear_weights(h, lim_w=None, rec_w=None):
    lw = (c_double * 3)(*lim_w) if lim_w is not None else None
    rw = (c_double * len(rec_w))(*rec_w) if rec_w is not None else None
    _check(_lib.hw_set_linear_weights(h, lw, rw), h)


def hw_set_flag_export(h, on):
    _check(_lib.hw_set_flag_export(h, 1 if on else 0), h)


def hw_get_flags(h, stage, T, H):
    _check(_lib.hw_get_flags(h, int(stage), T.ctypes.data_as(P_uchar), H.ctypes.data_as(P_uchar)), h)


def hw_get_time(h, times):
    steps = c_long()
    _check(_lib.hw_get_time(h, _dptr(times), ctypes.byref(steps)), h)
    return steps.value


def hw_set_time(h, t):
    _check(_lib.hw_set_time(h, float(t)), h)


def hw_set_mesh_1d(h, faces):
    """faces: None (uniform mesh) or a contiguous float64 array of nx + 1 face coordinates."""
    _check(_lib.hw_set_mesh_1d(h, _dptr(faces)), h)


def hw_get_stats(h, ndir):
    """(alpha per direction, flagged cells per stage, hybrid cells per stage)."""
    a = (c_double * 2)()
    f = (c_long * 3)()
    y = (c_long * 3)()
    _check(_lib.hw_get_stats(h, a, f, y), h)
    return tuple(a[:ndir]), tuple(f), tuple(y)


def hw_profile_steps(h, nsteps, dt=0.0):
    """(ms per stage, ms per step, (ms per flags, limiter, HWENO, stage-kernel launch))."""
    a, b = c_double(), c_double()
    k = (c_double * 4)()
    _check(_lib.hw_profile_steps(h, int(nsteps), float(dt), ctypes.byref(a), ctypes.byref(b), k), h)
    return a.value, b.value, tuple(k)


def hw_batch_steps(h, nsteps, persistent=-1):
    _check(_lib.hw_batch_steps(h, int(nsteps), int(persistent)), h)


def hw_batch_tune(h):
    """(tile width, persistent, persistent grid) chosen by the autotuner."""
    g = (c_int * 3)()
    _check(_lib.hw_batch_tune(h, g), h)
    return tuple(g)


def hw_batch_set_form(h, tile, persistent, grid):
    _check(_lib.hw_batch_set_form(h, int(tile), int(persistent), int(grid)), h)


def hw_apply_operator_adjoint(h, d_in, d_lambda, d_out):
    _check(_lib.hw_apply_operator_adjoint(h, c_void_p(d_in), c_void_p(d_lambda), c_void_p(d_out)), h)


def hw_forward_ckpt(h, nsteps, dt, k):
    _check(_lib.hw_forward_ckpt(h, int(nsteps), float(dt), int(k)), h)


def hw_adjoint(h, d_lambda_T, d_grad_U0):
    _check(_lib.hw_adjoint(h, c_void_p(d_lambda_T), c_void_p(d_grad_U0)), h)


def hw_apply_operator_noalloc(cfg, d_in, d_L, d_lim=None, stream=None):
    _check(_lib.hw_apply_operator_noalloc(ctypes.byref(cfg), c_void_p(d_in), c_void_p(d_L),
                                          c_void_p(d_lim) if d_lim else None, stream))


def hw_last_error(h=None):
    return (_lib.hw_last_error(h) or b"").decode()


def hw_status_string(status):
    return _lib.hw_status_string(int(status)).decode()
