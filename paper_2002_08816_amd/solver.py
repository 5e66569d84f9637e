"""Python handles over the C ABI (include/hweno.h).  Arrays cross the boundary as numpy
host arrays or torch device tensors; every step of the scheme runs in the HIP library."""
import hashlib
import json
import os

import numpy as np

from . import capi

_EQ = {"advection": capi.HW_ADVECTION, "burgers": capi.HW_BURGERS, "euler": capi.HW_EULER}
_BC = {"periodic": capi.HW_BC_PERIODIC, "transmissive": capi.HW_BC_TRANSMISSIVE,
       "reflective": capi.HW_BC_REFLECTIVE, "dmr": capi.HW_BC_DMR, "step": capi.HW_BC_STEP}
_TC = {"kxrcf": capi.HW_TC_KXRCF, "none": capi.HW_TC_NONE, "all": capi.HW_TC_ALL}


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the HIP library needs an MI355X (gfx950)")
    return torch


def new_stream():
    """A torch stream of default priority for one handle.  Its raw hipStream_t is given to
    the library, so torch copies and events on it are ordered with the library's work
    (the null stream cannot be captured into a HIP graph)."""
    torch = _torch()
    ts = torch.cuda.Stream()
    return ts, capi.c_void_p(ts.cuda_stream)


def make_config(dim, nx, ny=1, domain=(0.0, 1.0, 0.0, 1.0), eq="euler", adv=(1.0, 1.0),
                gamma=1.4, bc=("periodic", "periodic"), ng_edge=3, lim_w=None, rec_w=None,
                eps=1e-6, cfl=0.6, tc_mode="kxrcf", step=None, inflow=None):
    """step: the corner (x, y) of the forward step, inflow: its (rho, u, v, p) (bc "step";
    default: Example 3.11's (0.6, 0.2) and Mach 3 (1.4, 3, 0, 1))."""
    cfg = capi.hw_config_default(dim)
    cfg.nx, cfg.ny = int(nx), int(ny) if dim == 2 else 1
    cfg.x0, cfg.x1 = float(domain[0]), float(domain[1])
    if dim == 2:
        cfg.y0, cfg.y1 = float(domain[2]), float(domain[3])
    cfg.eq = _EQ[eq]
    cfg.adv[0], cfg.adv[1] = float(adv[0]), float(adv[1] if len(adv) > 1 else 0.0)
    cfg.gamma_gas = float(gamma)
    if isinstance(bc, str):
        bc = (bc, bc)
    cfg.bc_x, cfg.bc_y = _BC[bc[0]], _BC[bc[1]]
    cfg.ng_edge = int(ng_edge)
    if lim_w is not None:
        for i, v in enumerate(lim_w):
            cfg.lim_w[i] = float(v)
    if rec_w is not None:
        for i in range(5):
            cfg.rec_w[i] = float(rec_w[i]) if i < len(rec_w) else 0.0
    cfg.eps, cfg.cfl = float(eps), float(cfl)
    cfg.tc_mode = _TC[tc_mode]
    if step is not None:
        cfg.step_x, cfg.step_y = float(step[0]), float(step[1])
    if inflow is not None:
        for i in range(4):
            cfg.inflow[i] = float(inflow[i])
    return cfg


class Solver:
    """One mesh (dim = 1 or 2).  State arrays: (nmom, ncomp, nx) in 1D and
    (nmom, ncomp, ny, nx) in 2D, nmom = dim + 1 (averages, x moments[, y moments])."""

    def __init__(self, dim, nx, ny=1, **kw):
        self.dim = dim
        self.cfg = make_config(dim, nx, ny, **kw)
        self.tstream, self.stream = new_stream()
        self.h = capi.hw_create(self.cfg, self.stream)
        self.cells, self.ncomp, self.nmom = capi.hw_get_sizes(self.h)
        self.shape = (self.nmom, self.ncomp) + ((self.cfg.ny, self.cfg.nx) if dim == 2 else (self.cfg.nx,))

    def close(self):
        if self.h:
            capi.hw_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_mesh(self, faces):
        """1D: cells [faces[i], faces[i+1]] of different sizes (nx + 1 increasing
        coordinates), or None for the configuration's uniform mesh."""
        f = None if faces is None else np.ascontiguousarray(faces, dtype=np.float64)
        if f is not None and f.shape != (self.cfg.nx + 1,):
            raise ValueError(f"faces shape {f.shape} != ({self.cfg.nx + 1},)")
        capi.hw_set_mesh_1d(self.h, f)

    def set_state(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        if U.shape != self.shape:
            raise ValueError(f"state shape {U.shape} != {self.shape}")
        capi.hw_set_state(self.h, U[0], U[1], U[2] if self.dim == 2 else None)

    def get_state(self):
        U = np.empty(self.shape)
        t = capi.hw_get_state(self.h, U[0], U[1], U[2] if self.dim == 2 else None)
        return U, t

    def step(self, dt=0.0):
        capi.hw_step(self.h, dt)

    def steps(self, n, dt=0.0):
        capi.hw_steps(self.h, n, dt)

    def run(self, T, max_steps=10 ** 9):
        return capi.hw_run(self.h, T, max_steps)

    def set_linear_weights(self, lim_w=None, rec_w=None):
        capi.hw_set_linear_weights(self.h, lim_w, rec_w)

    def flag_export(self, on=True):
        capi.hw_set_flag_export(self.h, on)

    def flags(self, stage):
        T = np.empty(self.cells, np.uint8)
        H = np.empty(self.cells, np.uint8)
        capi.hw_get_flags(self.h, stage, T, H)
        sh = self.shape[2:]
        return T.reshape(sh), H.reshape(sh)

    def time(self):
        t = np.empty(1)
        steps = capi.hw_get_time(self.h, t)
        return float(t[0]), steps

    def set_time(self, t):
        """Sets the time of the current state (time-dependent boundary data read it)."""
        capi.hw_set_time(self.h, t)

    def stats(self):
        """(Lax-Friedrichs speed per direction of the current state, troubled cells per stage
        of the last step, HWENO cells per stage of the last step)."""
        return capi.hw_get_stats(self.h, self.dim)

    def apply_operator(self, U):
        """L(U) and the limited state (numpy in, numpy out; device buffers from torch)."""
        torch = _torch()
        U = np.ascontiguousarray(U, dtype=np.float64)
        with torch.cuda.stream(self.tstream):
            d_in = torch.from_numpy(U).cuda()
            d_L = torch.empty_like(d_in)
            d_W = torch.empty_like(d_in)
            capi.hw_apply_operator(self.h, d_in.data_ptr(), d_L.data_ptr(), d_W.data_ptr())
            L, W = d_L.cpu(), d_W.cpu()
        self.tstream.synchronize()
        return L.numpy(), W.numpy()

    def profile(self, nsteps, dt=0.0):
        return capi.hw_profile_steps(self.h, nsteps, dt)

    # ------------------------------------------------------------ reverse mode (2D scalar)
    def _on_stream(self, fn):
        """Runs fn() (which enqueues library work on the handle's stream) ordered after
        the caller's current torch stream, and orders that stream after it."""
        torch = _torch()
        cur = torch.cuda.current_stream()
        self.tstream.wait_stream(cur)
        fn()
        cur.wait_stream(self.tstream)

    def apply_operator_adjoint(self, U, lam):
        """(dL/dU)^T lam at U (numpy in, numpy out)."""
        torch = _torch()
        d_in = torch.from_numpy(np.ascontiguousarray(U, dtype=np.float64)).cuda()
        d_l = torch.from_numpy(np.ascontiguousarray(lam, dtype=np.float64)).cuda()
        d_o = torch.empty_like(d_in)
        self._on_stream(lambda: capi.hw_apply_operator_adjoint(self.h, d_in.data_ptr(), d_l.data_ptr(),
                                                               d_o.data_ptr()))
        return d_o.cpu().numpy()

    def forward_ckpt(self, nsteps, dt, k):
        """nsteps fixed-dt steps of the current state, recorded for adjoint()."""
        self._on_stream(lambda: capi.hw_forward_ckpt(self.h, nsteps, dt, k))

    def adjoint(self, lam_T):
        """Gradient of the recorded run for the final-state cotangent lam_T (a device
        tensor of the state's shape, or a numpy array); returns the same kind."""
        torch = _torch()
        as_np = isinstance(lam_T, np.ndarray)
        d_l = (torch.from_numpy(np.ascontiguousarray(lam_T, dtype=np.float64)).cuda() if as_np
               else lam_T.detach().to(torch.float64).contiguous())
        if tuple(d_l.shape) != self.shape or not d_l.is_cuda:
            raise ValueError(f"cotangent must be a device array of shape {self.shape}")
        d_g = torch.empty_like(d_l)
        self._on_stream(lambda: capi.hw_adjoint(self.h, d_l.data_ptr(), d_g.data_ptr()))
        return d_g.cpu().numpy() if as_np else d_g

    def set_state_tensor(self, U):
        """Sets the state from a device tensor of the state's shape (time reset to 0)."""
        torch = _torch()
        U = U.detach().to(torch.float64).contiguous()
        if tuple(U.shape) != self.shape or not U.is_cuda:
            raise ValueError(f"state must be a device tensor of shape {self.shape}")
        self._on_stream(lambda: capi.hw_set_state_device(self.h, U.data_ptr()))

    def get_state_tensor(self):
        torch = _torch()
        out = torch.empty(self.shape, dtype=torch.float64, device="cuda")
        self._on_stream(lambda: capi.hw_get_state_device(self.h, out.data_ptr()))
        return out


class BatchSolver:
    """Independent 1D instances of different sizes (concatenated state
    (2, ncomp, sum(nx)), instance by instance inside each component)."""

    def __init__(self, sizes, x0=None, x1=None, **kw):
        self.sizes = np.asarray(sizes, dtype=np.int64)
        self.cfg = make_config(1, int(self.sizes[0]), **kw)
        self.tstream, self.stream = new_stream()
        self.h = capi.hw_batch_create(self.cfg, list(self.sizes), x0, x1, self.stream)
        self.cells, self.ncomp, self.nmom = capi.hw_get_sizes(self.h)
        self.shape = (2, self.ncomp, self.cells)
        self.offsets = np.concatenate([[0], np.cumsum(self.sizes)])

    def close(self):
        if self.h:
            capi.hw_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_states(self, Us):
        U = np.concatenate([np.asarray(u, dtype=np.float64) for u in Us], axis=-1)
        if U.shape != self.shape:
            raise ValueError(f"state shape {U.shape} != {self.shape}")
        U = np.ascontiguousarray(U)
        capi.hw_set_state(self.h, U[0], U[1], None)

    def get_states(self):
        U = np.empty(self.shape)
        capi.hw_get_state(self.h, U[0], U[1], None)
        return [U[..., a:b] for a, b in zip(self.offsets[:-1], self.offsets[1:])]

    def times(self):
        t = np.empty(len(self.sizes))
        steps = capi.hw_get_time(self.h, t)
        return t, steps

    def steps(self, n, persistent=None):
        """n graph-replayed CFL steps; persistent None uses the autotuned launch form."""
        capi.hw_batch_steps(self.h, n, -1 if persistent is None else (1 if persistent else 0))

    def tune(self, cache=None):
        """Picks the launch form; returns (tile width, persistent, persistent grid).  With a
        cache file (JSON), a form stored there for the same workload and device is applied
        without timing; otherwise the autotuner runs and its choice is stored."""
        key = None
        if cache is not None:
            torch = _torch()
            sig = {"sizes": hashlib.sha1(self.sizes.tobytes()).hexdigest(), "n": int(len(self.sizes)),
                   "eq": int(self.cfg.eq), "tc": int(self.cfg.tc_mode), "bc": int(self.cfg.bc_x),
                   "device": torch.cuda.get_device_name()}
            key = json.dumps(sig, sort_keys=True)
            table = {}
            if os.path.exists(cache):
                with open(cache) as f:
                    table = json.load(f)
            if key in table:
                tile, persistent, grid = (int(v) for v in table[key])
                capi.hw_batch_set_form(self.h, tile, persistent, grid)
                return tile, persistent, grid
        choice = capi.hw_batch_tune(self.h)
        if cache is not None:
            table = {}
            if os.path.exists(cache):
                with open(cache) as f:
                    table = json.load(f)
            table[key] = list(choice)
            tmp = cache + ".tmp"
            with open(tmp, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return choice

    def set_form(self, tile, persistent, grid=0):
        """Sets the launch form directly (tile width, persistent 0/1, persistent grid)."""
        capi.hw_batch_set_form(self.h, tile, persistent, grid)

    def set_meshes(self, faces):
        """Cells of different sizes: one array of n_b + 1 increasing face coordinates per
        instance, or None for the uniform meshes of the batch's configuration."""
        if faces is None:
            capi.hw_set_mesh_1d(self.h, None)
            return
        if len(faces) != len(self.sizes):
            raise ValueError(f"{len(faces)} face arrays for {len(self.sizes)} instances")
        fs = []
        for f, n in zip(faces, self.sizes):
            f = np.asarray(f, dtype=np.float64)
            if f.shape != (int(n) + 1,):
                raise ValueError(f"faces shape {f.shape} != ({int(n) + 1},)")
            fs.append(f)
        capi.hw_set_mesh_1d(self.h, np.ascontiguousarray(np.concatenate(fs)))

    def stats(self):
        """(Lax-Friedrichs speed over all instances, troubled and HWENO cell counts per stage
        of the last step; the counts need flag export, else -1)."""
        return capi.hw_get_stats(self.h, 1)

    def flag_export(self, on=True):
        capi.hw_set_flag_export(self.h, on)

    def flags(self, stage):
        """Per-instance (T, H) flag arrays of stage 0, 1 or 2 of the last step."""
        T = np.empty(self.cells, np.uint8)
        H = np.empty(self.cells, np.uint8)
        capi.hw_get_flags(self.h, stage, T, H)
        cut = lambda A: [A[a:b] for a, b in zip(self.offsets[:-1], self.offsets[1:])]
        return cut(T), cut(H)
