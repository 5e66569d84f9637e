#!/usr/bin/env python3
"""Benchmark of the hybrid HWENO stage operator on one MI355X.

Headline workload: 2D Euler (gamma = 1.4) on a 1024 x 1024 uniform mesh of [0, 1]^2,
periodic, averages plus x/y first moments of 4 components (12 FP64 fields per cell),
2-point Gauss rule on edges, KXRCF troubled cells with the limiter and characteristic
HWENO, CFL 0.6 time step computed on the device.  Seeded synthetic shock-plus-isentropic-
vortex initial state (hweno_inputs.euler_shock_vortex_2d).

One benchmark step = one TVD-RK3 step: three stages of four launches each (troubled-cell
flags and work lists, limiter over the flagged list, HWENO over the hybrid list, the stage
kernel) and the time-step launch, replayed from captured graphs (of eight steps, and of one
step for a remainder).  value = cell-stage updates per second = 3 * 1024^2 * K / (time of
K steps), inputs resident in HBM before the timed region.

Beside the headline, on the same GPU:
* batched: 512 independent 1D Euler instances, sizes log-uniform in [256, 8192]
  (hweno_inputs.batch_euler_1d), 200 CFL steps each through the captured step graph with
  the autotuned tile width and launch form; compared with the untuned default (256-cell
  tiles, one workgroup per tile), and with the plain single-instance solver run instance
  after instance (on a sample of instances); batched.roofline prices the algorithmic
  128 B per cell-stage over the whole step;
* adjoint: 2D Burgers 256^2 on [0, 4]^2, NG = 3, 200 steps of dt = 1/(200 pi), checkpoints
  every 20 steps; the backward pass (recompute included) and the recorded forward run
  as multiples of the plain forward run;
* adjoint_euler: the same figures for 2D Euler, the headline shock + vortex state on a
  256^2 periodic mesh (NG = 2, KXRCF, 100 fixed steps, checkpoints every 20 steps);
* adjoint_step: the same on the forward step's boundaries (Example 3.11, 480 x 160,
  NG = 3, the flow at T = 0.5, 40 fixed steps, checkpoints every 20 steps);
* shock_tests: the 1D shock tests of Section 3.2 at the paper's sizes (Lax, Example 3.6,
  N = 200 to T = 0.16; Shu-Osher, Example 3.7, N = 400 to T = 1.8; two blast waves between
  reflective walls, Example 3.8, N = 800 to T = 0.038; discontinuous Burgers,
  Example 3.5, N = 80 to T = 1.5/pi): wall time of the whole run to T (CFL 0.6, one
  call), and the run's troubled share (troubled cells over cells, averaged over every
  stage of every step; a second, step-by-step run reads the stage counts), beside the
  share the paper quotes where it quotes one; the hybrid share (cells reconstructed with
  HWENO, troubled cells and their neighbours) beside it;
* dmr: the double Mach reflection (Example 3.10) at the paper's 1920 x 480 to T = 0.2:
  wall time, steps, cell-stage updates/s, troubled and hybrid shares at T;
* forward_step: the Mach 3 forward step (Example 3.11) at the paper's 960 x 320 to T = 4,
  the same figures over the fluid cells;
* nonuniform_1d: the 1D Euler Riemann workload (N = 2000) on a smoothly stretched mesh
  beside the same data on the uniform mesh (time to T = 0.2 and per step).

roofline: for the dominant kernel, the stage kernel (stage2d_kernel <EULER, NG=2>, the
launch that reads the stage input and u^n and writes the output): algorithmic HBM bytes
per launch (read the stage input and write the output: 192 B/cell; stages 2 and 3 also
read u^n: 288 B/cell; mean 256 B/cell) divided by its mean launch duration, measured with
HIP events around it on the library's stream.  roofline.stage gives the same bytes over
the whole stage (its four launches: flags, limiter, HWENO, stage kernel).  traffic: HBM
bytes per launch (and per stage) measured with rocprofv3 counters, read from the committed
counter summary when it was taken on the current kernel sources.
fp64: the stage kernel's FP64 arithmetic rate against the FP64 vector peak (78.6 TFLOP/s):
flops per launch from the committed FP64 instruction counters (an FMA counts 2, add, mul
and transcendental 1, each per lane of a 64-lane wave) over the measured launch duration,
when the counters were taken on the current kernel sources.
cpu_baseline: the CPU oracle (numpy) on two TVD-RK3 steps of the same 1024^2 state, run on
the host's cores: the mesh is cut into row slabs, each evaluated by the unchanged oracle
(Scheme2D.operator_padded on the slab plus three wrapped ghost layers: the whole-mesh
operator's values, up to numpy's rounding) in its own single-threaded process; the Lax-Friedrichs speeds and the
Runge-Kutta combination are taken on the whole mesh.  single_thread gives the same sample
in one process on one thread.

Graphs: the step graphs the timed region replays (of eight steps and of one step) are
captured before the warm-up steps, from the initial state, which is then set again.
"""
import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
N = 1024
BYTES_PER_CELL_STAGE = 8 * 12 * (2 + 2.0 / 3.0)   # 256 B
METRIC = "FP64 cell-stage updates/s, 2D Euler 1024²; batched & adjoint vs plain"
CSRC = os.path.join(ROOT, "paper_2002_08816_amd", "csrc")
STAGE2D_SOURCES = ["stage2d.hip", "hw_tile2d.h", "hw_device.h", "hw_coeffs2d.h", "hw_stage.h", "hw_dmr.h",
                   "hw_step.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "stage2d_euler_1024_hbm_traffic.md")
FP64_FILE = os.path.join(ROOT, "profiles", "stage2d_euler_1024_instruction_mix.md")
FP64_PEAK_TFLOPS = 78.6
# launch form of the 512-instance batch for counter runs: the autotuner's choice for it on
# MI355X (128-cell tiles, one workgroup per tile)
BATCH_FORM = (128, 0, 0)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched comparison")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint comparison")
    ap.add_argument("--no-shock-tests", action="store_true", help="skip the 1D shock tests")
    ap.add_argument("--no-dmr", action="store_true", help="skip the double Mach reflection run")
    ap.add_argument("--no-step", action="store_true", help="skip the forward-step run")
    ap.add_argument("--no-nonuniform", action="store_true",
                    help="skip the 1D run on a mesh of cells of different sizes")
    ap.add_argument("--profile-run", nargs="?", const="headline", default=None,
                    choices=["headline", "batched", "adjoint", "adjoint_euler"],
                    help="counter-collection run: a 256 MiB device copy (calibration), then "
                         "4 steps of the headline workload (default), 4 steps of the 512-"
                         "instance batch in its tuned form, or one checkpointed forward and "
                         "adjoint pass of the 2D Burgers workload or of the 2D Euler 256^2 "
                         "workload (20 steps); no timing output")
    return ap.parse_args()


def stage2d_source_digest():
    """Digest of the stage kernels' code: comments and blank lines do not count."""
    h = hashlib.sha256()
    for name in STAGE2D_SOURCES:
        with open(os.path.join(CSRC, name)) as f:
            for line in f:
                code = line.split("//", 1)[0].strip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per stage-kernel launch and per stage from the committed counter summary,
    or (None, None) when it was taken on other kernel sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None, None
    txt = open(TRAFFIC_FILE).read()
    m = re.search(r"bytes_per_launch:\s*([0-9.eE+]+)", txt)
    st = re.search(r"bytes_per_stage:\s*([0-9.eE+]+)", txt)
    d = re.search(r"source_digest:\s*([0-9a-f]+)", txt)
    if not m or not st or not d or d.group(1) != stage2d_source_digest():
        return None, None
    return float(m.group(1)), float(st.group(1))


def measured_fp64_flops():
    """FP64 flops per stage-kernel launch from the committed instruction counters, or None
    when they were taken on other kernel sources."""
    if not os.path.exists(FP64_FILE):
        return None
    txt = open(FP64_FILE).read()
    f = re.search(r"fp64_flops_per_launch:\s*([0-9.eE+]+)", txt)
    d = re.search(r"source_digest:\s*([0-9a-f]+)", txt)
    if not f or not d or d.group(1) != stage2d_source_digest():
        return None
    return float(f.group(1))


_SLAB = {}


def _slab_operator(args):
    """L and the limited state of rows j0..j1 of the mesh from the padded slab Up."""
    j0, j1, Up, ax, ay = args
    o = _SLAB["oracle"]
    L, info = o.operator_padded(Up, ax, ay)
    return j0, j1, L, info["Vt"], info["Wt"]


def _slab_pool(procs):
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor
    from threadpoolctl import threadpool_limits
    ctx = multiprocessing.get_context("fork")

    def init():
        threadpool_limits(limits=1)
    return ProcessPoolExecutor(max_workers=procs, mp_context=ctx, initializer=init)


def _oracle_stage(o, U, pool, nslab):
    """One whole-mesh operator evaluation from nslab row slabs (periodic mesh)."""
    import numpy as np
    ax, ay = o.alphas(U)
    n = U.shape[-1]
    cols = np.arange(-3, n + 3) % n
    bounds = np.linspace(0, n, nslab + 1).astype(int)
    jobs = []
    for j0, j1 in zip(bounds[:-1], bounds[1:]):
        rows = np.arange(j0 - 3, j1 + 3) % n
        jobs.append((j0, j1, U[:, :, rows][:, :, :, cols], ax, ay))
    L = np.empty_like(U)
    W = U.copy()
    for j0, j1, Ls, Vt, Wt in (pool.map(_slab_operator, jobs) if pool else map(_slab_operator, jobs)):
        L[:, :, j0:j1] = Ls
        W[1, :, j0:j1] = Vt
        W[2, :, j0:j1] = Wt
    return L, W


def _oracle_steps(o, U0, nsteps, pool, nslab):
    U = U0
    for _ in range(nsteps):
        dt = o.cfl_dt(U, 0.6)
        L0, W0 = _oracle_stage(o, U, pool, nslab)
        L1, W1 = _oracle_stage(o, W0 + dt * L0, pool, nslab)
        L2, W2 = _oracle_stage(o, 0.75 * W0 + 0.25 * W1 + 0.25 * dt * L1, pool, nslab)
        U = W0 / 3.0 + 2.0 / 3.0 * W2 + 2.0 / 3.0 * dt * L2
    return U


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(U0):
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle.scheme2d import Scheme2D
    o = Scheme2D("euler", N, N, ng_edge=2, tc_mode="kxrcf")
    _SLAB["oracle"] = o
    nproc = os.cpu_count() or 1
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = nproc
    # one GPU's share of a multi-GPU host's cores: at most 16 worker processes
    procs = max(1, min(16, avail))
    nsteps = 2
    with _slab_pool(procs) as pool:
        list(pool.map(abs, range(procs)))       # workers started before the clock
        t0 = time.perf_counter()
        U = _oracle_steps(o, U0, nsteps, pool, 4 * procs)
        el = time.perf_counter() - t0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        V = _oracle_steps(o, U0, nsteps, None, 1)
        el1 = time.perf_counter() - t0
    # slabs of other shapes can round differently inside numpy (summation paths depend on
    # the array layout): the two runs agree to rounding, not bit for bit
    assert np.isfinite(U).all()
    assert all(np.abs(U[m, c] - V[m, c]).max() <= 1e-12 * np.abs(V[m, c]).max()
               for m in range(3) for c in range(4))
    sample = f"{nsteps} TVD-RK3 steps ({3 * nsteps} stages) of the {N}x{N} 2D Euler state"
    return {"value": 3 * nsteps * N * N / el, "unit": "cell-stage updates/s", "cores": procs,
            "kind": "oracle",
            "sample": f"{sample}, {el:.1f} s in {procs} single-threaded processes over "
                      f"{4 * procs} row slabs",
            "cpu_model": cpu_model(), "nproc": nproc, "cpus_available": avail,
            "single_thread": {"value": 3 * nsteps * N * N / el1, "cores": 1,
                              "sample": f"{sample}, {el1:.1f} s on one host thread"}}


def timed(stream, fn):
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    stream.synchronize()
    e0.record(stream)
    fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1)


def bench_batched(seed):
    import numpy as np
    import hweno_inputs as hi
    from paper_2002_08816_amd import BatchSolver, Solver
    Us, sizes = hi.batch_euler_1d(seed)
    nsteps = 200
    cells = int(np.sum(sizes))
    bs = BatchSolver(sizes, eq="euler", bc="transmissive", tc_mode="kxrcf")
    # before tuning: 256-cell tiles, one workgroup per tile
    bs.set_states(Us)
    bs.steps(9, persistent=False)         # captures the 8-step and 1-step graphs; warm-up
    bs.set_states(Us)
    ms_np = timed(bs.tstream, lambda: bs.steps(nsteps, persistent=False))
    bs.set_states(Us)
    tile, persist, grid = bs.tune()
    bs.steps(9)
    bs.set_states(Us)
    ms_p = timed(bs.tstream, lambda: bs.steps(nsteps))
    t_p, _ = bs.times()
    bad = [b for b, u in enumerate(bs.get_states()) if not np.isfinite(u).all()]
    bs.close()
    # plain single-instance solver, instance after instance, on a sample
    sample = list(range(0, len(sizes), 16))
    s_cells, ms_plain = 0, 0.0
    for b in sample:
        s = Solver(1, int(sizes[b]), eq="euler", bc="transmissive", tc_mode="kxrcf")
        s.set_state(Us[b])
        s.steps(9)
        s.set_state(Us[b])
        ms_plain += timed(s.tstream, lambda: s.steps(nsteps))
        s_cells += int(sizes[b])
        s.close()
    rate = lambda c, ms: 3.0 * c * nsteps / (ms * 1e-3)
    r_p, r_np, r_plain = rate(cells, ms_p), rate(cells, ms_np), rate(s_cells, ms_plain)
    # algorithmic bytes: 6 FP64 fields read and written per cell-stage, u^n read in stages
    # 2 and 3: 128 B per cell-stage on average
    gbps = r_p * 128.0 / 1e9
    return {
        "workload": f"512 independent 1D Euler instances, N log-uniform in [256, 8192] "
                    f"(sum {cells} cells), transmissive, KXRCF, per-instance CFL dt, "
                    f"{nsteps} steps, captured step graph",
        "value": r_p, "unit": "cell-stage updates/s", "ms_per_step": ms_p / nsteps,
        "tuned": {"tile_cells": tile, "persistent": bool(persist), "grid": grid},
        "untuned_256_cell_tiles": {"value": r_np, "ms_per_step": ms_np / nsteps},
        "plain_one_instance_at_a_time": {"value": r_plain, "instances_sampled": len(sample)},
        "vs_plain": r_p / r_plain,
        "roofline": {"bound": "hbm", "achieved": gbps, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbps / HBM_PEAK_GBS,
                     "basis": "algorithmic 128 B per cell-stage over the whole captured step "
                              "(3 stage launches and the time-step kernel)"},
        "min_final_time": float(np.min(t_p)),
        "finite": not bad,
        # instances whose state lost positivity and became non-finite (the oracle does the
        # same on these inputs: a shock leaving through a transmissive boundary face that is
        # the boundary cell's only inflow face is never flagged under the mirror reading)
        "nonfinite_instances": bad,
    }


def _adjoint_leg(s, U0, nsteps, dt, k):
    import numpy as np
    import torch
    s.set_state(U0)
    s.steps(9, dt)
    s.set_state(U0)
    ms_plain = timed(s.tstream, lambda: s.steps(nsteps, dt))
    s.set_state(U0)
    s.forward_ckpt(nsteps, dt, k)
    lam = torch.from_numpy(np.random.default_rng(1).normal(size=s.shape)).cuda()
    s.adjoint(lam)                                   # warm-up
    s.set_state(U0)
    ms_rec = timed(s.tstream, lambda: s.forward_ckpt(nsteps, dt, k))
    ms_adj = timed(s.tstream, lambda: s.adjoint(lam))
    return {
        "forward_ms_per_step": ms_plain / nsteps,
        "recorded_forward_ms_per_step": ms_rec / nsteps,
        "backward_ms_per_step": ms_adj / nsteps,
        "adjoint_step_over_forward_step": ms_adj / ms_plain,
        "recorded_forward_over_forward": ms_rec / ms_plain,
    }


def bench_adjoint(seed):
    import hweno_inputs as hi
    from paper_2002_08816_amd import Solver
    n, nsteps, k = 256, 200, 20
    dt = 1.0 / (200.0 * math.pi)
    U0, _ = hi.burgers_modes_2d(seed, n=n)
    s = Solver(2, n, n, domain=(0.0, 4.0, 0.0, 4.0), eq="burgers", ng_edge=3, tc_mode="kxrcf")
    res = _adjoint_leg(s, U0, nsteps, dt, k)
    s.close()
    res = {"workload": f"2D Burgers {n}x{n} on [0,4]^2 periodic, NG=3, KXRCF, {nsteps} steps of "
                       f"dt=1/(200 pi), checkpoint every {k}", **res}
    return res


def bench_adjoint_euler(seed):
    """Reverse mode of 2D Euler: the headline shock + vortex state on a 256^2 periodic
    mesh, NG = 2, KXRCF, 100 fixed steps of half the initial CFL step, checkpoints every
    20 steps."""
    import hweno_inputs as hi
    from paper_2002_08816_amd import Solver
    n, nsteps, k = 256, 100, 20
    U0, _ = hi.euler_shock_vortex_2d(seed, n=n)
    s = Solver(2, n, n, eq="euler", ng_edge=2, tc_mode="kxrcf")
    s.set_state(U0)
    ax, ay = s.stats()[0]
    dt = 0.5 * 0.6 / (ax * n + ay * n)
    res = _adjoint_leg(s, U0, nsteps, dt, k)
    s.close()
    return {"workload": f"2D Euler {n}x{n} periodic, shock + isentropic vortex, NG=2, KXRCF, "
                        f"{nsteps} steps of half the initial CFL step, checkpoint every {k}",
            "dt": dt, **res}


def bench_adjoint_step(seed):
    """Reverse mode of 2D Euler on the forward step (Example 3.11 boundaries, the paper's
    corner): 480 x 160 on [0, 3] x [0, 1], NG = 3, KXRCF, the Mach 3 free stream advanced
    on the GPU to T = 0.5 (shocks at the step and the walls), then 40 fixed steps of half
    its CFL step, checkpoints every 20 steps."""
    import hweno_inputs as hi
    from paper_2002_08816_amd import Solver
    nx, ny, nsteps, k = 480, 160, 40, 20
    s = Solver(2, nx, ny, domain=(0.0, 3.0, 0.0, 1.0), eq="euler", ng_edge=3, tc_mode="kxrcf",
               bc="step", step=(0.6, 0.2))
    s.set_state(hi.example_3_11(nx, ny))
    s.run(0.5)
    U0, _ = s.get_state()
    s.set_state(U0)
    ax, ay = s.stats()[0]
    dt = 0.5 * 0.6 / (ax * nx / 3.0 + ay * ny)
    res = _adjoint_leg(s, U0, nsteps, dt, k)
    s.close()
    return {"workload": f"forward step (Example 3.11) {nx}x{ny} on [0,3]x[0,1], NG=3, KXRCF, "
                        f"state at T=0.5, {nsteps} steps of half its CFL step, checkpoint every {k}",
            "dt": dt, **res}


def bench_shock_tests():
    import hweno_inputs as hi
    from paper_2002_08816_amd import Solver
    cases = [
        # the paper's share: cells where the HWENO methodology is used (Lax), troubled
        # cells (Shu-Osher, blast)
        ("lax", "euler", "transmissive", (-0.5, 0.5), 200, 0.16, hi.example_3_6(200), (0.1341, "hybrid")),
        ("shu_osher", "euler", "transmissive", (-5.0, 5.0), 400, 1.8, hi.example_3_7(400), (0.0354, "troubled")),
        ("blast", "euler", "reflective", (0.0, 1.0), 800, 0.038, hi.example_3_8(800), (0.1394, "troubled")),
        ("burgers_shock", "burgers", "periodic", (0.0, 2.0), 80, 1.5 / math.pi, hi.example_3_1(80), None),
    ]
    out = {}
    for name, eq, bc, dom, n, T, U0, paper in cases:
        s = Solver(1, n, domain=dom, eq=eq, bc=bc, tc_mode="kxrcf")
        s.set_state(U0)
        s.run(T)                                   # warm-up (graph capture)
        s.set_state(U0)
        res = {}
        ms = timed(s.tstream, lambda: res.setdefault("r", s.run(T)))
        steps, t = res["r"]
        s.flag_export(True)
        s.set_state(U0)
        flagged, hybrid, k = 0, 0, 0
        while k < steps:
            s.run(T, max_steps=1)
            st = s.stats()
            flagged += sum(st[1])
            hybrid += sum(st[2])
            k += 1
        s.close()
        out[name] = {"cells": n, "T": T, "steps": steps, "ms_to_T": ms,
                     "troubled_share": flagged / (3.0 * steps * n),
                     "hybrid_share": hybrid / (3.0 * steps * n),
                     "paper_share": paper[0] if paper else None,
                     "paper_quantity": paper[1] if paper else None}
    return out


def _bench_2d_shock(workload, nx, ny, domain, bc, U0, T, T_warm, fluid=None):
    """One run of a 2D shock problem to T in one hw_run call (after a short warm-up run that
    captures the step graphs), timed with HIP events on the library's stream; then one step
    with flag export for the troubled and hybrid shares at T (over the fluid cells)."""
    import numpy as np
    from paper_2002_08816_amd import Solver
    s = Solver(2, nx, ny, domain=domain, eq="euler", ng_edge=3, tc_mode="kxrcf", bc=bc)
    s.set_state(U0)
    s.run(T_warm)
    s.set_state(U0)
    res = {}
    ms = timed(s.tstream, lambda: res.setdefault("r", s.run(T)))
    steps, t = res["r"]
    U, _ = s.get_state()
    s.flag_export(True)
    s.step(0.0)
    _, flagged, hybrid = s.stats()
    s.close()
    fl = np.ones((ny, nx), bool) if fluid is None else fluid
    rho = U[0, 0][fl]
    p = 0.4 * (U[0, 3][fl] - 0.5 * (U[0, 1][fl] ** 2 + U[0, 2][fl] ** 2) / rho)
    ncell = int(fl.sum())
    return {"workload": workload, "steps": steps, "ms_to_T": ms, "ms_per_step": ms / steps,
            "cell_stage_updates_per_s": 3.0 * ncell * steps / (ms * 1e-3),
            "troubled_share_at_T": flagged[0] / ncell, "hybrid_share_at_T": hybrid[0] / ncell,
            "positive": bool(rho.min() > 0 and p.min() > 0), "finite": bool(np.isfinite(U).all())}


def bench_dmr():
    """Example 3.10 at the paper's size: 1920 x 480 to T = 0.2, 3-point edge rule."""
    import hweno_inputs as hi
    nx, ny = 1920, 480
    return _bench_2d_shock("double Mach reflection (Example 3.10), 1920x480 on [0,4]x[0,1], NG=3, "
                           "KXRCF, CFL 0.6, to T=0.2", nx, ny, (0.0, 4.0, 0.0, 1.0), "dmr",
                           hi.example_3_10(nx, ny), 0.2, 0.005)


def bench_step():
    """Example 3.11 at the paper's size: 960 x 320 to T = 4, 3-point edge rule (the cell
    count and shares are those of the fluid cells, outside the step)."""
    import numpy as np
    import hweno_inputs as hi
    nx, ny = 960, 320
    jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    fluid = ~((ii >= 192) & (jj < 64))          # the step: x > 0.6, y < 0.2
    return _bench_2d_shock("Mach 3 forward step (Example 3.11), 960x320 on [0,3]x[0,1], NG=3, "
                           "KXRCF, CFL 0.6, to T=4", nx, ny, (0.0, 3.0, 0.0, 1.0), "step",
                           hi.example_3_11(nx, ny), 4.0, 0.01, fluid)


def bench_nonuniform(seed):
    """The 1D Euler Riemann workload (N = 2000, transmissive, KXRCF, CFL 0.6, T = 0.2) on
    a stretched mesh (cell sizes varying smoothly by a factor 1.86, x = s + 0.3 sin(2 pi s)
    / (2 pi)) beside the same data on the uniform mesh: wall time to T (one call, HIP
    events), steps, and the time per step of both."""
    import numpy as np
    import hweno_inputs as hi
    from paper_2002_08816_amd import Solver
    n, T = 2000, 0.2
    prm = hi.euler_riemann_params(np.random.default_rng(2000 + seed))
    f = hi.euler_riemann_func(*prm)
    out = {"workload": f"1D Euler Riemann data, N={n}, transmissive, KXRCF, CFL 0.6, to T={T}"}
    for name, faces in (("stretched", hi.stretched_faces(n, 0.0, 1.0, amp=0.3)),
                        ("uniform", np.linspace(0.0, 1.0, n + 1))):
        U0 = hi.project_1d_faces(f, faces)
        s = Solver(1, n, eq="euler", bc="transmissive", tc_mode="kxrcf")
        if name == "stretched":
            s.set_mesh(faces)
        s.set_state(U0)
        s.run(T)                                    # warm-up (graph capture)
        s.set_state(U0)
        res = {}
        ms = timed(s.tstream, lambda: res.setdefault("r", s.run(T)))
        steps, t = res["r"]
        U, _ = s.get_state()
        s.close()
        out[name] = {"steps": steps, "ms_to_T": ms, "ms_per_step": ms / steps,
                     "max_over_min_cell": float(np.diff(faces).max() / np.diff(faces).min()),
                     "finite": bool(np.isfinite(U).all())}
    return out


def profile_run(seed, leg):
    import numpy as np
    import torch
    import hweno_inputs as hi
    from paper_2002_08816_amd import BatchSolver, Solver
    a = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")   # 256 MiB
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    if leg == "headline":
        U0, _ = hi.euler_shock_vortex_2d(seed, N)
        s = Solver(2, N, N, eq="euler", ng_edge=2, tc_mode="kxrcf")
        s.set_state(U0)
        s.steps(4)
        s.tstream.synchronize()
        s.close()
        print("profile run done: 1 copy of 256 MiB, 12 stages (4 launches each)", flush=True)
    elif leg == "batched":
        Us, sizes = hi.batch_euler_1d(seed)
        bs = BatchSolver(sizes, eq="euler", bc="transmissive", tc_mode="kxrcf")
        bs.set_form(BATCH_FORM[0], BATCH_FORM[1], BATCH_FORM[2])
        bs.set_states(Us)
        bs.steps(4)
        bs.tstream.synchronize()
        bs.close()
        print(f"profile run done: 1 copy of 256 MiB, 12 batched stages ({int(np.sum(sizes))} "
              f"cells, {BATCH_FORM[0]}-cell tiles)", flush=True)
    elif leg == "adjoint_euler":
        n, k = 256, 20
        U0, _ = hi.euler_shock_vortex_2d(seed, n=n)
        s = Solver(2, n, n, eq="euler", ng_edge=2, tc_mode="kxrcf")
        s.set_state(U0)
        ax, ay = s.stats()[0]
        s.forward_ckpt(k, 0.5 * 0.6 / (ax * n + ay * n), k)
        lam = torch.from_numpy(np.random.default_rng(1).normal(size=s.shape)).cuda()
        s.adjoint(lam)
        s.tstream.synchronize()
        s.close()
        print(f"profile run done: 1 copy of 256 MiB, {k} recorded Euler steps and their adjoint",
              flush=True)
    else:
        n, k = 256, 20
        U0, _ = hi.burgers_modes_2d(seed, n=n)
        s = Solver(2, n, n, domain=(0.0, 4.0, 0.0, 4.0), eq="burgers", ng_edge=3,
                   tc_mode="kxrcf")
        s.set_state(U0)
        s.forward_ckpt(k, 1.0 / (200.0 * math.pi), k)
        lam = torch.from_numpy(np.random.default_rng(1).normal(size=s.shape)).cuda()
        s.adjoint(lam)
        s.tstream.synchronize()
        s.close()
        print(f"profile run done: 1 copy of 256 MiB, {k} recorded steps and their adjoint",
              flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch
    import hweno_inputs as hi
    from paper_2002_08816_amd import Solver

    torch.cuda.set_device(0)
    if args.profile_run:
        profile_run(args.seed, args.profile_run)
        return
    U0, prm = hi.euler_shock_vortex_2d(args.seed, N)
    s = Solver(2, N, N, eq="euler", ng_edge=2, tc_mode="kxrcf", bc="periodic")
    s.set_state(U0)
    s.steps(9)                 # captures the 8-step and the 1-step graph
    s.set_state(U0)
    s.steps(args.warmup)
    torch.cuda.synchronize()
    ms = timed(s.tstream, lambda: s.steps(args.steps))
    torch.cuda.synchronize()
    U, t = s.get_state()
    if not np.isfinite(U).all():
        raise RuntimeError("non-finite state after the timed steps")
    # per-stage and per-launch durations (events around every stage and between its launches)
    ms_stage, ms_step, ms_kern = s.profile(10)
    s.flag_export(True)
    s.step(0.0)
    T, H = s.flags(0)
    troubled, hybrid = float(T.mean()), float(H.mean())
    s.close()
    print(f"headline done: {ms / args.steps:.3f} ms/step, {ms_stage:.4f} ms/stage, "
          f"{ms_kern[3]:.4f} ms/stage-kernel launch", file=sys.stderr, flush=True)

    cell_stages = 3.0 * N * N * args.steps
    value = cell_stages / (ms * 1e-3)
    bytes_launch = BYTES_PER_CELL_STAGE * N * N
    achieved = bytes_launch / (ms_kern[3] * 1e-3) / 1e9
    achieved_stage = bytes_launch / (ms_stage * 1e-3) / 1e9
    traffic, traffic_stage = measured_traffic()
    flops = measured_fp64_flops()
    fp64 = None
    if flops is not None:
        tf = flops / (ms_kern[3] * 1e-3) / 1e12
        fp64 = {"kernel": "stage2d_kernel <EULER, NG=2>", "flops_per_launch": flops,
                "achieved_tflops": tf, "peak_tflops": FP64_PEAK_TFLOPS, "frac": tf / FP64_PEAK_TFLOPS}
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-stage updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "2D Euler 1024x1024 periodic, shock + isentropic vortex, "
                               "2-point edge Gauss, KXRCF, CFL 0.6 device dt",
                   "cells": N * N, "fields_per_cell": 12, "seed": args.seed,
                   "troubled_fraction_stage1": troubled, "hybrid_fraction_stage1": hybrid},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "stage2d_kernel <EULER, NG=2>",
                     "ms_per_launch": ms_kern[3],
                     "algorithmic_bytes_per_launch": bytes_launch,
                     "source_digest": stage2d_source_digest(),
                     "stage": {"kernels": "stage2d_flags_kernel + stage2d_limit_kernel + "
                                          "stage2d_hweno_kernel + stage2d_kernel",
                               "ms_per_stage": ms_stage,
                               "ms_per_launch": {"flags": ms_kern[0], "limit": ms_kern[1],
                                                 "hweno": ms_kern[2], "stage_kernel": ms_kern[3]},
                               "achieved": achieved_stage, "frac": achieved_stage / HBM_PEAK_GBS,
                               "traffic": traffic_stage}},
        "fp64": fp64,
    }
    if not args.no_batched:
        out["batched"] = bench_batched(args.seed)
        out["batched"]["vs_headline"] = out["batched"]["value"] / value
        print("batched done", file=sys.stderr, flush=True)
    if not args.no_adjoint:
        out["adjoint"] = bench_adjoint(args.seed)
        out["adjoint_euler"] = bench_adjoint_euler(args.seed)
        out["adjoint_step"] = bench_adjoint_step(args.seed)
        print("adjoint done", file=sys.stderr, flush=True)
    if not args.no_shock_tests:
        out["shock_tests"] = bench_shock_tests()
        print("shock tests done", file=sys.stderr, flush=True)
    if not args.no_dmr:
        out["dmr"] = bench_dmr()
        print("dmr done", file=sys.stderr, flush=True)
    if not args.no_nonuniform:
        out["nonuniform_1d"] = bench_nonuniform(args.seed)
        print("non-uniform mesh done", file=sys.stderr, flush=True)
    if not args.no_step:
        out["forward_step"] = bench_step()
        print("forward step done", file=sys.stderr, flush=True)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(U0)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
