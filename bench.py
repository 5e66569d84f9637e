#!/usr/bin/env python3
"""Benchmark of the hybrid HWENO stage operator on one MI355X.

Workload (the headline configuration): 2D Euler (gamma = 1.4) on a 1024 x 1024 uniform
mesh of [0, 1]^2, periodic, averages plus x/y first moments of 4 components (12 FP64
fields per cell), 2-point Gauss rule on edges, KXRCF troubled cells with the limiter and
characteristic HWENO, CFL 0.6 time step computed on the device.  Seeded synthetic
shock-plus-isentropic-vortex initial state (hweno_inputs.euler_shock_vortex_2d).

One benchmark step = one TVD-RK3 step (three fused stage launches and the time-step
launch).  value = cell-stage updates per second = 3 * 1024^2 * K / (time of K steps),
inputs resident in HBM before the timed region.

roofline: algorithmic HBM bytes of the stage kernel per launch (read the stage input and
write the output: 192 B/cell; stages 2 and 3 also read u^n: 288 B/cell; mean 256 B/cell)
divided by the mean stage-kernel duration measured with HIP events on the library's
stream.  cpu_baseline: the CPU oracle (numpy, one thread) on one operator evaluation of
the same 1024^2 state.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
N = 1024
BYTES_PER_CELL_STAGE = 8 * 12 * (2 + 2.0 / 3.0)   # 256 B


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--traffic", default=None,
                    help="JSON file with measured HBM bytes per stage launch (rocprofv3 --pmc)")
    return ap.parse_args()


def cpu_baseline(U0):
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle.scheme2d import Scheme2D
    o = Scheme2D("euler", N, N, ng_edge=2, tc_mode="kxrcf")
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        L, info = o.operator(U0)
        el = time.perf_counter() - t0
    assert np.isfinite(L).all()
    return {"value": N * N / el, "unit": "cell-stage updates/s", "cores": 1, "kind": "oracle",
            "sample": f"one operator evaluation (one stage) of the {N}x{N} 2D Euler state, "
                      f"{el:.1f} s on one host thread"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch
    import hweno_inputs as hi
    from paper_2002_08816_amd import Solver

    torch.cuda.set_device(0)
    U0, prm = hi.euler_shock_vortex_2d(args.seed, N)
    s = Solver(2, N, N, eq="euler", ng_edge=2, tc_mode="kxrcf", bc="periodic")
    s.set_state(U0)
    s.steps(args.warmup)
    torch.cuda.synchronize()
    s.tstream.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(s.tstream)
    s.steps(args.steps)
    ev1.record(s.tstream)
    ev1.synchronize()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    U, t = s.get_state()
    if not np.isfinite(U).all():
        raise RuntimeError("non-finite state after the timed steps")
    # per-launch stage-kernel duration (events around every stage launch)
    ms_stage, ms_step = s.profile(10)
    s.flag_export(True)
    s.step(0.0)
    T, H = s.flags(0)
    troubled = float(T.mean())
    s.close()

    cell_stages = 3.0 * N * N * args.steps
    value = cell_stages / (ms * 1e-3)
    bytes_launch = BYTES_PER_CELL_STAGE * N * N
    achieved = bytes_launch / (ms_stage * 1e-3) / 1e9
    traffic = None
    if args.traffic and os.path.exists(args.traffic):
        traffic = json.load(open(args.traffic)).get("bytes_per_launch")
    out = {
        "metric": "FP64 cell-stage updates/s, 2D Euler 1024^2",
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
                   "troubled_fraction_stage1": troubled},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "stage2d_kernel<EULER, NG=2>", "ms_per_launch": ms_stage,
                     "algorithmic_bytes_per_launch": bytes_launch},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(U0)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
