"""Benchmark: coupled-step MLUPS of the Biot LBM on one MI355X.

Workload: the 2D loaded-strip consolidation problem on 512 x 512 cells (unit load
on the central quarter of the top, drained elsewhere on the top, impermeable
rollers on the other sides; E = 1, nu = 0.3, kappa = 1, c0 = 1, alpha = 1;
multigrid with 9 levels, K = 4, gamma = 3/4, 3 V-cycles per step, centred
coupling r = 1/2).  A step is one full coupled time step (explicit force, three
V-cycles, flow update) over the whole grid; inputs are resident in HBM.

Prints one JSON line.  ``value`` is FP32 (shifted storage) MLUPS; the FP64
path is reported beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def _rel(a, b):
    import numpy as np
    return float(np.sqrt(np.sum((a - b) ** 2)) / np.sqrt(np.sum(b * b)))


def time_steps(solver, steps, warmup):
    import torch
    solver.step(warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(solver.stream)
    solver.step(steps)
    ev1.record(solver.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, ev0.elapsed_time(ev1) / 1e3


def cpu_baseline(problem, seconds_target=20.0, max_steps=40):
    """The FP64 oracle on the host's cores, on a bounded number of steps of the
    same workload."""
    from oracle.oracle import Oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    threads = max(1, min(threads, 16))
    o = Oracle(problem, threads=threads)
    t0 = time.perf_counter()
    o.step(1)
    one = time.perf_counter() - t0
    n = int(max(1, min(max_steps, seconds_target / max(one, 1e-6))))
    t0 = time.perf_counter()
    o.step(n)
    dt = time.perf_counter() - t0
    return {"value": problem.ncells * n / dt / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{n} coupled steps of the same 512x512 workload after 1 untimed step, FP64 C oracle, "
                      f"{threads} OpenMP threads"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 run")
    ap.add_argument("--kernel-iters", type=int, default=50)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(problems shard one per GPU; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2409_11382_amd import lbm
    from paper_2409_11382_amd import problem as P

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    lbm.load_library()
    prob = P.loaded_strip(n=args.n, alpha=1.0, ne_fixed=3, K=4)
    N = prob.ncells

    s32 = lbm.Solver(prob, "fp32_shifted")
    wall32, ev32 = time_steps(s32, args.steps, args.warmup)
    mlups32 = N * args.steps / wall32 / 1e6
    # dominant kernel: the finest-level smoothing sweep (HIP events on the solver stream)
    us, nbytes = s32.time_kernel(0, args.kernel_iters)
    achieved = nbytes / (us * 1e-6) / 1e9
    F32 = s32.fields()

    out = {
        "metric": "coupled-step MLUPS (FP32 vs FP64) + batched solves/s and p99 latency",
        "value": round(mlups32, 3),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * wall32 / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"loaded_strip_{args.n}x{args.n}", "alpha": prob.alpha, "nu": 0.3, "E": 1.0,
                   "kappa": float(prob.kappa), "c0": prob.c0, "levels": prob.num_levels(), "K": prob.K,
                   "gamma": prob.gamma, "ne_fixed": prob.ne_fixed, "r": prob.r,
                   "precision": "fp32_shifted (fp64 D, coupling, norms, coarsest)"},
        "roofline": {"bound": "hbm", "kernel": "finest-level smoothing sweep (k_tsweep<float,float,smooth,shift>)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "avg_us": round(us, 3), "bytes_per_launch": nbytes},
        "event_ms_per_step": round(1e3 * ev32 / args.steps, 5),
    }
    if not args.no_fp64:
        s64 = lbm.Solver(prob, "fp64")
        wall64, _ = time_steps(s64, args.steps, args.warmup)
        F64 = s64.fields()
        out["fp64"] = {"value": round(N * args.steps / wall64 / 1e6, 3), "unit": "MLUPS",
                       "ms_per_step": round(1e3 * wall64 / args.steps, 5)}
        out["fp32_shifted_rel_l2_vs_gpu_fp64"] = {k: _rel(F32[k], F64[k]) for k in ("eta", "p")}
        out["fp32_speedup_over_fp64"] = round(wall64 / wall32, 3)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(prob)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
