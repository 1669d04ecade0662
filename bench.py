"""Benchmark: cell updates per second of the FP32 patch update on one MI355X.

Workload (one step = one full pass of ghost fill + wave-propagation update +
friction + positivity + step control over every patch): uniform 2048 x 2048
cells as 64 x 64 patches of 32 x 32 on a 10 km square of seeded fractal
terrain (100 +/- 50 m), circular reservoir of depth 20 m and radius 400 m,
Manning n = 0.033, walls.  Reported beside it: the same run on the FP64
path, the step kernel's HBM roofline fraction (algorithmic 28 B per FP32 cell
update), and the CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np

METRIC = "cell-updates/s and % HBM roofline, FP32-batched AMR vs FP64 plain, 1 MI355X"
HBM_PEAK_GBS = 8000.0
BYTES_PER_UPDATE = {"f32": 28.0, "f64": 56.0}


def workload():
    from paper_2403_15435_amd import inputs
    return inputs.reservoir_fractal(level=6, m=32, L=10000.0, seed=2, radius=400.0, h_res=20.0, manning_n=0.033)


def run_gpu(sc, precision, warmup, steps):
    import torch
    import paper_2403_15435_amd as gf
    ctx = gf.Context([sc], precision=precision, max_patches=4096)
    ctx.set_initial(0)
    ctx.step(warmup)
    torch.cuda.synchronize()
    ctx.profile_enable(True)
    t0 = time.perf_counter()
    st = ctx.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launches, ms = ctx.profile_read()
    ctx.profile_enable(False)
    cells = int(st.cell_updates)
    mass = ctx.mass(0)
    ctx.close()
    return {"wall": wall, "cell_updates": cells, "steps": int(st.steps), "launches": launches,
            "kernel_ms": ms, "rejected": int(st.rejected), "mass": mass.tolist()}


def cpu_baseline(sc, steps=8):
    import oracle
    from paper_2403_15435_amd.inputs import initial_state
    oracle.build(force=False)
    o = oracle.Oracle(sc)
    lv = o.leaves()
    for k in range(lv.shape[0]):
        h, hu, hv = initial_state(sc, lv[k], o.get_field(k, 3), "f64")
        o.set_field(k, 0, np.asarray(h, np.float64))
        o.set_field(k, 1, np.asarray(hu, np.float64))
        o.set_field(k, 2, np.asarray(hv, np.float64))
    t0 = time.perf_counter()
    o.advance(steps)
    dt = time.perf_counter() - t0
    cells = o.steps * lv.shape[0] * sc.m * sc.m
    return {"value": cells / dt, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{o.steps} adaptive steps of the full 2048^2 workload (FP64, one thread), {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--fp64-steps", type=int, default=500)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); multi-GPU sharding is not built", file=sys.stderr)
        sys.exit(2)
    import paper_2403_15435_amd as gf
    sc = workload()
    print(f"[bench] workload ready: {sc.name}, {4096} patches", file=sys.stderr, flush=True)
    r32 = run_gpu(sc, gf.GF_FP32, args.warmup, args.steps)
    print(f"[bench] fp32 done: {r32}", file=sys.stderr, flush=True)
    r64 = run_gpu(sc, gf.GF_FP64, min(args.warmup, 20), args.fp64_steps)
    print(f"[bench] fp64 done: {r64}", file=sys.stderr, flush=True)
    cups32 = r32["cell_updates"] / r32["wall"]
    cups64 = r64["cell_updates"] / r64["wall"]
    cells_per_launch = 4096 * 32 * 32
    avg_launch_s = r32["kernel_ms"] / max(r32["launches"], 1) / 1e3
    achieved = BYTES_PER_UPDATE["f32"] * cells_per_launch / avg_launch_s / 1e9
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(sc)
        print(f"[bench] cpu baseline: {cpu}", file=sys.stderr, flush=True)
    line = {
        "metric": METRIC, "value": cups32, "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * r32["wall"] / max(r32["steps"], 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "uniform 2048x2048 cells (64x64 patches of 32x32), 10 km fractal terrain 100+/-50 m, "
                               "reservoir h=20 m r=400 m, n=0.033, walls, adaptive CFL 0.9",
                   "patches": 4096, "cells": cells_per_launch},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "step_kernel<32,256> (fp32)", "avg_launch_us": avg_launch_s * 1e6},
        "fp64_plain": {"value": cups64, "unit": "cell-updates/s", "steps": r64["steps"],
                       "speedup_fp32_over_fp64": cups32 / cups64},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
