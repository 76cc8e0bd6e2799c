#!/usr/bin/env python
"""Throughput of the diffuse-interface rigid-body step on one MI355X.

Workload: Mach 2.8 planar shock (ideal gas, gamma 1.4, pre-shock rho = 1,
p = 1) over a static rigid cylinder (radius 0.1 at (0.3, 0.25)) on a uniform
1024 x 512 grid on [0,1] x [0,0.5]; r from the signed distance with a two-cell
tanh width; MUSCL-BVD-THINC, HLLC-LM, Youngs normals, original seeding, CFL 0.4.
A step is one whole time step of the hot path: rigid band + seeding, three
SSP-RK3 stages of direction sweeps with the RK combine, and the device-side
CFL reduction that sets dt (no host synchronisation inside the timed region).

value: cell-updates/s of the plain FP64 path (interior cells x steps / time).
The FP32 path runs the same steps and is reported beside it, with its
relative L1 difference from the FP64 path after a common fixed-dt sequence.
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

PEAK_HBM_GBS = 8000.0


def algorithmic_bytes_per_cell_step(n_dyn, n_static, elem):
    """Per step: 3 stage reads of the input state, 2 reads of U^n (stages 2
    and 3), 3 writes of the dynamic fields; static fields read 3 times."""
    return elem * (8 * n_dyn + 3 * n_static)


def run_gpu(prob, precision, steps, warmup, cfl, timing_steps):
    import torch
    from paper_2111_11806_amd import rbdi
    stream = torch.cuda.current_stream()
    s = rbdi.Solver(prob, precision, stream=stream)
    s.advance(cfl, warmup, 0.0)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    s.advance(cfl, steps, 0.0)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    st = s.status()
    # per-kernel durations, recorded live with HIP event pairs on the same
    # stream over a further stretch of the same run
    s.set_kernel_timing(True)
    s.advance(cfl, timing_steps, 0.0)
    kt = s.kernel_times()
    s.set_kernel_timing(False)
    return s, ms, wall, st, kt


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--nx", type=int, default=1024)
    ap.add_argument("--ny", type=int, default=512)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    from paper_2111_11806_amd import inputs, rbdi

    prob = inputs.shock_cylinder(args.nx, args.ny)
    ncell = prob.ncells
    cfl = prob.cfl
    timing_steps = max(20, min(200, args.steps // 5))

    s64, ms64, wall64, st64, kt64 = run_gpu(prob, "fp64", args.steps, args.warmup, cfl, timing_steps)
    value = ncell * args.steps / (ms64 * 1e-3)

    # roofline of one RK stage of the sweeps (the y sweep and the final x
    # sweep together), algorithmic bytes = one third of the per-step bytes
    n_dyn, n_static = 4, 1
    B64 = algorithmic_bytes_per_cell_step(n_dyn, n_static, 8)
    sx_ms, sx_n = kt64["sweep_x"]
    sy_ms, sy_n = kt64["sweep_y"]
    stage_s = (sx_ms / max(sx_n, 1) + sy_ms / max(sy_n, 1)) * 1e-3
    achieved = (B64 / 3.0) * ncell / stage_s / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None,
            "kernel": "one RK stage: k_sweep<y> + k_sweep<x, final> (fp64)",
            "bytes_per_cell_step": B64,
            "avg_us": {"sweep_x": round(sx_ms / max(sx_n, 1) * 1e3, 2),
                       "sweep_y": round(sy_ms / max(sy_n, 1) * 1e3, 2),
                       "seed": round(kt64["seed"][0] / max(kt64["seed"][1], 1) * 1e3, 2),
                       "cfl_dt": round(kt64["cfl_dt"][0] / max(kt64["cfl_dt"][1], 1) * 1e3, 2)}}

    out = {"metric": "cell-updates/s per step (FP64 plain; FP32 beside it) on the 1024x512 "
                     "Mach 2.8 shock / rigid cylinder workload; HBM GB/s % of peak",
           "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms64 / args.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "shock_cylinder", "nx": args.nx, "ny": args.ny, "cells": ncell,
                      "mach": 2.8, "cfl": cfl, "recon": prob.recon, "riemann": prob.riemann,
                      "t_reached": st64["t"]},
           "roofline": roof}

    if not args.no_fp32:
        s32, ms32, wall32, st32, kt32 = run_gpu(prob, "fp32", args.steps, args.warmup, cfl, timing_steps)
        v32 = ncell * args.steps / (ms32 * 1e-3)
        # L1 difference of FP32 from FP64 after the same fixed-dt sequence
        a = rbdi.Solver(prob, "fp64")
        b = rbdi.Solver(prob, "fp32")
        dt = 0.9 * a.compute_dt(cfl)
        for _ in range(200):
            a.step(dt)
            b.step(dt)
        ua, ub = a.get_state_cons(), b.get_state_cons()
        num = np.abs(ua - ub).reshape(ua.shape[0], -1).sum(1)
        den = np.maximum(np.abs(ua).reshape(ua.shape[0], -1).sum(1), 1e-300)
        rel = num / den
        out["fp32"] = {"value": v32, "ms_per_step": ms32 / args.steps, "speedup_vs_fp64": v32 / value,
                       "rel_l1_vs_fp64_after_200_fixed_dt_steps": {n: float(x) for n, x in
                                                                   zip(prob.cons_names(), rel)},
                       "avg_us": {"sweep_x": round(kt32["sweep_x"][0] / max(kt32["sweep_x"][1], 1) * 1e3, 2),
                                  "sweep_y": round(kt32["sweep_y"][0] / max(kt32["sweep_y"][1], 1) * 1e3, 2)}}

    if not args.no_cpu_baseline:
        import oracle
        o = oracle.Oracle(prob)
        nsteps = 0
        t0 = time.perf_counter()
        while True:
            o.step(o.compute_dt(cfl))
            nsteps += 1
            if time.perf_counter() - t0 > args.cpu_seconds or nsteps >= 200:
                break
        cpu_s = time.perf_counter() - t0
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        out["cpu_baseline"] = {"value": ncell * nsteps / cpu_s, "unit": "cell-updates/s", "cores": threads,
                               "kind": "oracle",
                               "sample": "the same 1024x512 workload, first %d steps from t=0 (CFL dt "
                                         "computed by the oracle), %.1f s, OpenMP threads=%d"
                                         % (nsteps, cpu_s, threads)}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
