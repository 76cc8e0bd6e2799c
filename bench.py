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
import numpy as np
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "traffic_sweeps_shock_cylinder_1024x512_fp64.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2111_11806_amd", "csrc", f)
                  for f in ("rbdi_api.hip", "rbdi_batch.hpp", "rbdi_kernels.hpp", "rbdi_mlp.hpp", "rbdi_physics.hpp")]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(ncell):
    """HBM bytes of one RK stage (y sweep + x sweep, averages per launch) from
    the rocprofv3 FETCH_SIZE / WRITE_SIZE summary, each counter scaled by what
    it reads for a device copy of known size; None when the summary is
    missing or was taken on other kernel sources, or on another grid."""
    if not os.path.exists(TRAFFIC_PROFILE):
        return None
    kv = {}
    with open(TRAFFIC_PROFILE) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    try:
        if kv.get("source_sha1") != kernel_source_hash() or int(kv["cells"]) != ncell:
            return None
        cb = float(kv["copy_bytes_read"])
        f_scale = cb / (float(kv["copy_fetch_kib"]) * 1024.0)
        w_scale = float(kv["copy_bytes_written"]) / (float(kv["copy_write_kib"]) * 1024.0)
        fetch = (float(kv["sweep_y_fetch_kib"]) + float(kv["sweep_x_fetch_kib"])) * 1024.0 * f_scale
        write = (float(kv["sweep_y_write_kib"]) + float(kv["sweep_x_write_kib"])) * 1024.0 * w_scale
        return fetch + write
    except (KeyError, ValueError, ZeroDivisionError):
        return None


def hbm_copy(nbytes=1 << 30, reps=20):
    """Device-to-device copy of nbytes (torch), GB/s counting read + write."""
    import torch
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    del x, y
    return {"bytes_per_launch": 2 * nbytes, "gbs": round(2 * nbytes * reps / (ms * 1e-3) / 1e9, 1)}


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
    # kernel durations without per-launch event overhead: the sweeps of the
    # middle stage of the last step, replayed back to back on its buffers
    kt["replay_us"] = {"sweep_x": s.kernel_replay(0, 50), "sweep_y": s.kernel_replay(1, 50)}
    return s, ms, wall, st, kt


def run_batched(steps, warmup, precision="fp32"):
    """The 64-instance batch (seed 2111, sizes in {128..512}^2, 1-4 rigid
    ellipses, Mach in [1.5, 3]): autotuned batched launches vs the same
    instances advanced one after another with their own launches."""
    import torch
    from paper_2111_11806_amd import inputs, rbdi
    probs = inputs.batch()
    cells = sum(p.ncells for p in probs)
    cfl = probs[0].cfl
    stream = torch.cuda.current_stream()

    def timed(fn):
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    sv = [rbdi.Solver(p, precision, stream=stream) for p in probs]
    b = rbdi.Batch(sv)
    tune = b.autotune(reps=3)
    b.advance(cfl, warmup)
    ms_b = timed(lambda: b.advance(cfl, steps))
    bad = sum(s.status(raise_on_error=False)["nonphysical"] for s in sv)
    b.close()
    del sv
    sq = [rbdi.Solver(p, precision, stream=stream) for p in probs]
    for s in sq:
        s.advance(cfl, warmup)

    def seq():
        for s in sq:
            s.advance(cfl, steps)
    ms_s = timed(seq)
    del sq
    return {"workload": "batch of 64 shock / rigid-ellipse instances, seed 2111", "instances": len(probs),
            "cells": cells, "steps": steps, "dtype": "f32" if precision == "fp32" else "f64",
            "value": cells * steps / (ms_b * 1e-3), "unit": "cell-updates/s", "ms_per_step": ms_b / steps,
            "sequential_value": cells * steps / (ms_s * 1e-3), "speedup_vs_sequential": ms_s / ms_b,
            "nonphysical_members": int(bad),
            "tuning": {k: (round(v, 2) if isinstance(v, float) else v) for k, v in tune.items()}}


def run_copper(n, steps, warmup):
    """3D copper indenter (n^3): plain FP64 (exact closure) against FP32 with
    the surrogate closure, and the two mixed variants; the network is trained
    first on the solver's own stretches (32^3 run) by the library's kernels."""
    import torch
    from paper_2111_11806_amd import inputs, rbdi, surrogate
    t0 = time.perf_counter()
    V = surrogate.generate(inputs.copper_indenter(32), steps=40, every=10)
    net, info = surrogate.train(V, iters=1500, batch=4096, lr=2e-3, seed=0)
    train_s = time.perf_counter() - t0
    prob = inputs.copper_indenter(n)
    stream = torch.cuda.current_stream()
    out = {"workload": "copper_indenter", "n": n, "cells": prob.ncells, "steps": steps,
           "training": {"samples": info["samples"], "tau_max": info["tau_max"], "iters": len(info["losses"]),
                        "final_loss": float(np.mean(info["losses"][-20:])), "seconds": round(train_s, 2)}}
    for name, prec, surr in (("fp64_exact", "fp64", False), ("fp32_surrogate", "fp32", True),
                             ("fp32_exact", "fp32", False), ("fp64_surrogate", "fp64", True)):
        s = rbdi.Solver(prob, prec, stream=stream)
        if surr:
            s.set_surrogate(net)
        s.advance(prob.cfl, warmup, prob.t_end)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        s.advance(prob.cfl, steps, prob.t_end)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        st = s.status(raise_on_error=False)
        out[name] = {"ms_per_step": round(ms, 3), "value": prob.ncells / (ms * 1e-3),
                     "nonphysical": st["nonphysical"], "surrogate_cells": st["surr_net"],
                     "exact_fallback_cells": st["surr_exact"]}
        s.close()
        del s
    out["speedup_fp32_surrogate_vs_fp64"] = out["fp64_exact"]["ms_per_step"] / out["fp32_surrogate"]["ms_per_step"]
    return out


def run_wedge(steps, warmup, normal="elvira"):
    """Mach 1.7 shock onto the 25-degree wedge, 1200 x 800 (the uniform grid
    of the finest of three levels), ELVIRA normals, FP64, device CFL steps."""
    import torch
    from paper_2111_11806_amd import inputs, rbdi
    prob = inputs.wedge(1200, 800, normal=normal)
    stream = torch.cuda.current_stream()
    s = rbdi.Solver(prob, "fp64", stream=stream)
    s.advance(prob.cfl, warmup, prob.t_end)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    s.advance(prob.cfl, steps, prob.t_end)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    st = s.status(raise_on_error=False)
    out = {"workload": "wedge (Mach 1.7, 25 deg)", "nx": 1200, "ny": 800, "cells": prob.ncells, "normal": normal,
           "dtype": "f64", "steps": steps, "ms_per_step": round(ms, 4), "value": prob.ncells / (ms * 1e-3),
           "unit": "cell-updates/s", "t_reached": st["t"], "band_cells": st["band_cells"],
           "nonphysical": st["nonphysical"]}
    s.close()
    return out


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
    ap.add_argument("--batch-steps", type=int, default=200)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--copper-n", type=int, default=256)
    ap.add_argument("--copper-steps", type=int, default=5)
    ap.add_argument("--no-copper", action="store_true")
    ap.add_argument("--wedge-steps", type=int, default=500)
    ap.add_argument("--no-wedge", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
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
    rx, ry = kt64["replay_us"]["sweep_x"], kt64["replay_us"]["sweep_y"]
    stage_s = (rx + ry) * 1e-6
    achieved = (B64 / 3.0) * ncell / stage_s / 1e9
    traffic = measured_traffic(ncell)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4),
            "traffic": None if traffic is None else round(traffic),
            "algorithmic_bytes_per_stage": round(B64 / 3.0 * ncell),
            "kernel": "one RK stage: k_sweep<y> + k_sweep<x, final> (fp64)",
            "bytes_per_cell_step": B64,
            "avg_us": {"sweep_x": round(rx, 2), "sweep_y": round(ry, 2)},
            "avg_us_dispatch_events": {"sweep_x": round(sx_ms / max(sx_n, 1) * 1e3, 2),
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
           "roofline": roof,
           "hbm_copy": hbm_copy()}

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
                       "avg_us": {"sweep_x": round(kt32["replay_us"]["sweep_x"], 2),
                                  "sweep_y": round(kt32["replay_us"]["sweep_y"], 2)}}

    if not args.no_batch:
        out["batched"] = run_batched(args.batch_steps, 10)

    if not args.no_copper:
        out["copper"] = run_copper(args.copper_n, args.copper_steps, 2)

    if not args.no_wedge:
        out["wedge"] = run_wedge(args.wedge_steps, 20)

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
