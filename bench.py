#!/usr/bin/env python
"""Throughput of the diffuse-interface rigid-body step on one MI355X.

Headline workload (the configuration the metric compares plain FP64 with
FP32 + surrogate on): 3D elastoplastic copper (Romenskii, rho0 8930, G0
46 GPa, perfect plasticity 0.12 GPa) below air, 256^3 cells on a 25.6 mm
cube, a rigid flat-ended cylinder (radius 20 cells) pressed in at 200 m/s;
MUSCL-BVD-THINC, HLLC, Youngs normals, original seeding, CFL 0.3. Every leg
first advances past contact (t = 0.6 us; the flat end meets the copper at
0.5 us), so the plastic return and the surrogate run under load, then does
W untimed and K timed steps.

A step is one whole time step of the hot path: rigid band + seeding, three
SSP-RK3 stages of direction sweeps (z, y, then x with the RK combine and the
elastoplastic sources), and the device-side CFL reduction that sets dt (no
host synchronisation inside the timed region).

value: cell-updates/s of the plain FP64 path (exact closure). Beside it:
FP32 with the surrogate closure (its speedup over plain FP64 and its
per-field relative L1 / Linf against FP64 after a common dt sequence), FP32
with the exact closure, the roofline of one RK stage, the 1024 x 512 Mach 2.8
shock / cylinder workload (FP64 and FP32), the 64-instance batch, the wedge,
the extrusion with a piston (two rigid motions), and the CPU oracle on the
host.
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
TRAFFIC_CYLINDER = os.path.join(ROOT, "profiles", "traffic_sweeps_shock_cylinder_1024x512_fp64.txt")
TRAFFIC_COPPER = os.path.join(ROOT, "profiles", "traffic_sweeps_copper_indenter_256_fp64.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2111_11806_amd", "csrc", f)
                  for f in ("rbdi_api.hip", "rbdi_batch.hpp", "rbdi_kernels.hpp", "rbdi_mlp.hpp", "rbdi_physics.hpp")]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(path, ncell, sweeps):
    """HBM bytes of one RK stage (the named sweeps, averages per launch) from
    a rocprofv3 FETCH_SIZE / WRITE_SIZE summary under profiles/, each counter
    scaled by what it reads for a device copy of known size; None when the
    summary is missing or was taken on other kernel sources, or on another
    grid."""
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    try:
        if kv.get("source_sha1") != kernel_source_hash() or int(kv["cells"]) != ncell:
            return None
        f_scale = float(kv["copy_bytes_read"]) / (float(kv["copy_fetch_kib"]) * 1024.0)
        w_scale = float(kv["copy_bytes_written"]) / (float(kv["copy_write_kib"]) * 1024.0)
        fetch = sum(float(kv[f"{k}_fetch_kib"]) for k in sweeps) * 1024.0 * f_scale
        write = sum(float(kv[f"{k}_write_kib"]) for k in sweeps) * 1024.0 * w_scale
        return round(fetch + write)
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
    t_start = s.status()["t"]
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
    st["t_start"] = t_start
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


COPPER_PREROLL_T = 0.6e-6  # past the contact at 0.5 us


def stage_roofline(ms_stage_us, bytes_per_cell_step, ncell, kernel, avg_us, traffic=None, design_bytes=None):
    """HBM roofline of one RK stage: algorithmic bytes (one third of the
    per-step bytes) over the summed durations of the stage's sweeps.
    design_bytes: what the direction-split sweeps move by design (each sweep
    reads the stage input, the y/x sweeps read the accumulator D the earlier
    ones wrote, the x sweep U^n), the measured traffic's reference."""
    achieved = (bytes_per_cell_step / 3.0) * ncell / (ms_stage_us * 1e-6) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
            "algorithmic_bytes_per_stage": round(bytes_per_cell_step / 3.0 * ncell),
            "design_bytes_per_stage": design_bytes,
            "bytes_per_cell_step": bytes_per_cell_step, "kernel": kernel,
            "avg_us": {k: round(v, 2) for k, v in avg_us.items()}}


def design_bytes_per_stage(dim, nfields, elem, ncell):
    """Plane accesses per field and stage of the direction-split sweeps: 3D
    z (read U, write D), y (read U, D; write D), x (read U, U^n, D; write
    U): 9; 2D y + x: 6."""
    return (9 if dim == 3 else 6) * nfields * elem * ncell


def copper_leg(prob, precision, net, steps, warmup, stream):
    """One leg of the copper workload: pre-roll past contact, W untimed and K
    timed device-CFL steps, per-kernel times (dispatch events) and the
    sweeps of one stage replayed back to back."""
    import torch
    from paper_2111_11806_amd import rbdi
    s = rbdi.Solver(prob, precision, stream=stream)
    if net is not None:
        s.set_surrogate(net)
    s.advance(prob.cfl, 400, COPPER_PREROLL_T)  # steps after t_end do no work
    # the library's autotuner: x-sweep block size from timed steps of this
    # state (restored after each trial)
    x_waves, _ = s.autotune(prob.cfl, nsteps=3)
    s.advance(prob.cfl, warmup, 0.0)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    st0 = s.status(raise_on_error=False)
    e0.record(stream)
    s.advance(prob.cfl, steps, 0.0)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    st = s.status(raise_on_error=False)
    s.set_kernel_timing(True)
    s.advance(prob.cfl, 2, 0.0)
    kt = s.kernel_times()
    s.set_kernel_timing(False)
    rep = {"sweep_x": s.kernel_replay(0, 10), "sweep_y": s.kernel_replay(1, 10), "sweep_z": s.kernel_replay(2, 10)}
    out = {"ms_per_step": round(ms, 3), "value": prob.ncells / (ms * 1e-3), "x_waves": x_waves,
           "t_start_timed": st0["t"], "t_end_timed": st["t"], "nonphysical": st["nonphysical"],
           "surrogate_closures": st["surr_net"], "exact_fallback_closures": st["surr_exact"],
           "replay_us": {k: round(v, 1) for k, v in rep.items()},
           "dispatch_us": {k: round(kt[k][0] / max(kt[k][1], 1) * 1e3, 1) for k in ("sweep_x", "sweep_y", "sweep_z",
                                                                              "seed", "band")}}
    s.close()
    return out


def field_errors(ua, ub, names, keep):
    """Per conserved field over the cells where keep: relative L1 and Linf of
    ub against ua (components of a vector or tensor judged against at least
    1% of their family's mean norm, as the parity tests do)."""
    fam = {n: [i for i, m in enumerate(names) if (m in ("mx", "my", "mz")) == (n in ("mx", "my", "mz"))
               and (m.startswith("V") and len(m) == 3) == (n.startswith("V") and len(n) == 3)] for n in names}
    a = np.where(keep, ua, 0.0)
    b = np.where(keep, ub, 0.0)
    out = {}
    for q, n in enumerate(names):
        d = np.abs(b[q] - a[q])
        n1 = np.abs(a[q]).sum()
        f1 = 0.01 * np.mean([np.abs(a[i]).sum() for i in fam[n]])
        ninf = np.abs(a[q]).max()
        finf = 0.01 * max(np.abs(a[i]).max() for i in fam[n])
        out[n] = {"l1": float(d.sum() / max(n1, f1, 1e-300)), "linf": float(d.max() / max(ninf, finf, 1e-300))}
    return out


COPPER_PRECONTACT_T = 0.45e-6  # the flat end meets the copper at 0.5 us


def copper_accuracy(prob, net, nsteps, stream):
    """FP32 + surrogate and FP32 exact against plain FP64 over a common dt
    sequence (FP64's CFL dt each step) from t = 0 through the contact, per
    conserved field over the non-rigid cells (rigid cells hold seeded ghost
    states), beside the floor that FP32 storage of the state alone sets: the
    FP64 path with its state rounded to FP32 after every step (rounded on
    the device). Reported just before the contact (t = 0.45 us), after
    nsteps steps (t past the contact), and for one further step of the FP32
    paths from the FP64 state (the error a single step adds)."""
    import torch
    from paper_2111_11806_amd import rbdi
    a = rbdi.Solver(prob, "fp64", stream=stream)
    b = rbdi.Solver(prob, "fp32", stream=stream)
    b.set_surrogate(net)
    e = rbdi.Solver(prob, "fp32", stream=stream)
    c = rbdi.Solver(prob, "fp64", stream=stream)
    buf = torch.empty(a.shape, dtype=torch.float64, device="cuda")
    names = prob.cons_names()
    ir = names.index("r")

    def report():
        ua = a.get_state_cons()
        keep = ua[ir] <= 0.5
        return {"t": a.t, "surrogate_fp32": field_errors(ua, b.get_state_cons(), names, keep),
                "exact_fp32": field_errors(ua, e.get_state_cons(), names, keep),
                "fp32_storage_floor": field_errors(ua, c.get_state_cons(), names, keep)}

    out = {}
    t, k = 0.0, 0
    while t < COPPER_PREROLL_T or k < nsteps:
        dt = a.compute_dt(prob.cfl)
        if t < COPPER_PRECONTACT_T <= t + dt:
            out["before_contact"] = dict(report(), steps=k)
        for s in (a, b, e, c):
            s.step(dt)
        c.get_state_cons_device(buf.data_ptr())
        buf.copy_(buf.float().double())
        c.set_state_cons_device(buf.data_ptr())
        t += dt
        k += 1
    out["through_contact"] = dict(report(), steps=k)
    # one step of the FP32 paths from the FP64 state (their own times match:
    # they took the same dt sequence): the error a single step adds
    ua = a.get_state_cons()
    b.set_state_cons(ua)
    e.set_state_cons(ua)
    dt = a.compute_dt(prob.cfl)
    for s in (a, b, e):
        s.step(dt)
    ua = a.get_state_cons()
    keep = ua[ir] <= 0.5
    out["one_step_from_fp64_state"] = {"t": a.t, "surrogate_fp32": field_errors(ua, b.get_state_cons(), names, keep),
                                       "exact_fp32": field_errors(ua, e.get_state_cons(), names, keep)}
    for s in (a, b, e, c):
        s.close()
    return out


COPPER_LEGS = ("fp64_exact", "fp32_surrogate", "fp32_exact")


def run_copper(n, steps, warmup, accuracy_steps=100, legs_wanted=COPPER_LEGS):
    """The copper workload: plain FP64, FP32 + surrogate, FP32 exact; the
    network is trained first on the solver's own stretches (a 32^3 run) by
    the library's kernels. accuracy_steps = 0 skips the accuracy run."""
    import torch
    from paper_2111_11806_amd import inputs, surrogate
    net, training = None, None
    if "fp32_surrogate" in legs_wanted or accuracy_steps > 0:
        t0 = time.perf_counter()
        V = surrogate.generate(inputs.copper_indenter(32), steps=40, every=10)
        net, info = surrogate.train(V, iters=1500, batch=4096, lr=2e-3, seed=0)
        training = {"samples": info["samples"], "tau_max": info["tau_max"], "iters": len(info["losses"]),
                    "final_loss": float(np.mean(info["losses"][-20:])),
                    "seconds": round(time.perf_counter() - t0, 2)}
    prob = inputs.copper_indenter(n)
    stream = torch.cuda.current_stream()
    legs = {}
    for name, prec, surr in (("fp64_exact", "fp64", False), ("fp32_surrogate", "fp32", True),
                             ("fp32_exact", "fp32", False)):
        if name in legs_wanted:
            legs[name] = copper_leg(prob, prec, net if surr else None, steps, warmup, stream)
    acc = copper_accuracy(prob, net, accuracy_steps, stream) if accuracy_steps > 0 else None
    return prob, legs, acc, training


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


def run_extrusion(steps, warmup):
    """Extrusion of an aluminium block by a piston through a static wedge
    (two rigid bodies with their own motion), 2048 x 1728 (the finest of
    four levels on the 256 x 216 base grid, as a uniform grid), FP64 and
    FP32, device CFL steps from t = 0."""
    import torch
    from paper_2111_11806_amd import inputs, rbdi
    prob = inputs.extrusion()
    stream = torch.cuda.current_stream()
    out = {"workload": "extrusion (Al, piston 100 m/s, 15 deg wedge)", "nx": prob.n[0], "ny": prob.n[1],
           "cells": prob.ncells, "bodies": 1 + len(prob.bodies), "steps": steps, "unit": "cell-updates/s"}
    for prec in ("fp64", "fp32"):
        s = rbdi.Solver(prob, prec, stream=stream)
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
        out[prec] = {"ms_per_step": round(ms, 4), "value": prob.ncells / (ms * 1e-3), "t_reached": st["t"],
                     "nonphysical": st["nonphysical"]}
        s.close()
    return out


def run_slab_wall(steps, n=1024, ntrans=1024):
    """The void-opening face modifier at work: a 2D elastic copper slab
    across y (n cells along y, ntrans along x, periodic in x) that has struck
    a static rigid wall at 20 m/s, FP64, timed over `steps` device CFL steps
    from 0.95 of its contact time 2 L / c_L (the slab leaves the wall in
    them), with the modifier on and, for its cost, off (the wall then holds
    the slab)."""
    import torch
    from paper_2111_11806_amd import inputs, rbdi
    prob = inputs.copper_slab_wall(n=n, dim=2, axis=1, ntrans=ntrans)
    tc = 2.0 * 6e-3 / inputs.longitudinal_wave_speed(prob.materials[0])
    dt_est = prob.cfl * prob.dx[1] / inputs.longitudinal_wave_speed(prob.materials[0])
    stream = torch.cuda.current_stream()
    out = {"workload": "copper slab rebounding from a rigid wall (2D, 20 m/s)", "nx": prob.n[0], "ny": prob.n[1],
           "cells": prob.ncells, "dtype": "f64", "steps": steps, "unit": "cell-updates/s",
           "timed_from_t_over_contact_time": 0.95}
    for mode in (1, 0):
        s = rbdi.Solver(prob, "fp64", stream=stream)
        s.set_face_modifier(mode, prob.gap_gas)
        s.advance(prob.cfl, int(1.2 * 0.95 * tc / dt_est) + 10, 0.95 * tc)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        s.advance(prob.cfl, steps, 2.0 * tc)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        st = s.status(raise_on_error=False)
        out["modifier_on" if mode else "modifier_off"] = {"ms_per_step": round(ms, 4),
                                                          "value": prob.ncells / (ms * 1e-3),
                                                          "t_over_contact_time": st["t"] / tc,
                                                          "nonphysical": st["nonphysical"]}
        s.close()
    out["modifier_cost"] = out["modifier_on"]["ms_per_step"] / out["modifier_off"]["ms_per_step"] - 1.0
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(seconds):
    """The CPU FP64 oracle on the host (never tuned for speed), on bounded
    samples of the headline workload: the same copper indenter on a 64^3 grid
    (the oracle's cost per cell does not depend on the grid size), first with
    every host thread, then with one thread on a 32^3 grid."""
    import oracle
    from paper_2111_11806_amd import inputs
    out = {}
    for label, n, threads in (("all_threads", 64, os.cpu_count() or 1), ("one_thread", 32, 1)):
        oracle.set_threads(threads)
        prob = inputs.copper_indenter(n)
        o = oracle.Oracle(prob)
        o.step(o.compute_dt(prob.cfl))  # first step (allocation, first touch) untimed
        nsteps = 0
        t0 = time.perf_counter()
        while True:
            o.step(o.compute_dt(prob.cfl))
            nsteps += 1
            if time.perf_counter() - t0 > seconds or nsteps >= 200:
                break
        el = time.perf_counter() - t0
        out[label] = {"value": prob.ncells * nsteps / el, "cores": oracle.get_threads(),
                      "sample": "copper indenter %d^3, steps 2-%d from t = 0 (oracle CFL dt), %.1f s"
                                % (n, nsteps + 1, el)}
        del o
    oracle.set_threads(os.cpu_count() or 1)
    return out


def run_shock_cylinder(nx, ny, steps, warmup):
    """The 2D Mach 2.8 shock / rigid cylinder workload (FP64 and FP32)."""
    from paper_2111_11806_amd import inputs, rbdi
    prob = inputs.shock_cylinder(nx, ny)
    ncell = prob.ncells
    cfl = prob.cfl
    timing_steps = max(20, min(200, steps // 5))
    s64, ms64, wall64, st64, kt64 = run_gpu(prob, "fp64", steps, warmup, cfl, timing_steps)
    B64 = algorithmic_bytes_per_cell_step(4, 1, 8)
    rx, ry = kt64["replay_us"]["sweep_x"], kt64["replay_us"]["sweep_y"]
    traffic = measured_traffic(TRAFFIC_CYLINDER, ncell, ("sweep_y", "sweep_x"))
    roof = stage_roofline(rx + ry, B64, ncell, "one RK stage: k_sweep_tile<y> + k_sweep_x (fp64)",
                          {"sweep_x": rx, "sweep_y": ry}, traffic, design_bytes_per_stage(2, 5, 8, ncell))
    out = {"workload": "shock_cylinder", "nx": nx, "ny": ny, "cells": ncell, "dtype": "f64", "steps": steps,
           "warmup": warmup, "ms_per_step": ms64 / steps, "value": ncell * steps / (ms64 * 1e-3),
           "unit": "cell-updates/s", "t_start_timed": st64["t_start"], "t_reached": st64["t"],
           "flow_state": "timed from t = %.4g (after %d warm-up steps from t = 0) to t = %.4g; the roofline's "
                         "kernel durations are replays of the last step's middle stage" % (
                             st64["t_start"], warmup, st64["t"]),
           "roofline": roof}
    s32, ms32, wall32, st32, kt32 = run_gpu(prob, "fp32", steps, warmup, cfl, timing_steps)
    v32 = ncell * steps / (ms32 * 1e-3)
    a = rbdi.Solver(prob, "fp64")
    b = rbdi.Solver(prob, "fp32")
    dt = 0.9 * a.compute_dt(cfl)
    for _ in range(200):
        a.step(dt)
        b.step(dt)
    ua, ub = a.get_state_cons(), b.get_state_cons()
    num = np.abs(ua - ub).reshape(ua.shape[0], -1)
    den = np.abs(ua).reshape(ua.shape[0], -1)
    out["fp32"] = {"value": v32, "ms_per_step": ms32 / steps, "speedup_vs_fp64": v32 / out["value"],
                   "vs_fp64_after_200_fixed_dt_steps": {
                       n: {"l1": float(num[q].sum() / max(den[q].sum(), 1e-300)),
                           "linf": float(num[q].max() / max(den[q].max(), 1e-300))}
                       for q, n in enumerate(prob.cons_names())},
                   "avg_us": {"sweep_x": round(kt32["replay_us"]["sweep_x"], 2),
                              "sweep_y": round(kt32["replay_us"]["sweep_y"], 2)}}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed steps of the headline (copper) legs")
    ap.add_argument("--warmup", type=int, default=5, help="untimed steps after the pre-roll past contact")
    ap.add_argument("--copper-n", type=int, default=256)
    ap.add_argument("--accuracy-steps", type=int, default=100,
                    help="steps of the FP32 + surrogate vs FP64 comparison after contact (0: skip)")
    ap.add_argument("--copper-legs", default=",".join(COPPER_LEGS),
                    help="comma list of copper legs to run, or none (profiling runs); the JSON line "
                         "needs all three")
    ap.add_argument("--nx", type=int, default=1024)
    ap.add_argument("--ny", type=int, default=512)
    ap.add_argument("--cyl-steps", type=int, default=1000)
    ap.add_argument("--cyl-warmup", type=int, default=100)
    ap.add_argument("--no-cylinder", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=200)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--wedge-steps", type=int, default=500)
    ap.add_argument("--no-wedge", action="store_true")
    ap.add_argument("--extrusion-steps", type=int, default=300)
    ap.add_argument("--no-extrusion", action="store_true")
    ap.add_argument("--slab-steps", type=int, default=300)
    ap.add_argument("--no-slab", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    wanted = tuple(x for x in args.copper_legs.split(",") if x and x != "none")
    if set(wanted) != set(COPPER_LEGS):
        # a profiling run: the legs it names (none, or some copper legs, and
        # the shock/cylinder workload unless --no-cylinder), their timings and
        # the device copy that scales the traffic counters; no headline line
        out = {}
        if wanted:
            _, legs, _, _ = run_copper(args.copper_n, args.steps, args.warmup, 0, wanted)
            out["legs"] = {k: {"ms_per_step": v["ms_per_step"], "replay_us": v["replay_us"]}
                           for k, v in legs.items()}
        if not args.no_cylinder:
            c = run_shock_cylinder(args.nx, args.ny, args.cyl_steps, args.cyl_warmup)
            out["shock_cylinder"] = {"ms_per_step": c["ms_per_step"], "avg_us": c["roofline"]["avg_us"]}
        out["hbm_copy"] = hbm_copy()
        print(json.dumps(out))
        return
    prob, legs, acc, training = run_copper(args.copper_n, args.steps, args.warmup, args.accuracy_steps, wanted)
    ncell = prob.ncells
    L64, Ls, L32 = legs["fp64_exact"], legs["fp32_surrogate"], legs["fp32_exact"]
    n_dyn = prob.nfields  # every field of the elastoplastic system is dynamic (r moves with the body)
    B64 = algorithmic_bytes_per_cell_step(n_dyn, 0, 8)
    B32 = algorithmic_bytes_per_cell_step(n_dyn, 0, 4)

    def leg_roof(L, B, dtype):
        r = L["replay_us"]
        traffic = (measured_traffic(TRAFFIC_COPPER, ncell, ("sweep_z", "sweep_y", "sweep_x"))
                   if dtype == "f64" else None)
        return stage_roofline(r["sweep_x"] + r["sweep_y"] + r["sweep_z"], B, ncell,
                              "one RK stage: k_sweep_tile<z> + k_sweep_tile<y> + k_sweep_x%s (%s)"
                              % ("_surr" if dtype == "f32+surrogate" else "", dtype), r, traffic,
                              design_bytes_per_stage(3, prob.nfields, 8 if dtype == "f64" else 4, ncell))

    def worst_l1(part):
        return max(part.values(), key=lambda v: v["l1"])["l1"]

    stated = None
    if acc is not None:
        stated = {when: {"fp32_surrogate_vs_fp64_max_l1": worst_l1(acc[when]["surrogate_fp32"]),
                         "fp32_storage_floor_max_l1": worst_l1(acc[when]["fp32_storage_floor"]),
                         "t": acc[when]["t"], "steps": acc[when]["steps"]}
                  for when in ("before_contact", "through_contact") if when in acc}
        one = acc["one_step_from_fp64_state"]
        stated["one_step_from_fp64_state"] = {"fp32_surrogate_vs_fp64_max_l1": worst_l1(one["surrogate_fp32"]),
                                              "fp32_exact_vs_fp64_max_l1": worst_l1(one["exact_fp32"]),
                                              "t": one["t"]}
    out = {"metric": "cell-updates/s per step (FP32+surrogate vs FP64 plain) at stated L1 error; HBM GB/s %",
           "value": L64["value"], "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": L64["ms_per_step"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "copper_indenter", "n": args.copper_n, "cells": ncell,
                      "materials": "copper (Romenskii, rho0 8930, G0 46 GPa, yield 0.12 GPa) + air",
                      "indenter": "flat-ended rigid cylinder, radius 20 cells, -200 m/s",
                      "recon": prob.recon, "riemann": prob.riemann, "cfl": prob.cfl,
                      "timed_from_t": L64["t_start_timed"], "timed_to_t": L64["t_end_timed"]},
           "roofline": leg_roof(L64, B64, "f64"),
           "stated_l1_error": stated,
           "fp64_exact": L64,
           "fp32_surrogate": dict(Ls, speedup_vs_fp64=L64["ms_per_step"] / Ls["ms_per_step"],
                                  dtype="f32 (FP64 pressure, dt, reductions) + BF16 network",
                                  roofline=leg_roof(Ls, B32, "f32+surrogate"),
                                  vs_fp64=acc, training=training),
           "fp32_exact": dict(L32, speedup_vs_fp64=L64["ms_per_step"] / L32["ms_per_step"],
                              roofline=leg_roof(L32, B32, "f32")),
           "hbm_copy": hbm_copy()}

    if not args.no_cylinder:
        out["shock_cylinder"] = run_shock_cylinder(args.nx, args.ny, args.cyl_steps, args.cyl_warmup)
    if not args.no_batch:
        out["batched"] = run_batched(args.batch_steps, 10)
    if not args.no_wedge:
        out["wedge"] = run_wedge(args.wedge_steps, 20)
    if not args.no_extrusion:
        out["extrusion"] = run_extrusion(args.extrusion_steps, 10)
    if not args.no_slab:
        out["face_modifier"] = run_slab_wall(args.slab_steps)
    if not args.no_cpu_baseline:
        cb = cpu_baseline(args.cpu_seconds)
        a = cb["all_threads"]
        out["cpu_baseline"] = {"value": a["value"], "unit": "cell-updates/s", "cores": a["cores"],
                               "kind": "oracle", "sample": a["sample"], "cpu_model": cpu_model(),
                               "one_thread": cb["one_thread"]}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
