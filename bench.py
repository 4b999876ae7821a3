#!/usr/bin/env python3
"""Benchmark of the stencil sweep on one MI355X.

A bench "step" is one whole run of the workload: 100 fused-or-not time steps
of the 3D 7-point heat stencil on a 512^3 FP64 grid (zero-Dirichlet ghost
layer, alpha = 0.15, U[0,1) initial field plus one sin mode), i.e. every
stage of the hot path (plan choice, halo-tile loads, register/DPP pattern
mapping, fused steps, stores, pass loop) over one input.  Inputs are resident
in HBM before the timed region starts.

Prints ONE JSON line: throughput in Gcell-updates/s (Eq. 5 of the paper:
cells x steps / time), the dominant kernel's HBM roofline figures measured
with HIP events on the run stream, and the CPU oracle timed on a bounded
sample of the same workload.  Secondary figures (FP32 on the same workload,
the batched ensemble) are reported under "secondary".
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def time_runs(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = _events(torch)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3  # seconds


def heat3d_workload(torch, st, synth, dtype, n=512, steps=100, alpha=0.15, select=None):
    shape = (n, n, n)
    offs = synth.star_offsets(3, 1)
    wdt = "f64" if dtype == "f64" else "f32"
    w = list(synth.heat_weights(3, alpha, wdt))
    tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[dtype]
    # U[0,1) from seed 0 plus the closed-form mode, built on the device in
    # slices so the host never holds more than one plane set at a time
    u = torch.empty(shape, dtype=tdt, device="cuda")
    mode_axis = [np.sin(np.pi * (np.arange(n) + 1.0) / (n + 1.0))] * 3
    noise = synth.uniform_field(shape, seed=0)
    mode = np.einsum("i,j,k->ijk", *mode_axis)
    u.copy_(torch.from_numpy(noise + mode))
    del noise, mode
    work = torch.empty_like(u)
    plan = st.Plan(offs, shape, dtype, "zero")
    if select:
        plan.select(**select)
    return plan, u, work, w, steps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32", "bf16"])
    ap.add_argument("--tb", type=int, default=0, help="force the fused depth (0 = plan default)")
    ap.add_argument("--variant", type=int, default=-1, help="force a tiling candidate")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=2, help="oracle steps in the CPU sample")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the sweep runs on a single MI355X here; "
              "multi-GPU sharding is a design note, not a measured path.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2303_08365_amd as st
    import synth

    torch.cuda.init()
    dev = torch.cuda.get_device_properties(0)
    log(f"device: {dev.name} ({getattr(dev, 'gcnArchName', '?')}), CUs {dev.multi_processor_count}")

    n, T = 512, 100
    select = {}
    if args.variant >= 0:
        select["variant"] = args.variant
    elif args.tb > 0:
        select["tb"] = args.tb
    plan, u, work, w, T = heat3d_workload(torch, st, synth, args.dtype, n, T, select=select or None)
    info = plan.info()
    log(f"plan: {info}")
    cells = n ** 3

    def one():
        plan.run(u, w, T, work=work)

    secs = time_runs(torch, one, args.steps, args.warmup)
    ms_per_step = secs / args.steps * 1e3
    value = cells * T * args.steps / secs / 1e9
    # passes per run (launches of the dominant kernel): depth tb, count even
    tb = info["tb"]
    passes = -(-T // tb)
    if passes % 2 == 1 and tb > 1:
        passes += 1
    s_bytes = {"f64": 8, "f32": 4, "bf16": 2}[args.dtype]
    alg_bytes = 2.0 * s_bytes * cells  # one read + one write of the grid per pass
    launch_s = secs / (args.steps * passes)
    achieved = alg_bytes / launch_s / 1e9
    log(f"{value:.1f} Gcell/s, {ms_per_step:.3f} ms/run, {passes} passes of {launch_s*1e6:.1f} us, "
        f"{achieved:.0f} GB/s algorithmic per pass")

    kname = {0: "naive_kernel", 1: "stream2d_kernel", 2: "stream3d_kernel", 3: "varcoef"}[info["kernel"]]
    out = {
        "metric": "Gcell-updates/s (3D 7-point heat, 512^3, 100 steps, FP64)",
        "value": round(value, 3),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic: U[0,1) seed 0 plus one sin mode",
        "config": {"workload": f"3D 7-point heat stencil, {n}^3, {T} steps, alpha 0.15, zero boundary",
                   "grid": [n, n, n], "time_steps": T, "fused_depth": tb,
                   "tile": [info["tile_x"], info["tile_y"], info["tile_z"]],
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 1),
                     "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": None, "launches_per_step": passes,
                     "avg_launch_us": round(launch_s * 1e6, 2),
                     "alg_bytes_per_launch": alg_bytes},
    }
    single_pass_roofline = PEAK_HBM_GBS * 1e9 / (2 * s_bytes) / 1e9
    out["single_pass_roofline_frac"] = round(value / single_pass_roofline, 4)

    if not args.no_secondary:
        sec = {}
        try:
            if args.dtype == "f64":
                del u, work
                torch.cuda.empty_cache()
                p32, u32, w32b, wt32, _ = heat3d_workload(torch, st, synth, "f32", n, T)
                s32 = time_runs(torch, lambda: p32.run(u32, wt32, T, work=w32b), max(3, args.steps // 2), 1)
                sec["f32_same_workload_gcells"] = round(cells * T * max(3, args.steps // 2) / s32 / 1e9, 3)
                sec["f32_tb"] = p32.info()["tb"]
                del u32, w32b
                torch.cuda.empty_cache()
        except Exception as e:  # secondary figures never hide the headline
            sec["error"] = repr(e)
        out["secondary"] = sec

    if not args.no_cpu_baseline:
        import oracle
        sample_steps = args.cpu_steps
        u0 = synth.uniform_field((n, n, n), seed=0)
        threads = oracle.max_threads()
        t0 = time.perf_counter()
        oracle.heat(u0, 0.15, sample_steps, bc="zero", threads=threads)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(cells * sample_steps / dt / 1e9, 4), "unit": "Gcell-updates/s",
                               "cores": threads, "kind": "oracle",
                               "sample": f"oracle heat form, {n}^3 FP64, {sample_steps} of the {T} steps "
                                         f"({dt:.1f} s)"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
