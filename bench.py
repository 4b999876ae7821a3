#!/usr/bin/env python3
"""Benchmark of the stencil sweep on one MI355X.

Default workload (the headline): 100 time steps of the 3D 7-point heat
stencil on a 512^3 FP64 grid (zero-Dirichlet ghost layer, alpha = 0.15,
U[0,1) initial field from seed 0 plus one sin mode).  A bench "step" is one
whole run of that workload -- every stage of the hot path (plan choice,
halo-tile loads, register/DPP pattern mapping, fused time steps, stores,
pass loop) over one input that is resident in HBM before timing starts.

Prints ONE JSON line: throughput in Gcell-updates/s (Eq. 5 of the paper:
cells x time steps / time), the dominant kernel's HBM roofline figures
measured with HIP events on the run stream, and the CPU oracle timed on a
bounded sample of the same workload.  Secondary figures (FP32 on the same
workload, the batched FP32 ensemble) are reported under "secondary".

Other workloads (--workload): heat2d (2D 5-point FP64 512^2, 100 steps),
box2d (2D 9-point box FP32 8192^2, 1000 steps, periodic), box2d25 (2D
25-point box FP64 8192^2, 100 steps, zero rule), star25 (3D order-4 25-point
star FP32 512^3, 50 steps, periodic), batch (64 2D 5-point grids, sides
log-uniform in [256, 4096], 500 steps).  --tiling overlapped|tessellated
times one 2D tiling of Sec. 4.1's two kinds at a depth (A/B).
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
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "traffic.json")


# Device sources of the kernels whose counters profiles/traffic.json holds:
# the 3D streaming families (the headline) and the copy kernel that scales the
# counters; of internal.h only the 3D family's argument block.  Host planning
# code is left out: the launch configuration is part of the lookup key.
TRAFFIC_SOURCES = ("dev_common.h", "registry.h", "stream3d_impl.h", "s3d_r1_f64.hip", "s3d_r1_f32.hip",
                   "s3d_r1_bf16.hip", "pipe3d_impl.h", "p3d_r1.hip", "copy.hip")


def source_hash() -> str:
    """SHA-256 over TRAFFIC_SOURCES (names and bytes) and the Stream3DArgs /
    Stream3DKey definitions of internal.h."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2303_08365_amd", "csrc")
    for name in TRAFFIC_SOURCES:
        h.update(name.encode())
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(csrc, "internal.h"), "rb") as fh:
        text = fh.read()
    a = text.index(b"struct Stream3DArgs {")
    b = text.index(b"};", text.index(b"struct Stream3DKey {")) + 2
    h.update(b"internal.h:3d")
    h.update(text[a:b])
    return h.hexdigest()


def traffic_lookup(key):
    """Counter-measured HBM bytes per launch for this plan, or None when none
    were taken or the kernel sources changed since."""
    try:
        with open(TRAFFIC_JSON) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("sources_sha256") != source_hash():
        return None
    for e in t.get("entries", []):
        if e.get("key") == key:
            return e
    return None


def _counter_means(directory, counter):
    """Mean of `counter` per dispatch, per kernel name, from the rocprofv3
    counter CSV(s) found under `directory`."""
    import csv
    import glob
    out = {}
    paths = sorted(glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True))
    for path in paths:
        with open(path) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] != counter:
                    continue
                out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in out.items()}


def ingest_counters(directory, key, out_path):
    """Turn two rocprofv3 --pmc passes per kernel (FETCH_SIZE, WRITE_SIZE, in
    KiB per dispatch) into bytes per launch, scaled by what the same counters
    read for the streaming copy of a known size (one 512^3 FP64 grid)."""
    copy_bytes = 512 ** 3 * 8
    res = {}
    for counter in ("FETCH_SIZE", "WRITE_SIZE"):
        st_m = _counter_means(os.path.join(directory, f"stencil_{counter}"), counter)
        cp_m = _counter_means(os.path.join(directory, f"copy_{counter}"), counter)
        cp = [v for k, v in cp_m.items() if "copy_kernel" in k]
        sk = [(k, v) for k, v in st_m.items() if "st::" in k]
        if not cp or not sk:
            raise SystemExit(f"no counter rows for {counter} in {directory}")
        sk.sort(key=lambda kv: -kv[1])
        res[counter] = {"kernel": sk[0][0], "kib_per_dispatch": sk[0][1], "copy_kib_per_dispatch": cp[0],
                        "scale": copy_bytes / 1024.0 / cp[0]}
    fetch = res["FETCH_SIZE"]["kib_per_dispatch"] * res["FETCH_SIZE"]["scale"] * 1024.0
    write = res["WRITE_SIZE"]["kib_per_dispatch"] * res["WRITE_SIZE"]["scale"] * 1024.0
    entry = {"key": key, "kernel": res["FETCH_SIZE"]["kernel"], "fetch_bytes": fetch, "write_bytes": write,
             "traffic_bytes": fetch + write, "counters": res}
    doc = {"sources_sha256": source_hash(), "entries": [entry]}
    with open(out_path, "w") as f:
        json.dump(doc, f, indent=1)
    print(json.dumps(entry), flush=True)
BYTES = {"f64": 8, "f32": 4, "bf16": 2}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_runs(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3  # seconds


def passes_of(steps, tb):
    """Launches of the fused kernel per run (the pass list is made even)."""
    n = -(-steps // tb)
    if n % 2 == 1 and tb > 1:
        n += 1
    return n


def _tdt(torch, dtype):
    return {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[dtype]


def _select(args):
    if args.variant >= 0:
        return {"variant": args.variant}
    if args.tiling != "auto":
        return {"tiling": args.tiling, "tb": args.tb}
    if args.tb > 0:
        return {"tb": args.tb}
    return None


def select_tiling(plan, select):
    """Apply a selection: a candidate index, a fused depth, or the overlapped
    or tessellated 2D tiling at a depth (0: the plan's default depth) with
    the model's chunk."""
    sel = dict(select)
    tiling = sel.pop("tiling", None)
    if tiling is None:
        plan.select(**sel)
        return
    tb = sel.pop("tb", 0) or plan.info()["tb"]
    want = 1 if tiling == "tessellated" else 0
    ks = [k for k, c in enumerate(plan.candidates())
          if c["kernel"] == 1 and c["tessellated"] == want and c["tb"] == tb]
    if not ks:
        sys.exit(f"no {tiling} 2D tiling of depth {tb} for this workload")
    plan.select(variant=ks[0])


class Workload:
    """A plan, its device buffers and the figures needed for the report."""


def heat3d_input(synth, n=512):
    """The headline's initial field in FP64: U[0,1) from seed 0 plus the
    sin(pi x) sin(pi y) sin(pi z) mode."""
    mode = np.einsum("i,j,k->ijk", *([np.sin(np.pi * (np.arange(n) + 1.0) / (n + 1.0))] * 3))
    return synth.uniform_field((n, n, n), seed=0) + mode


def heat3d(torch, st, synth, dtype, select=None, n=512, steps=100, alpha=0.15, flux=False):
    w = Workload()
    shape = (n, n, n)
    wdt = "f64" if dtype == "f64" else "f32"
    w.coeffs = list(synth.heat_weights(3, alpha, wdt))
    w.u = torch.from_numpy(heat3d_input(synth, n)).to("cuda", _tdt(torch, dtype))
    w.work = torch.empty_like(w.u)
    # the library's default candidate (deterministic, so the counter-measured
    # traffic of profiles/ stays matched to the timed kernel)
    w.plan = st.Plan(synth.star_offsets(3, 1), shape, dtype, "zero")
    if select:
        select_tiling(w.plan, select)
    w.steps, w.cells, w.dtype = steps, n ** 3, dtype
    w.name = f"3D 7-point heat stencil, {n}^3, {steps} steps, alpha {alpha}, zero boundary"
    w.run = lambda: w.plan.run(w.u, w.coeffs, w.steps, work=w.work)
    if flux:
        # the same sweep through stencil_run_flux: FP64 outflow of every step
        w.flux = torch.zeros(1, dtype=torch.float64, device="cuda")
        w.run = lambda: w.plan.run_flux(w.u, w.coeffs, w.steps, w.flux, work=w.work)
    w.kernel_tb = w.plan.info()["tb"]
    return w


def flux_drift(torch, w):
    """One run of an outflow workload from its initial field: relative gap
    between the initial total and final total + outflow."""
    s0 = float(w.u.double().sum())
    w.flux.zero_()
    w.run()
    torch.cuda.synchronize()
    sT = float(w.u.double().sum())
    out = float(w.flux.cpu()[0])
    return (s0 - sT - out) / s0, out / s0


def heat2d(torch, st, synth, dtype, select=None, n=512, steps=100, alpha=0.2):
    w = Workload()
    shape = (n, n)
    w.coeffs = list(synth.heat_weights(2, alpha, "f64" if dtype == "f64" else "f32"))
    w.u = torch.from_numpy(synth.uniform_field(shape, seed=0)).to("cuda", _tdt(torch, dtype))
    w.work = torch.empty_like(w.u)
    # a 2 MiB grid: the run is launch-bound, so its passes replay from a graph;
    # fused depth and chunk length come from the library's autotuner
    w.plan = st.Plan(synth.star_offsets(2, 1), shape, dtype, "zero", graph=True, autotune=select is None)
    if select:
        select_tiling(w.plan, select)
    w.steps, w.cells, w.dtype = steps, n * n, dtype
    w.name = f"2D 5-point heat stencil, {n}^2, {steps} steps, alpha {alpha}, zero boundary"
    w.run = lambda: w.plan.run(w.u, w.coeffs, w.steps, work=w.work)
    w.kernel_tb = w.plan.info()["tb"]
    return w


def heat1d(torch, st, synth, dtype, select=None, n=10_000_000, steps=1000, alpha=0.25, radius=1):
    """Tab. 1's Heat-1D (radius 1) / Star-1D5P (radius 2) shape: 10^7 cells;
    1000 of its 10^5 steps; zero rule; U[0,1) seed 0."""
    w = Workload()
    shape = (n,)
    wdt = "f64" if dtype == "f64" else "f32"
    offs = synth.star_offsets(1, radius)
    if radius == 1:
        w.coeffs = list(synth.heat_weights(1, alpha, wdt))
    else:
        w.coeffs = list(synth.adjust_centre([0.0] + [alpha / (2 * radius)] * (2 * radius), wdt))
    w.u = torch.from_numpy(synth.uniform_field(shape, seed=0)).to("cuda", _tdt(torch, dtype))
    w.work = torch.empty_like(w.u)
    w.plan = st.Plan(offs, shape, dtype, "zero", autotune=select is None)
    if select:
        select_tiling(w.plan, select)
    w.steps, w.cells, w.dtype = steps, n, dtype
    w.name = f"1D {2 * radius + 1}-point star, {n} cells, {steps} steps, zero boundary"
    w.run = lambda: w.plan.run(w.u, w.coeffs, w.steps, work=w.work)
    w.kernel_tb = w.plan.info()["tb"]
    return w


def box27(torch, st, synth, dtype, select=None, n=512, steps=20):
    """Tab. 1's Box-3D27P shape class on the 512^3 grid: 27 weights of 1/27
    (centre-adjusted), zero rule, U[0,1) seed 0."""
    w = Workload()
    shape = (n, n, n)
    w.coeffs = list(synth.box_mean_weights(3, 1, "f64" if dtype == "f64" else "f32"))
    w.u = torch.from_numpy(synth.uniform_field(shape, seed=0)).to("cuda", _tdt(torch, dtype))
    w.work = torch.empty_like(w.u)
    w.plan = st.Plan(synth.box_offsets(3, 1), shape, dtype, "zero", autotune=select is None)
    if select:
        select_tiling(w.plan, select)
    w.steps, w.cells, w.dtype = steps, n ** 3, dtype
    w.name = f"3D 27-point box stencil, {n}^3, {steps} steps, zero boundary"
    w.run = lambda: w.plan.run(w.u, w.coeffs, w.steps, work=w.work)
    w.kernel_tb = w.plan.info()["tb"]
    return w


def box2d(torch, st, synth, dtype, select=None, n=8192, steps=1000):
    w = Workload()
    shape = (n, n)
    w.coeffs = list(synth.box_mean_weights(2, 1, "f64" if dtype == "f64" else "f32"))
    w.u = torch.from_numpy(synth.uniform_field(shape, seed=0)).to("cuda", _tdt(torch, dtype))
    w.work = torch.empty_like(w.u)
    w.plan = st.Plan(synth.box_offsets(2, 1), shape, dtype, "periodic", autotune=select is None)
    if select:
        select_tiling(w.plan, select)
    w.steps, w.cells, w.dtype = steps, n * n, dtype
    w.name = f"2D 9-point box stencil (weights 1/9), {n}^2, {steps} steps, periodic"
    w.run = lambda: w.plan.run(w.u, w.coeffs, w.steps, work=w.work)
    w.kernel_tb = w.plan.info()["tb"]
    return w


def box2d25(torch, st, synth, dtype, select=None, n=8192, steps=100):
    """Tab. 1's Box-2D25P shape class: the 5x5 box, weights 1/25
    (centre-adjusted), zero rule, U[0,1) seed 0."""
    w = Workload()
    shape = (n, n)
    w.coeffs = list(synth.box_mean_weights(2, 2, "f64" if dtype == "f64" else "f32"))
    w.u = torch.from_numpy(synth.uniform_field(shape, seed=0)).to("cuda", _tdt(torch, dtype))
    w.work = torch.empty_like(w.u)
    w.plan = st.Plan(synth.box_offsets(2, 2), shape, dtype, "zero", autotune=select is None)
    if select:
        select_tiling(w.plan, select)
    w.steps, w.cells, w.dtype = steps, n * n, dtype
    w.name = f"2D 25-point box stencil (weights 1/25), {n}^2, {steps} steps, zero boundary"
    w.run = lambda: w.plan.run(w.u, w.coeffs, w.steps, work=w.work)
    w.kernel_tb = w.plan.info()["tb"]
    return w


def star25(torch, st, synth, dtype, select=None, n=512, steps=50):
    w = Workload()
    shape = (n, n, n)
    w.coeffs = list(synth.star25_weights(0, "f64" if dtype == "f64" else "f32"))
    w.u = torch.from_numpy(synth.uniform_field(shape, seed=0)).to("cuda", _tdt(torch, dtype))
    w.work = torch.empty_like(w.u)
    w.plan = st.Plan(synth.star_offsets(3, 4), shape, dtype, "periodic", autotune=select is None)
    if select:
        select_tiling(w.plan, select)
    w.steps, w.cells, w.dtype = steps, n ** 3, dtype
    w.name = f"3D order-4 25-point star stencil, {n}^3, {steps} steps, periodic"
    w.run = lambda: w.plan.run(w.u, w.coeffs, w.steps, work=w.work)
    w.kernel_tb = w.plan.info()["tb"]
    return w


def batch(torch, st, synth, dtype, select=None, ngrids=64, steps=500):
    w = Workload()
    shapes = synth.batch_shapes(ngrids, seed=0)
    alphas = synth.batch_alphas(ngrids, seed=0)
    wdt = "f64" if dtype == "f64" else "f32"
    w.coeffs = [list(synth.heat_weights(2, a, wdt)) for a in alphas]
    w.grids = [torch.from_numpy(synth.uniform_field(s, seed=g)).to("cuda", _tdt(torch, dtype))
               for g, s in enumerate(shapes)]
    w.works = [torch.empty_like(g) for g in w.grids]
    # tile and fused depth chosen by the library's autotuner on these shapes;
    # the passes of a run replay from one captured HIP graph
    w.plan = st.BatchPlan(synth.star_offsets(2, 1), shapes, dtype, "zero", autotune=select is None,
                          graph=True)
    if select:
        select_tiling(w.plan, select)
    w.steps = steps
    w.cells = int(sum(a * b for a, b in shapes))
    w.dtype = dtype
    w.name = (f"{ngrids} 2D 5-point heat grids, sides log-uniform [256, 4096] (seed 0), "
              f"alpha U[0.05, 0.24], {steps} steps, zero boundary")
    w.run = lambda: w.plan.run(w.grids, w.works, w.coeffs, [steps] * ngrids)
    w.kernel_tb = w.plan.info()["tb"]
    return w


def varcoef(torch, st, synth, dtype, select=None, n=256, steps=200, every=20, alpha=0.1):
    """Forward with checkpoints plus the full adjoint (dL/du0, dL/dk) of an MSE loss."""
    w = Workload()
    shape = (n, n, n)
    u0, k, y = synth.varcoef_inputs(shape, seed=0)
    tdt = _tdt(torch, dtype)
    w.u0 = torch.from_numpy(u0).to("cuda", tdt)
    w.k = torch.from_numpy(k).to("cuda", tdt)
    w.y = torch.from_numpy(y).to("cuda", tdt)
    del u0, k, y
    w.u = torch.empty_like(w.u0)
    w.work = torch.empty_like(w.u0)
    w.lam = torch.empty_like(w.u0)
    w.gk = torch.empty_like(w.u0)
    w.ckpts = [torch.empty_like(w.u0) for _ in range(-(-steps // every))]
    w.seg = torch.empty((every - 1,) + shape, dtype=tdt, device="cuda")
    w.plan = st.varcoef_plan(shape, dtype)
    w.steps, w.cells, w.dtype = steps, n ** 3, dtype
    w.name = (f"3D variable-coefficient heat, {n}^3, {steps} steps, checkpoints every {every}, "
              f"forward + adjoint of an MSE loss")

    def run():
        w.u.copy_(w.u0)
        w.plan.run_ckpt(w.u, w.k, alpha, steps, w.work, every=every, ckpts=w.ckpts)
        torch.sub(w.u, w.y, out=w.lam)
        w.lam.mul_(2.0 / w.cells)
        w.gk.zero_()
        w.plan.adjoint(w.lam, steps, w.work, k=w.k, alpha=alpha, ckpts=w.ckpts, every=every,
                       grad_k=w.gk, seg=w.seg)

    w.run = run
    w.kernel_tb = 1
    return w


# Case study (paper Sec. 6.5): width of the initial Gaussian, in cells, chosen
# so that the closed-form zero-rule solution has 52.0 at the centre after
# 3.8e6 steps (derived from the oracle's spectral solution by
# tests/golden/case_study_sigma.py, stored in tests/golden/case_study_gaussian.txt).
CASE_SIGMA = 1376.2


def case_study(torch, st, synth, steps, n=9600, mu=0.23, amplitude=100.0, sigma=None, chunk=50_000):
    sigma = sigma or CASE_SIGMA
    u0 = synth.gaussian_plate(n, sigma, amplitude)
    c = n // 2 - 1
    out = {"metric": "case study: Heat-2D 5-point, zero rule", "n": n, "mu": mu, "steps": steps,
           "amplitude": amplitude, "sigma_cells": sigma, "initial_centre": float(u0[c, c])}
    finals = {}
    for dtype in ("f64", "f32"):
        wdt = "f64" if dtype == "f64" else "f32"
        coeffs = list(synth.heat_weights(2, mu, wdt))
        plan = st.Plan(synth.star_offsets(2, 1), (n, n), dtype, "zero", autotune=True)
        u = torch.from_numpy(u0).to("cuda", _tdt(torch, dtype))
        work = torch.empty_like(u)
        flux = torch.zeros(1, dtype=torch.float64, device="cuda")
        total0 = float(u.double().sum())
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        gpu_s, done = 0.0, 0
        while done < steps:
            k = min(chunk, steps - done)
            e0.record()
            plan.run_flux(u, coeffs, k, flux, work=work)
            e1.record()
            torch.cuda.synchronize()
            gpu_s += e0.elapsed_time(e1) / 1e3
            done += k
            log(f"case study {dtype}: {done} / {steps} steps, {n * n * done / gpu_s / 1e9:.1f} Gcell/s, "
                f"centre {float(u[c, c]):.6f}")
        finals[dtype] = u.double().cpu().numpy()
        totalT, outflow = float(finals[dtype].sum()), float(flux.cpu()[0])
        out[dtype] = {"gcells": round(n * n * steps / gpu_s / 1e9, 2), "gpu_seconds": round(gpu_s, 2),
                      "centre": float(finals[dtype][c, c]), "plan": plan.info(),
                      "outflow_fraction": round(outflow / total0, 6),
                      "total_plus_outflow_drift": float(f"{(totalT + outflow - total0) / total0:.3e}")}
        del u, work
        torch.cuda.empty_cache()
    # deviation of FP32 from FP64, in the form of the paper's Tab. 4
    ref, d = finals["f64"], np.abs(finals["f32"] - finals["f64"])
    rel = d / np.maximum(np.abs(ref), np.finfo(np.float64).tiny)
    out["f32_vs_f64_percent_of_cells"] = {
        "abs_gt_0.1": round(100.0 * float(np.mean(d > 0.1)), 2),
        "abs_gt_0.5": round(100.0 * float(np.mean(d > 0.5)), 2),
        "abs_gt_1.0": round(100.0 * float(np.mean(d > 1.0)), 2),
        "rel_gt_1pct": round(100.0 * float(np.mean(rel > 0.01)), 2),
        "rel_gt_3pct": round(100.0 * float(np.mean(rel > 0.03)), 2),
        "rel_gt_5pct": round(100.0 * float(np.mean(rel > 0.05)), 2),
        "max_abs": float(d.max()),
    }
    return out


WORKLOADS = {"varcoef": varcoef, "heat3d": heat3d, "heat2d": heat2d, "box2d": box2d, "box2d25": box2d25,
             "star25": star25, "batch": batch,
             "heat1d": heat1d, "star1d5": lambda *a, **k: heat1d(*a, radius=2, **k), "box27": box27}
DEFAULT_DTYPE = {"varcoef": "f32", "heat3d": "f64", "heat2d": "f64", "box2d": "f32", "box2d25": "f64",
                 "star25": "f32", "batch": "f32",
                 "heat1d": "f64", "star1d5": "f64", "box27": "f64"}
KERNEL_NAMES = {0: "naive_kernel", 1: "stream2d_kernel", 2: "stream3d_kernel", 3: "varcoef3d_kernel",
                4: "stream1d_kernel", 5: "box3d_kernel"}


def measure(torch, w, steps, warmup):
    secs = time_runs(torch, w.run, steps, warmup)
    value = w.cells * w.steps * steps / secs / 1e9
    passes = passes_of(w.steps, w.kernel_tb)
    launch_s = secs / (steps * passes)
    alg = 2.0 * BYTES[w.dtype] * w.cells
    return secs, value, passes, launch_s, alg


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="heat3d", choices=sorted(WORKLOADS))
    ap.add_argument("--dtype", default=None, choices=["f64", "f32", "bf16"])
    ap.add_argument("--tb", type=int, default=0, help="force the fused depth (0 = plan default)")
    ap.add_argument("--variant", type=int, default=-1, help="force a tiling candidate")
    ap.add_argument("--tiling", default="auto", choices=["auto", "overlapped", "tessellated"],
                    help="2D workloads: time the overlapped or the tessellated tiling (at --tb, else the "
                         "default depth)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--flux", action="store_true",
                    help="heat3d through stencil_run_flux (FP64 outflow of every step)")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the per-dtype error report against the oracle")
    ap.add_argument("--case-study", action="store_true",
                    help="the paper's thermal-diffusion case study (Heat-2D 9600^2, CFL 0.23, 3.8e6 steps, "
                         "Gaussian plate) in FP64 and FP32, with the FP32-vs-FP64 deviation table")
    ap.add_argument("--case-steps", type=int, default=3_800_000)
    ap.add_argument("--copy-probe", action="store_true",
                    help="time a plain 512^3 FP64 device copy instead (bandwidth reference)")
    ap.add_argument("--ingest-counters", default=None, metavar="DIR",
                    help="read rocprofv3 FETCH_SIZE/WRITE_SIZE passes from DIR for this workload's "
                         "plan and write DIR/traffic.json")
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

    if args.case_study:
        print(json.dumps(case_study(torch, st, synth, args.case_steps)), flush=True)
        return

    if args.copy_probe:
        # plain device copy of one 512^3 FP64 grid: the achievable-bandwidth
        # reference and the scale for the FETCH_SIZE / WRITE_SIZE counters
        src = torch.ones((512, 512, 512), dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        secs = time_runs(torch, lambda: st.copy(dst, src), args.steps, args.warmup)
        nbytes = 2.0 * src.numel() * 8
        print(json.dumps({"metric": "device copy GB/s", "value": round(nbytes * args.steps / secs / 1e9, 1),
                          "unit": "GB/s", "bytes_per_launch": nbytes,
                          "avg_launch_us": round(secs / args.steps * 1e6, 2)}), flush=True)
        return

    dtype = args.dtype or DEFAULT_DTYPE[args.workload]
    if args.flux:
        if args.workload != "heat3d":
            sys.exit("--flux applies to the heat3d workload")
        w = heat3d(torch, st, synth, dtype, _select(args), flux=True)
    else:
        w = WORKLOADS[args.workload](torch, st, synth, dtype, _select(args))
    info = w.plan.info()
    log(f"plan: {info}")
    tkey = [args.workload, dtype, info["kernel"], info["tb"], info["tile_x"], info["tile_y"], info["tile_z"],
            info["block"], info["workgroups"], info.get("pipeline", 0)] + \
        ([1] if info.get("tessellated") else [])
    if args.ingest_counters:
        ingest_counters(args.ingest_counters, tkey, os.path.join(args.ingest_counters, "traffic.json"))
        return
    secs, value, passes, launch_s, alg = measure(torch, w, args.steps, args.warmup)
    achieved = alg / launch_s / 1e9
    log(f"{value:.1f} Gcell/s, {secs / args.steps * 1e3:.3f} ms/run, {passes} passes of "
        f"{launch_s * 1e6:.1f} us, {achieved:.0f} GB/s algorithmic per pass")

    out = {
        "metric": "Gcell-updates/s & % HBM roofline",
        "value": round(value, 3),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(secs / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic (seeded U[0,1) fields; see DESIGN.md input recipe)",
        "config": {"workload": w.name, "cells": w.cells, "time_steps": w.steps,
                   "fused_depth": w.kernel_tb,
                   "tile": [info["tile_x"], info["tile_y"], info["tile_z"]],
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm",
                     "kernel": ("boxpipe3d_kernel" if info.get("pipeline") and info["kernel"] == 5 else
                                "pipe3d_kernel" if info.get("pipeline") else
                                "stream2d_kernel + tess2d_band_kernel" if info.get("tessellated") else
                                KERNEL_NAMES[info["kernel"]]),
                     "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None,
                     "launches_per_step": passes, "avg_launch_us": round(launch_s * 1e6, 2),
                     "alg_bytes_per_launch": alg},
        "single_pass_roofline_frac": round(value / (PEAK_HBM_GBS / (2 * BYTES[dtype])), 4),
    }
    tr = traffic_lookup(tkey)
    if tr is not None:
        out["roofline"]["traffic"] = round(tr["traffic_bytes"], 0)
        out["roofline"]["traffic_GBps"] = round(tr["traffic_bytes"] / launch_s / 1e9, 1)

    if not args.no_secondary and args.workload == "heat3d":
        sec = {}
        try:
            del w.u, w.work
            torch.cuda.empty_cache()
            w32 = heat3d(torch, st, synth, "f32")
            _, v32, _, _, _ = measure(torch, w32, max(3, args.steps // 2), 1)
            sec["f32_same_workload_gcells"] = round(v32, 3)
            sec["f32_fused_depth"] = w32.kernel_tb
            del w32
            torch.cuda.empty_cache()
            w16 = heat3d(torch, st, synth, "bf16")
            _, v16, _, _, _ = measure(torch, w16, max(3, args.steps // 2), 1)
            sec["bf16_same_workload_gcells"] = round(v16, 3)
            sec["bf16_fused_depth"] = w16.kernel_tb
            del w16
            torch.cuda.empty_cache()
            for fdt in ("f64", "f32"):
                wf = heat3d(torch, st, synth, fdt, flux=True)
                drift, frac = flux_drift(torch, wf)
                _, vf, _, _, _ = measure(torch, wf, max(3, args.steps // 2), 1)
                sec[f"{fdt}_with_outflow_gcells"] = round(vf, 3)
                sec[f"{fdt}_outflow_total_drift"] = float(f"{drift:.3e}")
                sec[f"{fdt}_outflow_fraction_of_total"] = round(frac, 6)
                del wf
                torch.cuda.empty_cache()
            wb = batch(torch, st, synth, "f32")
            _, vb, _, _, _ = measure(torch, wb, 2, 1)
            sec["batch64_f32_gcells"] = round(vb, 3)
            del wb
            torch.cuda.empty_cache()
        except Exception as e:  # secondary figures never hide the headline
            sec["error"] = repr(e)
        out["secondary"] = sec

    if not args.no_cpu_baseline and args.workload == "heat3d":
        cpu, acc = oracle_leg(torch, st, synth, args)
        out["cpu_baseline"] = cpu
        if acc:
            out["accuracy"] = acc
    print(json.dumps(out), flush=True)


def cpu_model() -> str:
    """The host CPU as /proc/cpuinfo names it, with its family / model /
    stepping numbers (a virtualised host may report a generic name)."""
    fields = {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if ":" not in line:
                    if fields:
                        break  # first processor only
                    continue
                k, v = (x.strip() for x in line.split(":", 1))
                fields.setdefault(k, v)
    except OSError:
        return "unknown"
    name = fields.get("model name", "unknown")
    ids = [f"{k} {fields[k]}" for k in ("cpu family", "model", "stepping") if k in fields]
    return f"{name} ({', '.join(ids)})" if ids else name


# Relative-deviation thresholds of the accuracy report: the paper's Tab. 4
# uses 1 %, 3 % and 5 %; the finer ones resolve FP32.
REL_THRESHOLDS = (1e-6, 1e-5, 1e-4, 1e-3, 1e-2, 3e-2, 5e-2)


def deviation(got, ref):
    """rel-L2, max |delta| and the percentage of cells whose |delta| / |ref|
    exceeds each threshold."""
    d = np.abs(got - ref)
    rel = d / np.maximum(np.abs(ref), 1e-300)
    out = {"rel_l2": float(np.sqrt(np.sum(d * d) / np.sum(ref * ref))), "max_abs": float(d.max()),
           "pct_rel_above": {f"{t:g}": round(100.0 * float(np.count_nonzero(rel > t)) / rel.size, 6)
                             for t in REL_THRESHOLDS}}
    return out


def oracle_leg(torch, st, synth, args):
    """The CPU oracle on the headline workload: the whole 100-step run on all
    host threads (timed: the all-core baseline; its result is the reference
    of the accuracy report), and two steps on one thread (timed).  Then one
    100-step GPU run per storage type from the same initial field (FP32 and
    bfloat16 start from the rounded field: their error includes that
    rounding), compared cell by cell with the oracle."""
    import oracle
    n, steps, alpha = 512, 100, 0.15
    u0 = heat3d_input(synth, n)
    threads = oracle.max_threads()
    t0 = time.perf_counter()
    ref = oracle.heat(u0, alpha, steps, bc="zero", threads=threads)
    dt_all = time.perf_counter() - t0
    one_steps = 2
    t0 = time.perf_counter()
    oracle.heat(u0, alpha, one_steps, bc="zero", threads=1)
    dt_one = time.perf_counter() - t0
    cpu = {"value": round(n ** 3 * steps / dt_all / 1e9, 4), "unit": "Gcell-updates/s", "cores": threads,
           "kind": "oracle",
           "sample": f"oracle heat form, the whole {n}^3 FP64 100-step run, {dt_all:.1f} s on {threads} "
                     f"threads; single thread: {one_steps} steps in {dt_one:.1f} s",
           "single_thread_value": round(n ** 3 * one_steps / dt_one / 1e9, 4),
           "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}
    acc = {}
    if args.no_accuracy:
        return cpu, acc
    for dtype in ("f64", "f32", "bf16"):
        try:
            w = heat3d(torch, st, synth, dtype)
            w.run()
            torch.cuda.synchronize()
            got = w.u.to(torch.float64).cpu().numpy()
            del w
            torch.cuda.empty_cache()
            acc[dtype] = deviation(got, ref)
            del got
        except Exception as e:  # the report never hides the headline
            acc[dtype] = {"error": repr(e)}
    acc["reference"] = "FP64 oracle, same initial field (unrounded), 100 steps"
    return cpu, acc


if __name__ == "__main__":
    main()
