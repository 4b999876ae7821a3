"""GPU: the thermal-diffusion case study (paper Sec. 6.5) scaled down for a
test.  The Gaussian plate of the full study (9600^2, width sigma, 3.8e6 steps
at CFL number 0.23) is shrunk 8x in space, so 64x fewer steps cover the same
diffusion: 1200^2, sigma/8, 59375 steps.  FP64 must match the closed-form
(DST-I) solution; FP32 is compared with FP64 in the form of Tab. 4, and its
total + FP64 outflow must track the initial total."""
import os

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import to_device, to_host

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _study():
    with open(os.path.join(HERE, "golden", "case_study_gaussian.txt")) as fh:
        row = [ln for ln in fh if ln.strip() and not ln.startswith("#")][0].split()
    n, mu, steps, amp, sigma, centre = int(row[0]), float(row[1]), int(row[2]), float(row[3]), float(row[4]), \
        float(row[5])
    return n, mu, steps, amp, sigma, centre


def test_case_study_scaled_fp64_matches_closed_form_and_fp32_tracks_it():
    import torch
    import paper_2303_08365_amd as st
    n_full, mu, steps_full, amp, sigma, _ = _study()
    n, sig, steps = n_full // 8, sigma / 8.0, steps_full // 64
    u0 = synth.gaussian_plate(n, sig, amp)
    offs = synth.star_offsets(2, 1)
    print(f"case study scaled: {n}^2 sigma {sig} steps {steps}", flush=True)
    res = {}
    for dtype in ("f64", "f32"):
        plan = st.Plan(offs, (n, n), dtype, "zero")
        g = to_device(u0, dtype)
        f = torch.zeros(1, dtype=torch.float64, device="cuda")
        plan.run_flux(g, list(synth.heat_weights(2, mu, dtype)), steps, f)
        res[dtype] = (to_host(g), float(f.cpu()[0]))
    ref = oracle.heat_spectral(u0, mu, steps)
    u64, out64 = res["f64"]
    u32, out32 = res["f32"]
    c = n // 2 - 1
    err64 = oracle.rel_l2(u64, ref)
    print(f"centre: closed form {ref[c, c]:.6f} FP64 {u64[c, c]:.6f} FP32 {u32[c, c]:.6f}; "
          f"FP64 rel-L2 {err64:.3e}", flush=True)
    # 59375 FP64 steps: rounding of about 1e-16 per step and cell, averaging
    # out over the steps (about sqrt(59375) x 1e-16 = 2.4e-14 per cell in a
    # random walk; measured 2.5e-12: the rounding of a smooth field is
    # correlated from step to step); bar 1e-11
    assert err64 <= 1e-11
    # total + outflow: FP64 to rounding, FP32 to its states' drift
    s0 = float(u0.sum())
    d64 = (u64.sum() + out64 - s0) / s0
    d32 = (u32.sum() + out32 - s0) / s0
    print(f"total + outflow - initial: FP64 {d64:.3e}, FP32 {d32:.3e} of the initial total", flush=True)
    assert abs(d64) <= 1e-12
    assert abs(d32) <= 1e-3
    d = np.abs(u32 - u64)
    print(f"FP32 vs FP64, percent of cells: |err| > 0.1: {100 * np.mean(d > 0.1):.2f}, "
          f"> 0.5: {100 * np.mean(d > 0.5):.2f}, > 1.0: {100 * np.mean(d > 1.0):.2f}; max {d.max():.4f}", flush=True)
