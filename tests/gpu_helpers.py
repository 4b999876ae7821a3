"""Shared helpers for the GPU parity tests (run the HIP path through the C ABI
binding; compare with the oracle on the same seeded inputs)."""
import numpy as np

import oracle
import synth

# Parity bars.  FP64 and FP32 are the stated tolerances on relative L2 after
# all steps.  bfloat16 storage rounds every step's result; bfloat16 keeps 8
# significant bits (7 stored, 1 implicit), so a round to nearest errs by at
# most 2**-8 of the value.  The step is non-expansive in the max norm when the
# absolute weights sum to at most 1, so after T steps every cell is within
# T * 2**-8 * max|u| of the exact value (checked per cell), and the relative L2
# is bounded by T * 2**-8 * max|u| / rms(u).
TOL = {"f64": 1e-12, "f32": 1e-5}

_TORCH_DT = {"f64": "float64", "f32": "float32", "bf16": "bfloat16"}


def bf16_tol(u_ref, steps):
    u = np.asarray(u_ref, dtype=np.float64)
    rms = float(np.sqrt(np.mean(u * u)))
    return max(1, steps) * 2.0 ** -8 * float(np.max(np.abs(u))) / max(rms, 1e-300)


def to_device(a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(
        device="cuda", dtype=getattr(torch, _TORCH_DT[dtype])).contiguous()


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.to(dtype=torch.float64).cpu().numpy()


def gpu_sweep(u0, offsets, weights, steps, bc="zero", dtype="f64", select=None, plan=None,
              work=None):
    """Run the HIP path; returns (result FP64 numpy, plan info)."""
    import paper_2303_08365_amd as st
    g = to_device(u0, dtype)
    if plan is None:
        plan = st.Plan(offsets, u0.shape, dtype, bc)
    if select is not None:
        plan.select(**select)
    plan.run(g, list(weights), steps, work=work)
    return to_host(g), plan.info()


def oracle_ref(u0, offsets, weights, steps, bc="zero", dtype="f64"):
    """Oracle on the storage-rounded inputs and compute-rounded weights."""
    wdt = "f64" if dtype == "f64" else "f32"
    return oracle.sweep(synth.round_to(u0, dtype), offsets, synth.round_to(np.asarray(weights), wdt),
                        steps, bc=bc)


def check(got, ref, dtype, steps, what=""):
    err = oracle.rel_l2(got, ref)
    tol = bf16_tol(ref, steps) if dtype == "bf16" else TOL[dtype]
    assert err <= tol, f"{what} rel-L2 {err:.3e} > {tol:.1e}"
    if dtype == "bf16":
        # per cell: the non-expansive bound T * 2^-8 * max|u| itself
        worst = float(np.max(np.abs(np.asarray(got) - np.asarray(ref))))
        bound = max(1, steps) * 2.0 ** -8 * float(np.max(np.abs(ref)))
        assert worst <= bound, f"{what} max |delta| {worst:.3e} > {bound:.3e}"
    return err
