"""GPU: outflow across the zero-rule boundary (stencil_run_flux) against the
oracle's FP64 outflow, on the same seeded inputs; the grid must end
bit-identical to stencil_run's; fused (in-pass) and one-step (band kernel)
sums must agree; at the full 512^3 heat size, total + outflow must stay
equal to the initial total."""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import TOL, check, oracle_ref, to_device, to_host

pytestmark = pytest.mark.gpu


def _run_flux(plan, u0, w, steps, dtype, flux0=0.0):
    import torch
    g = to_device(u0, dtype)
    f = torch.full((1,), flux0, dtype=torch.float64, device="cuda")
    plan.run_flux(g, list(w), steps, f)
    return to_host(g), float(f.cpu()[0])


def _ref_flux(u0, offs, w, steps, dtype):
    wdt = "f64" if dtype == "f64" else "f32"
    return oracle.sweep_flux(synth.round_to(u0, dtype), offs, synth.round_to(np.asarray(w), wdt), steps)


def _flux_tol(offs, w, shape, steps, dtype, u0):
    if dtype != "bf16":
        return TOL[dtype]
    # each state differs from the exact one by at most t * 2^-8 * max|u0|; the
    # step's outflow weighs the band with the leaving weights (sum W_leave)
    _, wleave = oracle.sweep_flux(np.ones(shape), offs, np.abs(np.asarray(w)), 1)
    return wleave * steps * steps * 2.0 ** -8 * float(np.max(np.abs(u0)))


def _close(got, ref, tol, dtype, what):
    if dtype == "bf16":
        assert abs(got - ref) <= tol, f"{what}: outflow {got!r} vs oracle {ref!r} (bound {tol:.3e})"
    else:
        assert abs(got - ref) <= tol * abs(ref), f"{what}: outflow {got!r} vs oracle {ref!r} rel {tol:.0e}"


CASES_3D = {
    "f64": [(20, 70, 300), (13, 29, 131), (5, 9, 7)],
    "f32": [(16, 45, 520), (11, 33, 259), (4, 6, 5)],
    "bf16": [(9, 40, 520), (7, 21, 97)],
}


@pytest.mark.parametrize("dtype,shape", [(d, s) for d, ss in CASES_3D.items() for s in ss])
def test_3d_heat_outflow_matches_oracle(dtype, shape):
    import paper_2303_08365_amd as st
    offs = synth.star_offsets(3, 1)
    w = synth.heat_weights(3, 0.15, "f64" if dtype == "f64" else "f32")
    steps = 9 if dtype != "bf16" else 5
    u0 = synth.uniform_field(shape, seed=21)
    print(f"flux 3d {dtype} {shape} steps {steps}", flush=True)
    plan = st.Plan(offs, shape, dtype, "zero")
    got, out = _run_flux(plan, u0, w, steps, dtype)
    ref, rout = _ref_flux(u0, offs, w, steps, dtype)
    check(got, ref, dtype, steps, "state")
    _close(out, rout, _flux_tol(offs, w, shape, steps, dtype, u0), dtype, f"{dtype} {shape}")
    # the grid is the one stencil_run gives, bit for bit
    g = to_device(u0, dtype)
    plan.run(g, list(w), steps)
    assert np.array_equal(to_host(g), got)


@pytest.mark.parametrize("dtype,shape", [("f64", (19, 70, 300)), ("f32", (14, 70, 520))])
def test_3d_outflow_every_pipeline_tiling(dtype, shape):
    # every candidate of the 7-point pipeline (registers or LDS queue, late or
    # early partial sums, with an outflow twin of its own or standing in for
    # one): the oracle's outflow, and the grid stencil_run gives, bit for bit
    import paper_2303_08365_amd as st
    offs = synth.star_offsets(3, 1)
    w = synth.heat_weights(3, 0.15, dtype)
    steps = 9
    u0 = synth.uniform_field(shape, seed=23)
    ref, rout = _ref_flux(u0, offs, w, steps, dtype)
    plan = st.Plan(offs, shape, dtype, "zero")
    ks = [k for k, c in enumerate(plan.candidates()) if c["kernel"] == 2 and c["pipeline"]]
    assert any(plan.candidates()[k]["pipeline"] >= 100 for k in ks), "no LDS-queue candidate"
    for k in ks:
        c = plan.candidates()[k]
        print(f"flux pipeline {dtype} {shape} cand {k} tb {c['tb']} pipe {c['pipeline']}", flush=True)
        plan.select(variant=k)
        got, out = _run_flux(plan, u0, w, steps, dtype)
        check(got, ref, dtype, steps, f"cand {k}")
        _close(out, rout, TOL[dtype], dtype, f"cand {k}")
        g = to_device(u0, dtype)
        plan.run(g, list(w), steps)
        assert np.array_equal(to_host(g), got), f"cand {k}: outflow run and plain run differ"


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("shape", [(24, 61, 530), (20, 40, 520), (300, 1100), (45, 77)])
def test_fused_and_one_step_outflow_agree(dtype, shape):
    # the fused twin sums inside its passes; the naive candidate runs one step
    # per pass with the band kernel: same states, sums in another order
    import paper_2303_08365_amd as st
    nd = len(shape)
    offs = synth.star_offsets(nd, 1)
    w = synth.heat_weights(nd, 0.15 if nd == 3 else 0.2, "f64" if dtype == "f64" else "f32")
    u0 = synth.uniform_field(shape, seed=22)
    plan = st.Plan(offs, shape, dtype, "zero")
    print(f"flux fused/band {dtype} plan {plan.info()}", flush=True)
    g1, f1 = _run_flux(plan, u0, w, 10, dtype)
    plan.select(kernel=0)
    g2, f2 = _run_flux(plan, u0, w, 10, dtype)
    assert np.array_equal(g1, g2)
    # FP64: the same products, summed in another order.  FP32 compute (3D):
    # the fused kernels first add up an x-face column in FP32 -- the
    # queued-plane kernel its K = 4 rows of one state, the pipeline its K rows
    # of the T_b = 4 states of one iteration, at most m = 16 values -- each
    # such sum off by at most (m - 1) * 2^-24 of itself (values >= 0); the
    # outflow adds N of them, with rounding errors of either sign, so the
    # total's relative error is of order (m - 1) * 2^-24 / sqrt(N): the bar is
    # ten times that, with N counted for the larger sums.  2D kernels add face
    # cells in FP64 directly.
    if dtype == "f64" or nd == 2:
        tol = 1e-13
    else:
        nz, ny, nx = shape
        m = 16
        n_sums = 2 * nz * ((ny + 3) // 4) * (10 // 4 + 1)  # two x faces, per wave, per iteration of 4 states
        tol = 10 * (m - 1) * 2.0 ** -24 / math.sqrt(n_sums)
    print(f"fused vs band outflow: relative gap {abs(f1 - f2) / abs(f2):.2e}, bar {tol:.2e}", flush=True)
    assert abs(f1 - f2) <= tol * abs(f2), (f1, f2)


@pytest.mark.parametrize("dtype,kind,r,shape", [
    ("f64", "star", 1, (512, 512)), ("f32", "box", 1, (130, 301)), ("f64", "star", 2, (67, 90)),
    ("f32", "star", 2, (14, 23, 40)), ("f64", "box", 1, (9, 12, 17)), ("bf16", "star", 1, (100, 260)),
    ("f64", "star", 3, (41,)), ("f64", "star", 1, (5000,)), ("f32", "star", 2, (3001,)),
    ("f64", "box", 1, (20, 33, 300)),
])
def test_other_patterns_outflow_matches_oracle(dtype, kind, r, shape):
    import paper_2303_08365_amd as st
    nd = len(shape)
    pattern = f"{kind}{nd}d r{r}"
    offs = synth.box_offsets(nd, r) if kind == "box" else synth.star_offsets(nd, r)
    rng = np.random.default_rng(23)
    wr = rng.uniform(0.2, 1.0, len(offs))
    w = synth.adjust_centre(wr / wr.sum(), "f64" if dtype == "f64" else "f32")
    steps = 7 if dtype != "bf16" else 4
    u0 = synth.uniform_field(shape, seed=24)
    print(f"flux {pattern} {dtype} {shape}", flush=True)
    plan = st.Plan(offs, shape, dtype, "zero")
    got, out = _run_flux(plan, u0, w, steps, dtype)
    ref, rout = _ref_flux(u0, offs, w, steps, dtype)
    check(got, ref, dtype, steps, "state")
    _close(out, rout, _flux_tol(offs, w, shape, steps, dtype, u0), dtype, f"{pattern} {dtype} {shape}")


def test_outflow_accumulates_and_edge_cases():
    import torch
    import paper_2303_08365_amd as st
    offs = synth.star_offsets(3, 1)
    w = synth.heat_weights(3, 0.15)
    shape = (18, 40, 260)
    u0 = synth.uniform_field(shape, seed=25)
    plan = st.Plan(offs, shape, "f64", "zero")
    # run(a) + run(b) adds up to run(a + b); the accumulator is added to
    _, whole = _run_flux(plan, u0, w, 11, "f64")
    g = to_device(u0, "f64")
    f = torch.full((1,), 5.0, dtype=torch.float64, device="cuda")
    plan.run_flux(g, list(w), 4, f)
    plan.run_flux(g, list(w), 7, f)
    assert abs((float(f.cpu()[0]) - 5.0) - whole) <= 1e-12 * whole
    # no steps: nothing added
    plan.run_flux(g, list(w), 0, f)
    assert float(f.cpu()[0]) == pytest.approx(5.0 + whole, rel=1e-12)
    # periodic: nothing leaves, the accumulator is untouched
    pplan = st.Plan(offs, shape, "f64", "periodic")
    gp = to_device(u0, "f64")
    fp = torch.full((1,), 3.25, dtype=torch.float64, device="cuda")
    pplan.run_flux(gp, list(w), 5, fp)
    assert float(fp.cpu()[0]) == 3.25
    with pytest.raises(ValueError):
        plan.run_flux(g, list(w), 1, torch.zeros(2, dtype=torch.float64, device="cuda"))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_heat3d_512_total_plus_outflow_is_conserved(dtype):
    # full size, the default plan: with weights summing to 1 (up to one
    # rounding) sum(u_T) + outflow = sum(u_0) up to rounding
    import torch
    import paper_2303_08365_amd as st
    shape = (512, 512, 512)
    offs = synth.star_offsets(3, 1)
    w = synth.heat_weights(3, 0.15, dtype)
    assert abs(float(np.sum(np.asarray(w, dtype=np.float64))) - 1.0) <= 1e-15
    u0 = synth.uniform_field(shape, seed=26)
    g = to_device(u0, dtype)
    s0 = float(g.double().sum())
    plan = st.Plan(offs, shape, dtype, "zero")
    print(f"flux heat3d 512^3 {dtype} plan {plan.info()}", flush=True)
    f = torch.zeros(1, dtype=torch.float64, device="cuda")
    plan.run_flux(g, list(w), 100, f)
    sT = float(g.double().sum())
    out = float(f.cpu()[0])
    drift = abs(s0 - sT - out) / s0
    print(f"heat3d 512^3 {dtype}: sum0 {s0:.17g} sumT {sT:.17g} outflow {out:.17g} drift {drift:.3e}",
          flush=True)
    assert out > 0
    assert drift <= (1e-13 if dtype == "f64" else 1e-5)


@pytest.mark.parametrize("dtype,kind", [("f64", "star"), ("f32", "star"), ("f64", "box"), ("bf16", "star")])
def test_batch_outflow_matches_oracle_per_grid(dtype, kind):
    import torch
    import paper_2303_08365_amd as st
    offs = synth.star_offsets(2, 1) if kind == "star" else synth.box_offsets(2, 1)
    shapes = [(40, 300), (129, 77), (256, 516), (33, 1030)]
    steps = [9, 4, 13, 6] if dtype != "bf16" else [4, 3, 5, 2]
    wdt = "f64" if dtype == "f64" else "f32"
    rng = np.random.default_rng(61)
    coeffs = []
    for _ in shapes:
        r = rng.uniform(0.2, 1.0, len(offs))
        coeffs.append(list(synth.adjust_centre(r / r.sum(), wdt)))
    u0s = [synth.uniform_field(sh, seed=62 + i) for i, sh in enumerate(shapes)]
    plan = st.BatchPlan(offs, shapes, dtype, "zero")
    print(f"batch flux {dtype} {kind} plan {plan.info()}", flush=True)
    grids = [to_device(u, dtype) for u in u0s]
    works = [torch.empty_like(g) for g in grids]
    flux = torch.full((len(shapes),), 0.5, dtype=torch.float64, device="cuda")
    plan.run(grids, works, coeffs, steps, flux=flux)
    out = flux.cpu().numpy() - 0.5
    plain = [to_device(u, dtype) for u in u0s]
    plan.run(plain, works, coeffs, steps)
    for g, (u0, w, t, got_g, pl) in enumerate(zip(u0s, coeffs, steps, grids, plain)):
        ref, rout = _ref_flux(u0, offs, w, t, dtype)
        h = to_host(got_g)
        check(h, ref, dtype, t, f"grid {g}")
        assert np.array_equal(h, to_host(pl)), g
        tol = _flux_tol(offs, w, u0.shape, t, dtype, u0)
        _close(out[g], rout, tol, dtype, f"batch grid {g}")


def test_batch_outflow_periodic_untouched():
    import torch
    import paper_2303_08365_amd as st
    offs = synth.star_offsets(2, 1)
    shapes = [(40, 300), (64, 64)]
    plan = st.BatchPlan(offs, shapes, "f64", "periodic")
    grids = [to_device(synth.uniform_field(sh, seed=70), "f64") for sh in shapes]
    works = [torch.empty_like(g) for g in grids]
    flux = torch.full((2,), 1.25, dtype=torch.float64, device="cuda")
    plan.run(grids, works, [list(synth.heat_weights(2, 0.2))] * 2, [5, 5], flux=flux)
    assert np.array_equal(flux.cpu().numpy(), np.array([1.25, 1.25]))
