"""GPU parity: the HIP sweep (through the C ABI) against the FP64 oracle,
element by element on the same seeded inputs, at sizes that span several
tiles and ragged tails; every tiling candidate of a plan against the
one-step kernel bit for bit; edge cases."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import check, gpu_sweep, oracle_ref, to_device, to_host

pytestmark = pytest.mark.gpu


def _weights(offsets, seed=0, dtype="f64"):
    # stable positive weights summing to 1, centre-adjusted for the dtype
    r = np.random.default_rng(seed).random(len(offsets))
    w = r / r.sum()
    return synth.adjust_centre(w, "f64" if dtype == "f64" else "f32")


# ---------------------------------------------------------------------------
# 2D: star and box, every candidate, both boundaries, all storage types
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("bc", ["zero", "periodic"])
@pytest.mark.parametrize("pattern", ["star", "box", "star_r2", "box_r2"])
@pytest.mark.parametrize("shape", [(37, 53), (130, 300), (257, 515)])
def test_2d_all_candidates_match_oracle(dtype, bc, pattern, shape):
    import paper_2303_08365_amd as st
    r = 2 if pattern.endswith("_r2") else 1
    offs = synth.star_offsets(2, r) if pattern.startswith("star") else synth.box_offsets(2, r)
    w = _weights(offs, 1, dtype)
    steps = 4 if dtype == "bf16" else 11
    u0 = synth.uniform_field(shape, seed=2)
    ref = oracle_ref(u0, offs, w, steps, bc, dtype)
    plan = st.Plan(offs, shape, dtype, bc)
    cands = plan.candidates()
    results = []
    for k, c in enumerate(cands):
        got, info = gpu_sweep(u0, offs, w, steps, bc, dtype, select={"variant": k}, plan=plan)
        assert info["variant"] == k
        print(f"2d {dtype} {bc} {pattern} {shape} cand {k} kernel {c['kernel']} tb {c['tb']}", flush=True)
        check(got, ref, dtype, steps, f"cand {k}")
        results.append(got)
    for k, r in enumerate(results[1:], 1):
        assert np.array_equal(r, results[0]), f"candidate {k} differs bitwise from candidate 0"


# ---------------------------------------------------------------------------
# 3D stars: radius 1 (7-point) and 4 (25-point)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("bc", ["zero", "periodic"])
@pytest.mark.parametrize("shape", [(17, 29, 31), (21, 40, 150), (12, 70, 260)])
def test_3d_star7_all_candidates_match_oracle(dtype, bc, shape):
    import paper_2303_08365_amd as st
    offs = synth.star_offsets(3, 1)
    w = _weights(offs, 3, dtype)
    steps = 3 if dtype == "bf16" else 7
    u0 = synth.uniform_field(shape, seed=4)
    ref = oracle_ref(u0, offs, w, steps, bc, dtype)
    plan = st.Plan(offs, shape, dtype, bc)
    results = []
    for k, c in enumerate(plan.candidates()):
        print(f"3d7 {dtype} {bc} {shape} cand {k} kernel {c['kernel']} tb {c['tb']}", flush=True)
        got, _ = gpu_sweep(u0, offs, w, steps, bc, dtype, select={"variant": k}, plan=plan)
        check(got, ref, dtype, steps, f"cand {k}")
        results.append(got)
    for k, r in enumerate(results[1:], 1):
        assert np.array_equal(r, results[0]), f"candidate {k} differs bitwise"


@pytest.mark.parametrize("dtype", ["f32", "f64", "bf16"])
@pytest.mark.parametrize("bc", ["periodic", "zero"])
@pytest.mark.parametrize("shape", [(13, 21, 37), (18, 40, 300)])
def test_3d_star25_matches_oracle(dtype, bc, shape):
    import paper_2303_08365_amd as st
    offs = synth.star_offsets(3, 4)
    w = synth.star25_weights(0, "f64" if dtype == "f64" else "f32")
    steps = 2 if dtype == "bf16" else 3
    u0 = synth.uniform_field(shape, seed=5)
    ref = oracle_ref(u0, offs, w, steps, bc, dtype)
    plan = st.Plan(offs, shape, dtype, bc)
    results = []
    for k, c in enumerate(plan.candidates()):
        print(f"3d25 {dtype} {bc} {shape} cand {k} kernel {c['kernel']} tb {c['tb']}", flush=True)
        got, _ = gpu_sweep(u0, offs, w, steps, bc, dtype, select={"variant": k}, plan=plan)
        check(got, ref, dtype, steps, f"cand {k}")
        results.append(got)
    for k, r in enumerate(results[1:], 1):
        assert np.array_equal(r, results[0]), f"candidate {k} differs bitwise"


# ---------------------------------------------------------------------------
# general patterns, 1D, 3D box (one-step kernel)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("case", ["asym2d", "star1d5", "box3d27", "star2d9", "box2d25", "heat1d"])
@pytest.mark.parametrize("bc", ["zero", "periodic"])
def test_general_patterns_match_oracle(case, bc):
    offs, shape = {
        "asym2d": ([(0, 0), (-1, 0), (0, 2), (1, -1), (0, -3)], (33, 47)),
        "star1d5": (synth.star_offsets(1, 2), (1001,)),
        "box3d27": (synth.box_offsets(3, 1), (9, 14, 23)),
        "star2d9": (synth.star_offsets(2, 2), (40, 61)),
        "box2d25": (synth.box_offsets(2, 2), (29, 35)),
        "heat1d": (synth.star_offsets(1, 1), (777,)),
    }[case]
    w = _weights(offs, 7)
    u0 = synth.uniform_field(shape, seed=8)
    got, info = gpu_sweep(u0, offs, w, 6, bc, "f64")
    check(got, oracle_ref(u0, offs, w, 6, bc, "f64"), "f64", 6, case)


# ---------------------------------------------------------------------------
# heat configurations in their literal increment form
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("ndim,shape,alpha,steps", [(2, (64, 96), 0.2, 30), (3, (20, 24, 130), 0.15, 12)])
def test_heat_form_matches_oracle_heat(ndim, shape, alpha, steps):
    offs = synth.star_offsets(ndim, 1)
    u0 = synth.uniform_field(shape, seed=0)
    got, _ = gpu_sweep(u0, offs, synth.heat_weights(ndim, alpha), steps, "zero", "f64")
    check(got, oracle.heat(u0, alpha, steps, bc="zero"), "f64", steps, "heat")
    got32, _ = gpu_sweep(u0, offs, synth.heat_weights(ndim, alpha, "f32"), steps, "zero", "f32")
    a32 = float(synth.round_to(np.array([alpha]), "f32")[0])
    check(got32, oracle.heat(synth.round_to(u0, "f32"), a32, steps, bc="zero"), "f32", steps, "heat f32")


# ---------------------------------------------------------------------------
# edge cases
# ---------------------------------------------------------------------------
def test_composability_is_bitwise():
    import paper_2303_08365_amd as st
    for offs, shape in [(synth.star_offsets(3, 1), (19, 33, 140)), (synth.box_offsets(2, 1), (70, 300))]:
        w = _weights(offs, 2)
        u0 = synth.uniform_field(shape, seed=1)
        plan = st.Plan(offs, shape, "f64")
        g = to_device(u0, "f64")
        plan.run(g, list(w), 3)
        plan.run(g, list(w), 6)
        a = to_host(g)
        b, _ = gpu_sweep(u0, offs, w, 9, plan=plan)
        assert np.array_equal(a, b)


def test_zero_steps_and_identity_weights():
    offs = synth.star_offsets(2, 1)
    u0 = synth.uniform_field((50, 70), seed=3)
    got, _ = gpu_sweep(u0, offs, [0.2] * 5, 0)
    assert np.array_equal(got, u0)
    got, _ = gpu_sweep(u0, offs, [1.0, 0, 0, 0, 0], 9)
    assert np.array_equal(got, u0)


@pytest.mark.parametrize("shape", [(1, 1), (1, 200), (200, 1), (3, 2), (1, 1, 1), (1, 5, 300), (40, 1, 1)])
def test_degenerate_shapes(shape):
    ndim = len(shape)
    offs = synth.star_offsets(ndim, 1)
    w = _weights(offs, 4)
    u0 = synth.uniform_field(shape, seed=9)
    for bc in ("zero", "periodic"):
        got, _ = gpu_sweep(u0, offs, w, 5, bc)
        check(got, oracle_ref(u0, offs, w, 5, bc), "f64", 5, f"{shape} {bc}")


def test_user_work_buffer_and_odd_step_counts():
    import paper_2303_08365_amd as st
    import torch
    offs = synth.star_offsets(3, 1)
    shape = (16, 24, 130)
    w = _weights(offs, 5)
    u0 = synth.uniform_field(shape, seed=6)
    plan = st.Plan(offs, shape, "f64")
    for k, c in enumerate(plan.candidates()):
        for steps in (1, 2, 3, 5):
            work = torch.empty(shape, dtype=torch.float64, device="cuda")
            got, _ = gpu_sweep(u0, offs, w, steps, select={"variant": k}, plan=plan, work=work)
            check(got, oracle_ref(u0, offs, w, steps), "f64", steps, f"cand {k} steps {steps}")


def test_unaligned_rows_take_the_scalar_path():
    # nx not a multiple of the lane width and a base offset that breaks 16-byte
    # alignment: the kernels must fall back to element access
    import paper_2303_08365_amd as st
    import torch
    offs = synth.star_offsets(2, 1)
    shape = (45, 131)
    w = _weights(offs, 6)
    u0 = synth.uniform_field(shape, seed=7)
    base = torch.zeros(shape[0] * shape[1] + 1, dtype=torch.float64, device="cuda")
    g = base[1:].view(shape)
    g.copy_(to_device(u0, "f64"))
    plan = st.Plan(offs, shape, "f64")
    plan.run(g, list(w), 8)
    check(to_host(g), oracle_ref(u0, offs, w, 8), "f64", 8, "unaligned")


@pytest.mark.parametrize("nbytes", [16, 4096 + 48, (1 << 22) + 16 * 7, 3 * (1 << 20) + 5])
def test_streaming_copy_is_exact(nbytes):
    import paper_2303_08365_amd as st
    import torch
    src = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, device="cuda")
    dst = torch.zeros_like(src)
    st.copy(dst, src)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)


# ---------------------------------------------------------------------------
# 1D stars (Tab. 1 Heat-1D, Star-1D5P): every candidate, both rules, all types
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("bc", ["zero", "periodic"])
@pytest.mark.parametrize("radius", [1, 2])
@pytest.mark.parametrize("n", [37, 1000, 4096, 20011, 65536])
def test_1d_star_all_candidates_match_oracle(dtype, bc, radius, n):
    import paper_2303_08365_amd as st
    offs = synth.star_offsets(1, radius)
    w = _weights(offs, 5, dtype)
    steps = 6 if dtype == "bf16" else 70
    u0 = synth.uniform_field((n,), seed=6)
    ref = oracle_ref(u0, offs, w, steps, bc, dtype)
    plan = st.Plan(offs, (n,), dtype, bc)
    results = []
    for k, c in enumerate(plan.candidates()):
        print(f"1d {dtype} {bc} r{radius} n {n} cand {k} kernel {c['kernel']} tb {c['tb']}", flush=True)
        got, _ = gpu_sweep(u0, offs, w, steps, bc, dtype, select={"variant": k}, plan=plan)
        check(got, ref, dtype, steps, f"cand {k}")
        results.append(got)
    assert plan.candidates()[0]["kernel"] == 4 or n < 64 * 16
    for k, r in enumerate(results[1:], 1):
        assert np.array_equal(r, results[0]), f"candidate {k} differs bitwise"


# ---------------------------------------------------------------------------
# 3D boxes (Tab. 1 Box-3D27P): the streaming kernel against the oracle and,
# bit for bit, against the one-step kernel
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("bc", ["zero", "periodic"])
@pytest.mark.parametrize("shape", [(9, 13, 21), (20, 37, 300), (35, 40, 129), (6, 16, 256), (10, 20, 64)])
def test_3d_box27_all_candidates_match_oracle(dtype, bc, shape):
    import paper_2303_08365_amd as st
    offs = synth.box_offsets(3, 1)
    w = _weights(offs, 7, dtype)
    steps = 3 if dtype == "bf16" else 5
    u0 = synth.uniform_field(shape, seed=8)
    ref = oracle_ref(u0, offs, w, steps, bc, dtype)
    plan = st.Plan(offs, shape, dtype, bc)
    assert plan.info()["kernel"] == st.KERNEL_BOX3D
    results = []
    for k, c in enumerate(plan.candidates()):
        print(f"box27 {dtype} {bc} {shape} cand {k} kernel {c['kernel']} tb {c['tb']} chunk {c['tile_z']}", flush=True)
        got, _ = gpu_sweep(u0, offs, w, steps, bc, dtype, select={"variant": k}, plan=plan)
        check(got, ref, dtype, steps, f"cand {k}")
        results.append(got)
    for k, r in enumerate(results[1:], 1):
        assert np.array_equal(r, results[0]), f"candidate {k} differs bitwise"


# 3D boxes, two steps per pass through the partial-sum pipeline (zero rule):
# several tiles in x and y with ragged last tiles, several z chunks with a
# short last one, odd step counts (the last pass takes one step on the
# one-step kernel); every pipeline candidate against the oracle and, bit for
# bit, against the one-step kernel
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("shape,steps", [((13, 50, 260), 4), ((40, 53, 256), 5), ((9, 70, 384), 3),
                                         ((35, 49, 512), 2)])
def test_3d_box27_pipeline_matches_oracle(dtype, shape, steps):
    import paper_2303_08365_amd as st
    offs = synth.box_offsets(3, 1)
    w = _weights(offs, 11, dtype)
    u0 = synth.uniform_field(shape, seed=12)
    ref = oracle_ref(u0, offs, w, steps, "zero", dtype)
    plan = st.Plan(offs, shape, dtype, "zero")
    cands = plan.candidates()
    pipes = [k for k, c in enumerate(cands) if c["pipeline"] > 0]
    assert pipes, f"no pipeline candidate for {shape} {dtype}"
    k1 = next(k for k, c in enumerate(cands) if c["tb"] == 1 and c["kernel"] == st.KERNEL_BOX3D)
    one, _ = gpu_sweep(u0, offs, w, steps, "zero", dtype, select={"variant": k1}, plan=plan)
    # FP64: the pipeline is the plan's default
    assert (cands[0]["pipeline"] > 0) == (dtype == "f64")
    for k in pipes:
        c = cands[k]
        print(f"box27 pipeline {dtype} {shape} steps {steps} cand {k} variant {c['pipeline']} "
              f"tile {c['tile_x']}x{c['tile_y']}x{c['tile_z']} wgs {c['workgroups']}", flush=True)
        got, _ = gpu_sweep(u0, offs, w, steps, "zero", dtype, select={"variant": k}, plan=plan)
        check(got, ref, dtype, steps, f"cand {k}")
        assert np.array_equal(got, one), f"candidate {k} differs bitwise from the one-step kernel"


# the FP64 box pipeline's edge cases: one and two planes, grids exactly one
# register tile high (24 rows; 16 for the 3-column form) or wide (128 / 192
# columns), every step count up to two passes
@pytest.mark.parametrize("shape", [(1, 24, 192), (2, 24, 128), (3, 25, 130), (2, 16, 192)])
@pytest.mark.parametrize("steps", [1, 2, 3, 4])
def test_3d_box27_pipeline_edge_cases(shape, steps):
    import paper_2303_08365_amd as st
    offs = synth.box_offsets(3, 1)
    w = _weights(offs, 13)
    u0 = synth.uniform_field(shape, seed=14)
    ref = oracle_ref(u0, offs, w, steps, "zero", "f64")
    plan = st.Plan(offs, shape, "f64", "zero")
    cands = plan.candidates()
    pipes = [k for k, c in enumerate(cands) if c["pipeline"] > 0]
    if shape[1] >= 24:
        assert cands[0]["pipeline"] == 1
    assert pipes
    k1 = next(k for k, c in enumerate(cands) if c["tb"] == 1 and c["kernel"] == st.KERNEL_BOX3D)
    one, _ = gpu_sweep(u0, offs, w, steps, "zero", "f64", select={"variant": k1}, plan=plan)
    check(one, ref, "f64", steps, "one-step kernel")
    for k in pipes:
        c = cands[k]
        print(f"box27 pipeline edge {shape} steps {steps} cand {k} variant {c['pipeline']} "
              f"tile {c['tile_x']}x{c['tile_y']}x{c['tile_z']}", flush=True)
        got, _ = gpu_sweep(u0, offs, w, steps, "zero", "f64", select={"variant": k}, plan=plan)
        check(got, ref, "f64", steps, f"cand {k}")
        assert np.array_equal(got, one), f"candidate {k} differs bitwise from the one-step kernel"
