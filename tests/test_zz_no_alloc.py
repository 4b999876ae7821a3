"""stencil_run_noalloc (the run call that allocates nothing: its ping-pong
buffer is the library's static device work space) against stencil_run with a
caller's work buffer, through the C ABI, on consecutive calls that shrink the
input, and against the FP64 oracle."""
import numpy as np
import pytest

import synth
from gpu_helpers import TOL, oracle_ref, to_device, to_host

import oracle

pytestmark = pytest.mark.gpu


def _pair(offs, shape, dtype, bc, w, steps, seed):
    """Run the same steps through stencil_run (caller's work buffer) and
    stencil_run_noalloc (static work space); return both results and the
    oracle's."""
    import paper_2303_08365_amd as st
    import torch
    u0 = synth.uniform_field(shape, seed=seed)
    plan = st.Plan(offs, shape, dtype, bc)
    a = to_device(u0, dtype)
    b = to_device(u0, dtype)
    plan.run(a, w, steps, work=torch.empty_like(a))
    plan.run_noalloc(b, w, steps)
    print(f"noalloc {dtype} {bc} {shape} steps {steps} plan {plan.info()}", flush=True)
    return to_host(a), to_host(b), oracle_ref(u0, offs, w, steps, bc, dtype)


def test_noalloc_matches_stencil_run_on_consecutive_shrinking_calls():
    # 3D 7-point heat FP64 (several tiles, ragged), then a smaller FP32 grid
    # under the periodic rule, then a single-step call (odd pass list: the
    # result comes back from the static space by a copy), then a small 2D grid
    cases = [
        (synth.star_offsets(3, 1), (40, 48, 200), "f64", "zero", list(synth.heat_weights(3, 0.15)), 9, 3),
        (synth.star_offsets(3, 1), (17, 29, 31), "f32", "periodic",
         list(synth.heat_weights(3, 0.15, "f32")), 7, 4),
        (synth.star_offsets(3, 1), (12, 20, 70), "f64", "zero", list(synth.heat_weights(3, 0.1)), 1, 5),
        (synth.box_offsets(2, 1), (37, 53), "f32", "zero", list(synth.box_mean_weights(2, 1, "f32")), 5, 6),
    ]
    for offs, shape, dtype, bc, w, steps, seed in cases:
        got_run, got_noalloc, ref = _pair(offs, shape, dtype, bc, w, steps, seed)
        # same passes, same kernels: bit for bit
        assert np.array_equal(got_run, got_noalloc), (shape, dtype)
        err = oracle.rel_l2(got_noalloc, ref)
        assert err <= TOL[dtype], (shape, dtype, err)


def test_noalloc_composes_and_records_into_a_callers_graph():
    # run(a) then run(b) equals run(a + b); a captured call replays like an
    # eager one (replays interleaved with eager calls on other grids that
    # reuse the same static space)
    import paper_2303_08365_amd as st
    import torch
    shape = (24, 40, 130)
    offs = synth.star_offsets(3, 1)
    w = list(synth.heat_weights(3, 0.15))
    u0 = synth.uniform_field(shape, seed=11)
    plan = st.Plan(offs, shape, "f64")
    one = to_device(u0, "f64")
    plan.run_noalloc(one, w, 4)
    plan.run_noalloc(one, w, 6)
    ref = to_device(u0, "f64")
    plan.run(ref, w, 10, work=torch.empty_like(ref))
    assert np.array_equal(to_host(one), to_host(ref))

    g = to_device(u0, "f64")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            plan.run_noalloc(g, w, 8)
    torch.cuda.synchronize()
    eager = to_device(u0, "f64")
    small = st.Plan(offs, (9, 16, 70), "f64")
    other = to_device(synth.uniform_field((9, 16, 70), seed=12), "f64")
    for rep in range(3):
        graph.replay()
        plan.run_noalloc(eager, w, 8)
        small.run_noalloc(other, w, 3)
        torch.cuda.synchronize()
        assert np.array_equal(to_host(g), to_host(eager)), rep
