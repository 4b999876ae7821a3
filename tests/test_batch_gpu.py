"""GPU parity of the batched ensemble: many 2D grids of uneven sizes and
coefficients in one launch per pass, against the oracle grid by grid."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import check, oracle_ref, to_device, to_host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("bc", ["zero", "periodic"])
def test_batch_matches_oracle_per_grid(dtype, bc):
    import paper_2303_08365_amd as st
    import torch
    shapes = synth.batch_shapes(7, seed=3, lo=24, hi=700)
    alphas = synth.batch_alphas(7, seed=3)
    offs = synth.star_offsets(2, 1)
    steps = [9, 9, 4, 0, 13, 1, 9]
    bp = st.BatchPlan(offs, shapes, dtype, bc)
    u0s = [synth.uniform_field(s, seed=10 + g) for g, s in enumerate(shapes)]
    coeffs = [synth.heat_weights(2, a, "f64" if dtype == "f64" else "f32") for a in alphas]
    grids = [to_device(u, dtype) for u in u0s]
    works = [torch.empty_like(g) for g in grids]
    bp.run(grids, works, coeffs, steps)
    for g in range(len(shapes)):
        ref = oracle.sweep(synth.round_to(u0s[g], dtype), offs, coeffs[g], steps[g], bc=bc)
        got = to_host(grids[g])
        if steps[g] == 0:
            assert np.array_equal(got, synth.round_to(u0s[g], dtype))
        else:
            check(got, ref, dtype, steps[g], f"grid {g} {shapes[g]}")


def test_batch_equals_single_grid_runs_bitwise():
    import paper_2303_08365_amd as st
    import torch
    shapes = [(300, 257), (64, 1100), (513, 40)]
    offs = synth.box_offsets(2, 1)
    coeffs = [synth.box_mean_weights(2, 1, "f32") for _ in shapes]
    bp = st.BatchPlan(offs, shapes, "f32", "periodic")
    u0s = [synth.uniform_field(s, seed=g) for g, s in enumerate(shapes)]
    grids = [to_device(u, "f32") for u in u0s]
    works = [torch.empty_like(g) for g in grids]
    bp.run(grids, works, coeffs, [17, 17, 17])
    tb = bp.info()["tb"]
    for g, s in enumerate(shapes):
        p = st.Plan(offs, s, "f32", "periodic").select(kernel=st.KERNEL_STREAM2D, tb=tb)
        one = to_device(u0s[g], "f32")
        p.run(one, list(coeffs[g]), 17)
        assert np.array_equal(to_host(grids[g]), to_host(one)), g


def test_batch_repeated_calls_reuse_the_table():
    import paper_2303_08365_amd as st
    import torch
    shapes = synth.batch_shapes(5, seed=1, lo=64, hi=512)
    offs = synth.star_offsets(2, 1)
    coeffs = [synth.heat_weights(2, 0.1, "f32")] * 5
    bp = st.BatchPlan(offs, shapes, "f32")
    u0s = [synth.uniform_field(s, seed=g) for g, s in enumerate(shapes)]
    grids = [to_device(u, "f32") for u in u0s]
    works = [torch.empty_like(g) for g in grids]
    for _ in range(3):
        bp.run(grids, works, coeffs, [4] * 5)
    for g in range(5):
        ref = oracle.sweep(synth.round_to(u0s[g], "f32"), offs, coeffs[g], 12)
        check(to_host(grids[g]), ref, "f32", 12, f"grid {g}")


def test_module_batch_run_matches_oracle():
    import paper_2303_08365_amd as st
    offs = synth.star_offsets(2, 1)
    shapes = [(40, 300), (129, 77), (256, 256)]
    alphas = [0.1, 0.2, 0.24]
    steps = [7, 12, 5]
    u0s = [synth.uniform_field(sh, seed=50 + i) for i, sh in enumerate(shapes)]
    grids = [to_device(u, "f64") for u in u0s]
    coeffs = [list(synth.heat_weights(2, a)) for a in alphas]
    st.batch_run(grids, coeffs, offs, steps)
    for g, u, w, t in zip(grids, u0s, coeffs, steps):
        check(to_host(g), oracle_ref(u, offs, w, t, "zero", "f64"), "f64", t, "batch_run")


@pytest.mark.parametrize("tb", [1, 2, 4, 8])
def test_batch_uneven_schedules_at_every_depth(tb):
    # one launch per pass covers every grid; each grid runs its own pass list:
    # remainders, the split that makes a list even, a lone step (copy back),
    # grids that idle in the late passes and a grid with no steps at all
    import paper_2303_08365_amd as st
    import torch
    steps = [0, 1, 2, 3, tb, tb + 1, 2 * tb + 1, 3 * tb, 5 * tb + 3, 7]
    shapes = synth.batch_shapes(len(steps), seed=11, lo=40, hi=600)
    alphas = synth.batch_alphas(len(steps), seed=11)
    offs = synth.star_offsets(2, 1)
    bp = st.BatchPlan(offs, shapes, "f64", "zero").select(kernel=st.KERNEL_STREAM2D, tb=tb)
    print(f"batch tb {tb} plan {bp.info()} steps {steps}", flush=True)
    u0s = [synth.uniform_field(s, seed=30 + g) for g, s in enumerate(shapes)]
    coeffs = [synth.heat_weights(2, a) for a in alphas]
    grids = [to_device(u, "f64") for u in u0s]
    works = [torch.empty_like(g) for g in grids]
    bp.run(grids, works, coeffs, steps)
    for g in range(len(shapes)):
        got = to_host(grids[g])
        if steps[g] == 0:
            assert np.array_equal(got, u0s[g])
        else:
            check(got, oracle.sweep(u0s[g], offs, coeffs[g], steps[g]), "f64", steps[g], f"grid {g} steps {steps[g]}")


def test_batch_graph_survives_outflow_calls_with_other_tables():
    # a graph-captured batch run, then an outflow run of the same plan with
    # more steps (another descriptor table), then the graph again: each replay
    # rewrites its own table, so results equal an eager plan's bit for bit
    import paper_2303_08365_amd as st
    import torch
    shapes = synth.batch_shapes(6, seed=21, lo=64, hi=500)
    offs = synth.star_offsets(2, 1)
    coeffs = [synth.heat_weights(2, a, "f32") for a in synth.batch_alphas(6, seed=21)]
    u0s = [synth.uniform_field(s, seed=60 + g) for g, s in enumerate(shapes)]
    eager = st.BatchPlan(offs, shapes, "f32")
    graph = st.BatchPlan(offs, shapes, "f32", graph=True)
    ga = [to_device(u, "f32") for u in u0s]
    gb = [to_device(u, "f32") for u in u0s]
    wa = [torch.empty_like(x) for x in ga]
    wb = [torch.empty_like(x) for x in gb]
    fa = torch.zeros(6, dtype=torch.float64, device="cuda")
    fb = torch.zeros(6, dtype=torch.float64, device="cuda")
    for rep, (steps, flux) in enumerate([(5, False), (23, True), (5, False), (5, False), (31, True), (5, False)]):
        eager.run(ga, wa, coeffs, [steps] * 6, flux=fa if flux else None)
        graph.run(gb, wb, coeffs, [steps] * 6, flux=fb if flux else None)
        torch.cuda.synchronize()
        for g in range(6):
            assert np.array_equal(to_host(ga[g]), to_host(gb[g])), (rep, g)
        assert np.array_equal(fa.cpu().numpy(), fb.cpu().numpy()), rep


def test_run_calls_record_into_a_callers_graph():
    # no run call allocates or waits, so each can be captured into the
    # caller's graph; replays (with other eager work and the same plans used
    # eagerly with other arguments in between) match eager runs
    import paper_2303_08365_amd as st
    import torch
    shp = (48, 40, 200)
    offs3 = synth.star_offsets(3, 1)
    w3 = list(synth.heat_weights(3, 0.15))
    p3 = st.Plan(offs3, shp, "f64")
    u0 = synth.uniform_field(shp, seed=7)
    g = to_device(u0, "f64")
    wk = torch.empty_like(g)
    flux = torch.zeros(1, dtype=torch.float64, device="cuda")
    shapes = synth.batch_shapes(4, seed=8, lo=64, hi=300)
    offs2 = synth.star_offsets(2, 1)
    c2 = [synth.heat_weights(2, 0.2, "f32")] * 4
    bp = st.BatchPlan(offs2, shapes, "f32")
    u2 = [synth.uniform_field(s, seed=80 + i) for i, s in enumerate(shapes)]
    bg = [to_device(u, "f32") for u in u2]
    bw = [torch.empty_like(x) for x in bg]
    bflux = torch.zeros(4, dtype=torch.float64, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            p3.run_flux(g, w3, 6, flux, work=wk)
            bp.run(bg, bw, c2, [5, 0, 9, 3], flux=bflux)
            bp.run(bg, bw, c2, [2, 2, 2, 2])
    torch.cuda.synchronize()
    ref3 = to_device(u0, "f64")
    rf = torch.zeros(1, dtype=torch.float64, device="cuda")
    rp3 = st.Plan(offs3, shp, "f64")
    rbp = st.BatchPlan(offs2, shapes, "f32")
    rbg = [to_device(u, "f32") for u in u2]
    rbw = [torch.empty_like(x) for x in rbg]
    rbf = torch.zeros(4, dtype=torch.float64, device="cuda")
    other = [to_device(u, "f32") for u in u2]
    for rep in range(3):
        graph.replay()
        rp3.run_flux(ref3, w3, 6, rf)
        rbp.run(rbg, rbw, c2, [5, 0, 9, 3], flux=rbf)
        rbp.run(rbg, rbw, c2, [2, 2, 2, 2])
        # the captured plan used eagerly with other arguments in between
        bp.run(other, [torch.empty_like(x) for x in other], c2, [3, 1, 4, 1])
        torch.cuda.synchronize()
        assert np.array_equal(to_host(g), to_host(ref3)), rep
        assert np.array_equal(flux.cpu().numpy(), rf.cpu().numpy()), rep
        for i in range(4):
            assert np.array_equal(to_host(bg[i]), to_host(rbg[i])), (rep, i)
        assert np.array_equal(bflux.cpu().numpy(), rbf.cpu().numpy()), rep
