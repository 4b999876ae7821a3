"""HIP-graph replay and autotuning.  Every graph replay is checked against
the eager result, with the program's own eager work and synchronisations
between replays; autotuned plans must still match the oracle."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import check, gpu_sweep, oracle_ref, to_device, to_host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("case", ["heat2d", "heat3d", "odd_single_steps"])
def test_graph_replays_match_eager(case):
    import paper_2303_08365_amd as st
    import torch
    if case == "heat2d":
        offs, shape, w, steps, sel = synth.star_offsets(2, 1), (300, 517), synth.heat_weights(2, 0.2), 13, None
    elif case == "heat3d":
        offs, shape, w, steps, sel = synth.star_offsets(3, 1), (40, 70, 260), synth.heat_weights(3, 0.15), 9, None
    else:  # one-step passes, odd count: the run ends with a device copy node
        offs, shape, w, steps, sel = synth.star_offsets(2, 1), (64, 256), synth.heat_weights(2, 0.1), 7, {"tb": 1}
    u0 = synth.uniform_field(shape, seed=3)
    eager = st.Plan(offs, shape, "f64")
    graph = st.Plan(offs, shape, "f64", graph=True)
    if sel:
        eager.select(**sel)
        graph.select(**sel)
    ref = to_device(u0, "f64")
    g = to_device(u0, "f64")
    wk_e = torch.empty_like(ref)
    wk_g = torch.empty_like(g)
    for rep in range(4):
        eager.run(ref, list(w), steps, work=wk_e)
        graph.run(g, list(w), steps, work=wk_g)
        # unrelated eager work between replays
        scratch = torch.full((1 << 20,), float(rep), device="cuda")
        scratch.mul_(2.0)
        torch.cuda.synchronize()
        assert np.array_equal(to_host(g), to_host(ref)), rep
    check(to_host(g), oracle_ref(u0, offs, w, 4 * steps), "f64", 4 * steps, case)


def test_batch_graph_and_autotune():
    import paper_2303_08365_amd as st
    import torch
    shapes = synth.batch_shapes(9, seed=5, lo=200, hi=900)
    alphas = synth.batch_alphas(9, seed=5)
    offs = synth.star_offsets(2, 1)
    coeffs = [synth.heat_weights(2, a, "f32") for a in alphas]
    u0s = [synth.uniform_field(s, seed=g) for g, s in enumerate(shapes)]
    plain = st.BatchPlan(offs, shapes, "f32")
    tuned = st.BatchPlan(offs, shapes, "f32", autotune=True, graph=True)
    print("autotuned batch plan", tuned.info(), flush=True)
    tuned_tb = tuned.info()["tb"]
    plain.select(variant=tuned.info()["variant"])
    ga = [to_device(u, "f32") for u in u0s]
    gb = [to_device(u, "f32") for u in u0s]
    wa = [torch.empty_like(x) for x in ga]
    wb = [torch.empty_like(x) for x in gb]
    steps = [11] * 9
    for rep in range(3):
        plain.run(ga, wa, coeffs, steps)
        tuned.run(gb, wb, coeffs, steps)
        torch.cuda.synchronize()
        for a, b in zip(ga, gb):
            assert np.array_equal(to_host(a), to_host(b)), rep
    for gi in range(9):
        ref = oracle.sweep(synth.round_to(u0s[gi], "f32"), offs, coeffs[gi], 33)
        check(to_host(gb[gi]), ref, "f32", 33, f"grid {gi} tb {tuned_tb}")


def test_autotuned_single_grid_plan_matches_oracle():
    import paper_2303_08365_amd as st
    offs = synth.star_offsets(3, 1)
    shape = (48, 64, 256)
    w = synth.heat_weights(3, 0.15)
    p = st.Plan(offs, shape, "f64", autotune=True)
    print("autotuned plan", p.info(), flush=True)
    u0 = synth.uniform_field(shape, seed=1)
    g = to_device(u0, "f64")
    p.run(g, list(w), 10)
    check(to_host(g), oracle_ref(u0, offs, w, 10), "f64", 10, "autotuned")


def test_autotune_cache_reuses_and_honours_stored_choice(tmp_path):
    import paper_2303_08365_amd as st
    path = tmp_path / "tune.txt"
    st.autotune_cache(str(path))
    try:
        offs = synth.star_offsets(2, 1)
        shape = (301, 700)
        p1 = st.Plan(offs, shape, "f32", "zero", autotune=True)
        # the file holds every choice of this process; ours is the 301 x 700 grid
        lines = [ln for ln in path.read_text().splitlines() if " grid 1x301x700 " in ln and " t1 " in ln]
        assert len(lines) == 1
        key, idx, n = lines[0].split("\t")
        assert int(idx) == p1.info()["variant"] and int(n) == p1.info()["ncandidates"]
        p2 = st.Plan(offs, shape, "f32", "zero", autotune=True)
        assert p2.info()["variant"] == p1.info()["variant"]
        # a stored choice is taken as it is, without timing
        other = (int(idx) + 1) % int(n)
        path.write_text(f"{key}\t{other}\t{n}\n")
        st.autotune_cache(str(path))
        p3 = st.Plan(offs, shape, "f32", "zero", autotune=True)
        assert p3.info()["variant"] == other
        w = synth.heat_weights(2, 0.2, "f32")
        u0 = synth.uniform_field(shape, seed=41)
        got, _ = gpu_sweep(u0, offs, w, 9, "zero", "f32", plan=p3)
        check(got, oracle_ref(u0, offs, w, 9, "zero", "f32"), "f32", 9, "cached choice")
    finally:
        st.autotune_cache(None)
