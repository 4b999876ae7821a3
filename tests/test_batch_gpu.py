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
