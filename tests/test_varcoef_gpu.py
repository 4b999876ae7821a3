"""GPU parity of the differentiable path: variable-coefficient forward with
checkpoints, the fused adjoint (dL/du0 and dL/dk), checkpoint-and-recompute,
the autograd function, finite differences, and the constant-weight
transposed sweep."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import to_device, to_host

pytestmark = pytest.mark.gpu

# FP32 bars for gradients.  dL/du0 is a linear image of dL/du_T and keeps the
# forward bar.  Every dL/dk term multiplies two first differences (u_f - u_j)
# and (lam_j - lam_f) of smooth fields; each difference carries the absolute
# rounding error of its operands (~2**-24 of |u|, |lam|) while its own size is
# smaller by the field's roughness, so the relative error grows by that ratio
# (about 10-100 for these inputs): 1e-4 bounds it with margin.
TOL_F32_GU = 1e-5
TOL_F32_GK = 1e-4


def _inputs(shape, dtype, seed=0):
    u0, k, y = synth.varcoef_inputs(shape, seed=seed)
    return synth.round_to(u0, dtype), synth.round_to(k, dtype), synth.round_to(y, dtype)


def _gpu_forward(u0, k, alpha, steps, dtype, every=0, naive=False):
    import paper_2303_08365_amd as st
    import torch
    plan = st.varcoef_plan(u0.shape, dtype, naive=naive)
    g = to_device(u0, dtype)
    kk = to_device(k, dtype)
    work = torch.empty_like(g)
    ck = None
    if every:
        ck = [torch.empty_like(g) for _ in range(-(-steps // every))]
    plan.run_ckpt(g, kk, alpha, steps, work, every=every, ckpts=ck)
    return g, kk, ck, plan


def _gpu_grads(u0, k, y, alpha, steps, dtype, every, naive=False):
    import torch
    g, kk, ck, plan = _gpu_forward(u0, k, alpha, steps, dtype, every, naive)
    uT = to_host(g)
    M = u0.size
    lam = to_device(2.0 * (uT - y) / M, dtype)
    gk = torch.zeros_like(kk)
    work = torch.empty_like(lam)
    seg = torch.empty((max(min(every, steps) - 1, 1),) + tuple(u0.shape), dtype=lam.dtype, device="cuda")
    plan.adjoint(lam, steps, work, k=kk, alpha=alpha, ckpts=ck, every=every, grad_k=gk, seg=seg)
    return uT, to_host(lam), to_host(gk)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(13, 17, 22), (5, 40, 9)])
def test_varcoef_forward_and_checkpoints_match_oracle(dtype, shape):
    u0, k, _ = _inputs(shape, dtype)
    steps, every, alpha = 11, 4, 0.1
    g, kk, ck, _ = _gpu_forward(u0, k, alpha, steps, dtype, every)
    ref, ref_ck = oracle.varcoef_forward(u0, k, alpha, steps, every=every)
    tol = 1e-12 if dtype == "f64" else 1e-5
    assert oracle.rel_l2(to_host(g), ref) <= tol
    assert len(ck) == ref_ck.shape[0] == 3
    for c in range(3):
        assert oracle.rel_l2(to_host(ck[c]), ref_ck[c]) <= tol, c


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_varcoef_adjoint_matches_oracle(dtype):
    shape, alpha, steps, every = (11, 14, 19), 0.1, 9, 4
    u0, k, y = _inputs(shape, dtype, seed=2)
    uT, gu, gk = _gpu_grads(u0, k, y, alpha, steps, dtype, every)
    ref_uT = oracle.varcoef_forward(u0, k, alpha, steps)
    ref_gu, ref_gk = oracle.varcoef_adjoint(u0, k, alpha, steps, 2.0 * (ref_uT - y) / u0.size)
    e_u, e_k = oracle.rel_l2(gu, ref_gu), oracle.rel_l2(gk, ref_gk)
    print(f"{dtype}: dL/du0 rel-L2 {e_u:.2e}, dL/dk rel-L2 {e_k:.2e}")
    if dtype == "f64":
        assert e_u <= 1e-12 and e_k <= 1e-12
    else:
        assert e_u <= TOL_F32_GU and e_k <= TOL_F32_GK


def test_checkpoint_interval_does_not_change_a_bit():
    shape, alpha, steps = (9, 12, 16), 0.1, 10
    u0, k, y = _inputs(shape, "f64", seed=4)
    base = _gpu_grads(u0, k, y, alpha, steps, "f64", 1)
    for every in (3, 4, 10, 25):
        other = _gpu_grads(u0, k, y, alpha, steps, "f64", every)
        for a, b in zip(base, other):
            assert np.array_equal(a, b), every


def test_stencil_fn_autograd_matches_oracle():
    import paper_2303_08365_amd as st
    import torch
    shape, alpha, steps, every = (8, 10, 12), 0.1, 6, 2
    u0, k, y = _inputs(shape, "f64", seed=6)
    tu = torch.from_numpy(u0).cuda().requires_grad_(True)
    tk = torch.from_numpy(k).cuda().requires_grad_(True)
    ty = torch.from_numpy(y).cuda()
    uT = st.StencilFn.apply(tu, tk, alpha, steps, every)
    loss = torch.mean((uT - ty) ** 2)
    loss.backward()
    ref_uT = oracle.varcoef_forward(u0, k, alpha, steps)
    ref_gu, ref_gk = oracle.varcoef_adjoint(u0, k, alpha, steps, 2.0 * (ref_uT - y) / u0.size)
    assert oracle.rel_l2(uT.detach().cpu().numpy(), ref_uT) <= 1e-12
    assert oracle.rel_l2(tu.grad.cpu().numpy(), ref_gu) <= 1e-12
    assert oracle.rel_l2(tk.grad.cpu().numpy(), ref_gk) <= 1e-12


def test_gradients_match_directional_finite_differences():
    # central differences of the loss computed by the GPU forward itself
    shape, alpha, steps, every = (10, 12, 14), 0.1, 8, 3
    u0, k, y = _inputs(shape, "f64", seed=8)
    uT, gu, gk = _gpu_grads(u0, k, y, alpha, steps, "f64", every)
    rng = np.random.default_rng(1)
    vu, vk = rng.standard_normal(shape), rng.standard_normal(shape)

    def loss(uu, kk):
        g, _, _, _ = _gpu_forward(uu, kk, alpha, steps, "f64")
        return float(np.mean((to_host(g) - y) ** 2))

    h = 1e-5
    fd_u = (loss(u0 + h * vu, k) - loss(u0 - h * vu, k)) / (2 * h)
    fd_k = (loss(u0, k + h * vk) - loss(u0, k - h * vk)) / (2 * h)
    assert abs(fd_u - float(np.sum(gu * vu))) <= 1e-7 * max(1.0, abs(fd_u))
    assert abs(fd_k - float(np.sum(gk * vk))) <= 1e-7 * max(1.0, abs(fd_k))


@pytest.mark.parametrize("bc", ["zero", "periodic"])
def test_constant_weight_adjoint_is_the_transpose(bc):
    import paper_2303_08365_amd as st
    import torch
    shape = (12, 30, 140)
    offs = [(0, 0, 0), (-1, 0, 0), (0, 2, 0), (0, 0, -1), (1, 1, 0), (0, -1, 3)]
    w = list(np.random.default_rng(3).random(6) / 6)
    v = synth.uniform_field(shape, seed=5)
    plan = st.Plan(offs, shape, "f64", bc)
    lam = to_device(v, "f64")
    plan.adjoint(lam, 4, torch.empty_like(lam), coeffs=w)
    ref = oracle.sweep_transpose(v, offs, w, 4, bc=bc)
    assert oracle.rel_l2(to_host(lam), ref) <= 1e-12
    # star stencil (mirrored pattern runs on the fused kernel)
    offs7 = synth.star_offsets(3, 1)
    w7 = list(np.random.default_rng(4).random(7) / 7)
    plan7 = st.Plan(offs7, shape, "f64", bc)
    lam = to_device(v, "f64")
    plan7.adjoint(lam, 5, torch.empty_like(lam), coeffs=w7)
    assert oracle.rel_l2(to_host(lam), oracle.sweep_transpose(v, offs7, w7, 5, bc=bc)) <= 1e-12


# Shapes the z-streaming kernels take (tiles of 128 columns x 16 / 8 rows fit
# inside the grid): ragged tiles in x and y, a single tile, wide rows.
STREAM_SHAPES = [(19, 37, 200), (9, 16, 128), (6, 50, 384)]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape", STREAM_SHAPES)
def test_varcoef_streaming_matches_naive_and_oracle(dtype, shape):
    alpha, steps, every = 0.1, 7, 3
    u0, k, y = _inputs(shape, dtype, seed=3)
    print(f"varcoef streaming {dtype} {shape}", flush=True)
    # forward: the streaming step reproduces the one-thread-per-cell step bit
    # for bit (same face order; the ghost layer comes from the loads)
    gs, _, cks, _ = _gpu_forward(u0, k, alpha, steps, dtype, every)
    gn, _, ckn, _ = _gpu_forward(u0, k, alpha, steps, dtype, every, naive=True)
    assert np.array_equal(to_host(gs), to_host(gn))
    for a, b in zip(cks, ckn):
        assert np.array_equal(to_host(a), to_host(b))
    ref = oracle.varcoef_forward(u0, k, alpha, steps)
    tol = 1e-12 if dtype == "f64" else 1e-5
    assert oracle.rel_l2(to_host(gs), ref) <= tol
    # adjoint: dL/du0 bit for bit; dL/dk sums its edge terms in another order
    uT, gu, gk = _gpu_grads(u0, k, y, alpha, steps, dtype, every)
    _, gun, gkn = _gpu_grads(u0, k, y, alpha, steps, dtype, every, naive=True)
    assert np.array_equal(gu, gun)
    assert oracle.rel_l2(gk, gkn) <= (1e-13 if dtype == "f64" else 1e-5)
    ref_gu, ref_gk = oracle.varcoef_adjoint(u0, k, alpha, steps, 2.0 * (ref - y) / u0.size)
    e_u, e_k = oracle.rel_l2(gu, ref_gu), oracle.rel_l2(gk, ref_gk)
    print(f"  dL/du0 {e_u:.2e}  dL/dk {e_k:.2e}", flush=True)
    if dtype == "f64":
        assert e_u <= 1e-12 and e_k <= 1e-12
    else:
        assert e_u <= TOL_F32_GU and e_k <= TOL_F32_GK


def test_varcoef_streaming_checkpoint_interval_does_not_change_a_bit():
    shape, alpha, steps = (11, 20, 128), 0.1, 10
    u0, k, y = _inputs(shape, "f64", seed=5)
    base = _gpu_grads(u0, k, y, alpha, steps, "f64", 1)
    for every in (3, 10, 25):
        other = _gpu_grads(u0, k, y, alpha, steps, "f64", every)
        for a, b in zip(base, other):
            assert np.array_equal(a, b), every
