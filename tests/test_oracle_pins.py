"""Pins for the CPU oracle against facts the paper and mathematics fix.

Each test checks the oracle against something other than itself: values
evaluated by hand (tests/golden), spectral closed forms (DST-I / FFT),
closed-form mode decay, combinatorial impulse responses, conservation and
the maximum principle, exact identities, and finite differences.  A dropped
term, a wrong sign, a transposed offset or a wrong boundary rule in the
oracle fails at least one of them.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.fft

import oracle
import synth

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


# --------------------------------------------------------------------------
# hand-evaluated 4x4 grids (Alg. 1 / Eq. 3)
# --------------------------------------------------------------------------
def _golden_4x4(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "heat2d_4x4.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            bc, steps, i, j, num, den = line.split()
            rows.append((bc, int(steps), int(i), int(j), Fraction(int(num), int(den))))
    return rows


def test_golden_4x4_heat_increment_form(golden_dir):
    u0 = np.arange(1, 17, dtype=np.float64).reshape(4, 4)
    rows = _golden_4x4(golden_dir)
    assert len(rows) >= 20
    for bc, steps, i, j, val in rows:
        out = oracle.heat(u0, 0.2, steps, bc=bc)
        # alpha = 0.2 is inexact in binary: allow a few ulps per step
        assert abs(out[i, j] - float(val)) <= 8 * steps * np.spacing(float(val)), (bc, steps, i, j)


def test_golden_4x4_weighted_form(golden_dir):
    # Alg. 1 weighted form with c1 = 1 - 4a, c2..c5 = a, same expected values
    u0 = np.arange(1, 17, dtype=np.float64).reshape(4, 4)
    offs = [(0, 0), (-1, 0), (0, 1), (0, -1), (1, 0)]   # c1..c5 placement of Alg. 1
    w = [1 - 4 * 0.2, 0.2, 0.2, 0.2, 0.2]
    for bc, steps, i, j, val in _golden_4x4(golden_dir):
        out = oracle.sweep(u0, offs, w, steps, bc=bc)
        assert abs(out[i, j] - float(val)) <= 8 * steps * np.spacing(float(val)), (bc, steps, i, j)


def test_alg1_coefficient_placement_is_oriented():
    # c3 multiplies A[i][j+1] (Alg. 1): with only c3 = 1 the field moves one
    # column towards lower j per step.
    u0 = np.zeros((3, 5))
    u0[1, 3] = 1.0
    out = oracle.sweep(u0, [(0, 0), (0, 1)], [0.0, 1.0], 1, bc="zero")
    assert out[1, 2] == 1.0 and out.sum() == 1.0
    out = oracle.sweep(u0, [(0, 0), (-1, 0)], [0.0, 1.0], 1, bc="zero")  # c2: A[i-1][j]
    assert out[2, 3] == 1.0 and out.sum() == 1.0


# --------------------------------------------------------------------------
# spectral closed forms
# --------------------------------------------------------------------------
def _dst_heat(u0, alpha, steps):
    g = np.zeros(u0.shape)
    for axis, n in enumerate(u0.shape):
        k = np.arange(1, n + 1)
        s = np.sin(np.pi * k / (2.0 * (n + 1))) ** 2
        view = [1] * u0.ndim
        view[axis] = n
        g = g + s.reshape(view)
    g = 1.0 - 4.0 * alpha * g
    c = scipy.fft.dstn(u0, type=1, norm="ortho")
    return scipy.fft.idstn(c * g ** steps, type=1, norm="ortho")


@pytest.mark.parametrize("shape,alpha,steps", [((6, 7), 0.2, 5), ((23,), 0.4, 9),
                                                ((5, 6, 7), 0.15, 6), ((17, 9), 0.11, 30)])
def test_zero_bc_heat_matches_dst_spectral(shape, alpha, steps):
    u0 = synth.uniform_field(shape, seed=3)
    ref = _dst_heat(u0, alpha, steps)
    assert oracle.rel_l2(oracle.heat(u0, alpha, steps, bc="zero"), ref) < 1e-13
    offs = synth.star_offsets(len(shape), 1)
    w = synth.heat_weights(len(shape), alpha)
    assert oracle.rel_l2(oracle.sweep(u0, offs, w, steps, bc="zero"), ref) < 1e-13


def _fft_periodic(u0, offsets, weights, steps):
    sym = np.zeros(u0.shape, dtype=np.complex128)
    grids = np.meshgrid(*[np.arange(n) for n in u0.shape], indexing="ij")
    for o, w in zip(offsets, weights):
        phase = sum(2j * np.pi * k * od / n for k, od, n in zip(grids, o, u0.shape))
        sym = sym + w * np.exp(phase)
    return np.real(np.fft.ifftn(np.fft.fftn(u0) * sym ** steps))


@pytest.mark.parametrize("case", ["box2d9", "star3d25", "asym2d", "star2d9", "box3d27"])
def test_periodic_matches_fft_spectral(case):
    rng = np.random.default_rng(11)
    if case == "box2d9":
        shape, offs, w, steps = (16, 21), synth.box_offsets(2, 1), synth.box_mean_weights(2, 1), 7
    elif case == "star3d25":
        shape, offs, w, steps = (10, 11, 12), synth.star_offsets(3, 4), synth.star25_weights(0), 3
    elif case == "asym2d":
        shape, offs = (9, 13), [(0, 0), (-1, 0), (0, 2), (1, -1), (0, -3)]
        w, steps = list(rng.random(5) / 5), 6
    elif case == "star2d9":
        shape, offs, w, steps = (12, 14), synth.star_offsets(2, 2), list(rng.random(9) / 9), 4
    else:
        shape, offs, steps = (6, 7, 8), synth.box_offsets(3, 1), 3
        w = synth.box_mean_weights(3, 1)
    u0 = synth.uniform_field(shape, seed=5)
    ref = _fft_periodic(u0, offs, w, steps)
    assert oracle.rel_l2(oracle.sweep(u0, offs, w, steps, bc="periodic"), ref) < 1e-13


# --------------------------------------------------------------------------
# closed-form single-mode decay, impulse responses
# --------------------------------------------------------------------------
@pytest.mark.parametrize("shape,alpha,steps", [((24, 20, 18), 0.15, 10), ((40, 33), 0.2, 25)])
def test_sin_mode_decays_by_closed_form_factor(shape, alpha, steps):
    mode = synth.sin_mode(shape)
    g = 1.0 - 4.0 * alpha * sum(math.sin(math.pi / (2.0 * (n + 1))) ** 2 for n in shape)
    out = oracle.heat(mode, alpha, steps, bc="zero")
    assert oracle.rel_l2(out, g ** steps * mode) < 1e-13
    # linearity: noise + mode minus noise alone isolates the mode's decay
    noise = synth.uniform_field(shape, seed=0)
    diff = oracle.heat(noise + mode, alpha, steps) - oracle.heat(noise, alpha, steps)
    assert np.max(np.abs(diff - g ** steps * mode)) < 1e-12


def test_closed_form_constant_from_reading_of_boundary():
    # The zero-ghost reading gives g^100 = 0.998313783162922 at N = 512,
    # alpha = 0.15 (3D); a fixed outer ring would give a different constant.
    g = 1.0 - 4.0 * 0.15 * 3 * math.sin(math.pi / (2.0 * 513)) ** 2
    assert abs(g ** 100 - 0.998313783162922) < 1e-15


def test_impulse_response_is_trinomial_and_exact():
    # Dyadic weights keep every partial sum exact in FP64, so the result must be
    # bit-exact: value at displacement m after T steps is the sum over
    # (n-, n0, n+) with n- - n+ = m of T!/(n-! n0! n+!) a^n- b^n0 c^n+,
    # where offset -1 (weight a) moves mass towards +x.
    a, b, c, T, n = 0.5, 0.25, 0.125, 10, 64
    u0 = np.zeros(n)
    u0[0] = 1.0
    out = oracle.sweep(u0, [(0,), (-1,), (1,)], [b, a, c], T, bc="periodic")
    for m in range(-T, T + 1):
        tot = Fraction(0)
        for nm in range(T + 1):
            npl = nm - m
            n0 = T - nm - npl
            if npl < 0 or n0 < 0:
                continue
            coef = math.factorial(T) // (math.factorial(nm) * math.factorial(n0) * math.factorial(npl))
            tot += coef * Fraction(a) ** nm * Fraction(b) ** n0 * Fraction(c) ** npl
        assert out[m % n] == float(tot), m
    assert np.count_nonzero(out) == 2 * T + 1


def test_impulse_response_2d_box_is_separable():
    # Box 1/9 = (1/3 row) x (1/3 column): T steps give the outer product of two
    # 1D trinomial rows, each divided by 3^T.
    T, n = 6, 32
    u0 = np.zeros((n, n))
    u0[0, 0] = 1.0
    out = oracle.sweep(u0, synth.box_offsets(2, 1), np.full(9, 1.0 / 9.0), T, bc="periodic")
    row = np.zeros(n)
    for m in range(-T, T + 1):
        tot = 0
        for nm in range(T + 1):
            npl = nm - m
            n0 = T - nm - npl
            if npl >= 0 and n0 >= 0:
                tot += math.factorial(T) // (math.factorial(nm) * math.factorial(n0) * math.factorial(npl))
        row[m % n] = tot / 3.0 ** T
    assert np.max(np.abs(out - np.outer(row, row))) < 1e-15


def test_impulse_response_3d_box_and_1d_star_closed_forms():
    # 3D box 1/27 = (1/3)^3 per axis: the impulse spreads as the product of
    # three trinomial rows; a 1D 5-point star with weights 1/5 spreads as the
    # pentanomial coefficients (coefficients of (1 + x + ... + x^4)^T) / 5^T
    T, n = 4, 16

    def trinomial_row():
        row = np.zeros(n)
        for m in range(-T, T + 1):
            tot = 0
            for nm in range(T + 1):
                npl = nm - m
                n0 = T - nm - npl
                if npl >= 0 and n0 >= 0:
                    tot += math.factorial(T) // (math.factorial(nm) * math.factorial(n0) * math.factorial(npl))
            row[m % n] = tot / 3.0 ** T
        return row

    u0 = np.zeros((n, n, n))
    u0[0, 0, 0] = 1.0
    out = oracle.sweep(u0, synth.box_offsets(3, 1), np.full(27, 1.0 / 27.0), T, bc="periodic")
    r = trinomial_row()
    assert np.max(np.abs(out - np.einsum("i,j,k->ijk", r, r, r))) < 1e-15
    poly = np.array([1.0])
    for _ in range(T):
        poly = np.convolve(poly, np.ones(5))
    u1 = np.zeros(64)
    u1[20] = 1.0
    out1 = oracle.sweep(u1, synth.star_offsets(1, 2), np.full(5, 0.2), T, bc="zero")
    ref1 = np.zeros(64)
    ref1[20 - 2 * T:20 + 2 * T + 1] = poly / 5.0 ** T
    assert np.max(np.abs(out1 - ref1)) < 1e-15


# --------------------------------------------------------------------------
# conservation, maximum principle, identities
# --------------------------------------------------------------------------
def test_mean_conserved_under_periodic_unit_sum():
    u0 = synth.uniform_field((12, 13, 14), seed=2)
    w = synth.star25_weights(0)
    assert abs(w.sum() - 1.0) < 1e-15
    out = oracle.sweep(u0, synth.star_offsets(3, 4), w, 20, bc="periodic")
    assert abs(out.mean() - u0.mean()) < 20 * 4e-16 * u0.mean() * 10
    w32 = synth.box_mean_weights(2, 1, "f32")
    assert np.sum(w32) == 1.0          # centre-adjusted FP32 weights sum exactly to 1
    u2 = synth.round_to(synth.uniform_field((40, 41), 1), "f32")
    out2 = oracle.sweep(u2, synth.box_offsets(2, 1), w32, 50, bc="periodic")
    assert abs(out2.mean() - u2.mean()) < 1e-13


def test_max_principle_zero_and_periodic():
    u0 = synth.uniform_field((30, 31), seed=4) - 0.3
    out = oracle.heat(u0, 0.25, 40, bc="zero")
    assert out.max() <= max(0.0, u0.max()) + 1e-14 and out.min() >= min(0.0, u0.min()) - 1e-14
    out = oracle.heat(u0, 0.25, 40, bc="periodic")
    assert out.max() <= u0.max() + 1e-14 and out.min() >= u0.min() - 1e-14
    # an unstable coefficient must break it (the pin has teeth)
    out = oracle.heat(u0, 0.4, 40, bc="periodic")
    assert out.max() > u0.max()


def test_identities_and_composability():
    u0 = synth.uniform_field((9, 10, 11), seed=8)
    offs = synth.star_offsets(3, 1)
    assert np.array_equal(oracle.heat(u0, 0.0, 7), u0)
    assert np.array_equal(oracle.sweep(u0, offs, synth.heat_weights(3, 0.1), 0), u0)
    w = synth.heat_weights(3, 0.13)
    a = oracle.sweep(oracle.sweep(u0, offs, w, 3), offs, w, 4)
    assert np.array_equal(a, oracle.sweep(u0, offs, w, 7))
    # OpenMP threading does not change a single bit
    assert np.array_equal(oracle.sweep(u0, offs, w, 5, threads=1),
                          oracle.sweep(u0, offs, w, 5, threads=4))


def test_heat_increment_form_equals_weighted_form():
    u0 = synth.uniform_field((20, 21, 22), seed=9)
    a = oracle.heat(u0, 0.15, 12, bc="zero")
    b = oracle.sweep(u0, synth.star_offsets(3, 1), synth.heat_weights(3, 0.15), 12, bc="zero")
    assert oracle.rel_l2(a, b) < 1e-14


# --------------------------------------------------------------------------
# transpose / adjoint of the constant-weight sweep
# --------------------------------------------------------------------------
@pytest.mark.parametrize("bc", ["zero", "periodic"])
def test_transpose_dot_product_and_mirror(bc):
    rng = np.random.default_rng(21)
    shape = (7, 8, 9)
    offs = [(0, 0, 0), (-1, 0, 0), (0, 2, 0), (0, 0, -1), (1, 1, 0), (0, -1, 3)]
    w = rng.random(6)
    x = rng.random(shape)
    y = rng.random(shape)
    Sx = oracle.sweep(x, offs, w, 3, bc=bc)
    STy = oracle.sweep_transpose(y, offs, w, 3, bc=bc)
    lhs, rhs = float(np.sum(Sx * y)), float(np.sum(x * STy))
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)
    mirrored = [tuple(-o for o in off) for off in offs]
    assert oracle.rel_l2(oracle.sweep(y, mirrored, w, 3, bc=bc), STy) < 1e-14


# --------------------------------------------------------------------------
# cone-sampled oracle equals the full sweep bit for bit
# --------------------------------------------------------------------------
@pytest.mark.parametrize("bc", ["zero", "periodic"])
@pytest.mark.parametrize("ndim,radius,steps", [(2, 1, 6), (3, 1, 4), (3, 2, 2), (1, 3, 5)])
def test_sweep_point_equals_full_sweep(bc, ndim, radius, steps):
    shape = {1: (37,), 2: (13, 17), 3: (9, 10, 11)}[ndim]
    offs = synth.star_offsets(ndim, radius)
    w = np.random.default_rng(1).random(len(offs)) / len(offs)
    u0 = synth.uniform_field(shape, seed=6)
    full = oracle.sweep(u0, offs, w, steps, bc=bc)
    rng = np.random.default_rng(2)
    pts = [tuple(0 for _ in shape), tuple(n - 1 for n in shape)]
    pts += [tuple(int(rng.integers(0, n)) for n in shape) for _ in range(6)]
    for p in pts:
        assert oracle.sweep_point(u0, offs, w, steps, p, bc=bc) == full[p], p


# --------------------------------------------------------------------------
# variable-coefficient heat and its adjoint
# --------------------------------------------------------------------------
def test_varcoef_unit_k_reduces_to_heat():
    u0 = synth.uniform_field((8, 9, 10), seed=1)
    out = oracle.varcoef_forward(u0, np.ones_like(u0), 0.12, 9)
    assert oracle.rel_l2(out, oracle.heat(u0, 0.12, 9, bc="zero")) < 1e-14


def test_varcoef_checkpoints_are_the_states():
    u0, k, _ = synth.varcoef_inputs((6, 7, 8), seed=0)
    uT, ck = oracle.varcoef_forward(u0, k, 0.1, 10, every=4)
    assert ck.shape[0] == 3
    assert np.array_equal(ck[0], u0)
    assert np.array_equal(ck[1], oracle.varcoef_forward(u0, k, 0.1, 4))
    assert np.array_equal(ck[2], oracle.varcoef_forward(u0, k, 0.1, 8))
    assert np.array_equal(uT, oracle.varcoef_forward(ck[2], k, 0.1, 2))


def test_varcoef_adjoint_matches_finite_differences():
    shape, alpha, steps = (4, 5, 4), 0.1, 4
    u0, k, y = synth.varcoef_inputs(shape, seed=0)
    M = u0.size

    def loss(u0_, k_):
        uT = oracle.varcoef_forward(u0_, k_, alpha, steps)
        return float(np.sum((uT - y) ** 2) / M)

    uT = oracle.varcoef_forward(u0, k, alpha, steps)
    gu, gk = oracle.varcoef_adjoint(u0, k, alpha, steps, 2.0 * (uT - y) / M)
    h = 1e-6
    fd_u = np.zeros(shape)
    fd_k = np.zeros(shape)
    for idx in np.ndindex(*shape):
        e = np.zeros(shape)
        e[idx] = h
        fd_u[idx] = (loss(u0 + e, k) - loss(u0 - e, k)) / (2 * h)
        fd_k[idx] = (loss(u0, k + e) - loss(u0, k - e)) / (2 * h)
    assert oracle.rel_l2(gu, fd_u) < 1e-7
    assert oracle.rel_l2(gk, fd_k) < 1e-7


def _golden_varcoef(golden_dir):
    vals = {}
    with open(os.path.join(golden_dir, "varcoef_1x2x3.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            q, y, x, num, den = line.split()
            vals.setdefault(q, np.zeros((1, 2, 3)))[0, int(y), int(x)] = float(Fraction(int(num), int(den)))
    return vals


_VC_K = np.array([[[1.0, 2.0, 3.0], [4.0, 5.0, 6.0]]])
_VC_U0 = np.array([[[3.0, 1.0, 2.0], [0.0, 2.0, 4.0]]])


def test_varcoef_golden_steps_pin_the_face_average(golden_dir):
    # hand-evaluated non-uniform k: a face mean other than the arithmetic one
    # (geometric, harmonic) or a dropped edge face changes these values
    g = _golden_varcoef(golden_dir)
    for steps, q in ((1, "u1"), (2, "u2")):
        got = oracle.varcoef_forward(_VC_U0, _VC_K, 0.1, steps)
        assert np.allclose(got, g[q], rtol=4e-15, atol=4e-15), (steps, got, g[q])


def test_varcoef_golden_gradient_pins_the_half_split(golden_dir):
    # one step, L = u1(0,1): dL/dk gives each interior face's derivative half
    # to either cell; dL/du0 carries the face means themselves
    g = _golden_varcoef(golden_dir)
    lam = np.zeros((1, 2, 3))
    lam[0, 0, 1] = 1.0
    gu, gk = oracle.varcoef_adjoint(_VC_U0, _VC_K, 0.1, 1, lam)
    assert np.allclose(gk, g["gk"], rtol=4e-15, atol=4e-16), gk
    assert np.allclose(gu, g["gu"], rtol=4e-15, atol=4e-16), gu


def test_varcoef_operator_is_symmetric():
    # one step is u -> A u with A symmetric: the scatter adjoint of one step
    # applied to v equals the forward step applied to v (no gk).
    u0, k, _ = synth.varcoef_inputs((5, 6, 7), seed=3)
    v = synth.uniform_field((5, 6, 7), seed=4)
    lam0, _ = oracle.varcoef_adjoint(u0, k, 0.1, 1, v)
    assert oracle.rel_l2(lam0, oracle.varcoef_forward(v, k, 0.1, 1)) < 1e-14


# --------------------------------------------------------------------------
# Eq. 5 metric against Tab. 3
# --------------------------------------------------------------------------
def test_metric_reproduces_tab3_naive_row(golden_dir):
    with open(os.path.join(golden_dir, "tab3_case_study.txt")) as f:
        line = [l for l in f if l.strip() and not l.startswith("#")][0]
    nx, ny, steps, secs, printed = line.split()
    g = oracle.stencils_per_second((int(nx), int(ny)), int(steps), float(secs)) / 1e9
    assert round(g, 1) == float(printed)
    assert abs(g - 2.81) < 0.005


# ---------------------------------------------------------------------------
# outflow across the zero-rule boundary
# ---------------------------------------------------------------------------
def test_outflow_1d_three_point_by_hand():
    # offset -1 (weight a) reads the left neighbour, so every cell passes a*u to
    # its right neighbour: the last cell loses a*u[n-1] through the right face;
    # offset +1 (weight b) passes b*u to the left: the first cell loses b*u[0]
    a, b = 0.125, 0.375
    u = np.array([3.0, 5.0, 7.0, 11.0])
    _, out = oracle.sweep_flux(u, [(0,), (-1,), (1,)], [0.5, a, b], 1)
    assert out == a * 11.0 + b * 3.0
    # swapping the weights swaps the faces
    _, out2 = oracle.sweep_flux(u, [(0,), (-1,), (1,)], [0.5, b, a], 1)
    assert out2 == b * 11.0 + a * 3.0


def test_outflow_equals_lost_total_for_unit_sum_weights():
    # sum_x u_{t+1} = (sum_p w_p) sum_x u_t - outflow_t: with weights summing to 1
    # the total drops by exactly the outflow (rounding aside)
    rng = np.random.default_rng(11)
    for ndim, pat in ((2, synth.box_offsets(2, 1)), (3, synth.star_offsets(3, 1)), (3, synth.star_offsets(3, 2)), (2, synth.star_offsets(2, 2))):
        w = rng.uniform(0.05, 1.0, len(pat))
        w /= w.sum()
        shape = (9, 7, 6)[:ndim] if ndim == 3 else (13, 10)
        u0 = rng.uniform(0.0, 1.0, shape)
        uT, out = oracle.sweep_flux(u0, pat, w, 7)
        assert out > 0
        assert math.isclose(u0.sum() - uT.sum(), out, rel_tol=1e-12)


def test_outflow_matches_unbounded_step_on_a_padded_grid():
    # independent definition: run one step on a grid padded by a ghost frame,
    # reading zeros outside the original grid; the heat landing on the frame is
    # what left
    rng = np.random.default_rng(12)
    pat = synth.box_offsets(3, 1)
    w = rng.uniform(-0.2, 0.6, len(pat))
    u = rng.uniform(-1.0, 1.0, (5, 6, 4))
    total = 0.0
    state = u.copy()
    for _ in range(3):
        pad = np.pad(state, 1)
        nxt = np.zeros_like(pad)
        big = np.pad(pad, 1)  # reads beyond the frame are zero too
        for off, wp in zip(pat, w):
            sl = tuple(slice(1 + o, 1 + o + n) for o, n in zip(off, pad.shape))
            nxt += wp * big[sl]
        frame = nxt.copy()
        frame[1:-1, 1:-1, 1:-1] = 0.0
        total += frame.sum()
        state = nxt[1:-1, 1:-1, 1:-1]
    uT, out = oracle.sweep_flux(u, pat, w, 3)
    np.testing.assert_allclose(uT, state, rtol=0, atol=1e-13)
    assert math.isclose(out, total, rel_tol=1e-12, abs_tol=1e-13)


def test_outflow_zero_for_identity_and_zero_steps():
    u = np.random.default_rng(13).uniform(0, 1, (4, 5))
    _, out = oracle.sweep_flux(u, [(0, 0)], [1.0], 5)
    assert out == 0.0
    _, out = oracle.sweep_flux(u, synth.star_offsets(2, 1), [0.6, 0.1, 0.1, 0.1, 0.1], 0)
    assert out == 0.0


@pytest.mark.parametrize("shape,alpha,steps", [((9, 11), 0.23, 40), ((31,), 0.4, 17), ((6, 5, 7), 0.15, 9)])
def test_heat_spectral_matches_loop_oracle(shape, alpha, steps):
    # two computations of the same exact result: the DST-I closed form and the
    # plain loop
    u0 = synth.uniform_field(shape, seed=31)
    assert oracle.rel_l2(oracle.heat_spectral(u0, alpha, steps), oracle.heat(u0, alpha, steps, bc="zero")) < 1e-13


def test_heat_spectral_sin_mode_and_gaussian_symmetry():
    n, alpha, steps = 40, 0.23, 300
    x = (np.arange(n) + 1.0) / (n + 1.0)
    mode = np.outer(np.sin(np.pi * x), np.sin(np.pi * x))
    g = 1.0 - 4.0 * alpha * 2.0 * math.sin(math.pi / (2.0 * (n + 1))) ** 2
    np.testing.assert_allclose(oracle.heat_spectral(mode, alpha, steps), g ** steps * mode, rtol=1e-12, atol=1e-15)
    # a centred Gaussian stays symmetric and its four centre cells stay equal
    u = oracle.heat_spectral(synth.gaussian_plate(n, 6.0), alpha, steps)
    np.testing.assert_allclose(u, u[::-1, :], rtol=0, atol=1e-12)
    np.testing.assert_allclose(u, u.T, rtol=0, atol=1e-12)
    c = n // 2 - 1
    assert abs(u[c, c] - u[c + 1, c + 1]) < 1e-12 and u[c, c] == np.max(u)
