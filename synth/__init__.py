"""Seeded synthetic inputs for the stencil sweep.

This module is shared by the CPU oracle tests, the GPU parity tests and the
benchmark.  It produces *inputs only* -- initial fields, stencil point lists,
weight tables, grid-size draws and conductivity fields -- and holds none of
the sweep's arithmetic, so that neither side of a parity check can lean on
the other.

Conventions (fixed here once, used everywhere):

* Arrays are dense C-order with shape ``(nz, ny, nx)`` (or ``(ny, nx)`` in
  2D); the last axis is unit-stride, matching the ``A[i][j]`` indexing of the
  paper's Heat-2D listing (Sec. 2.1, Alg. 1), where ``j`` is innermost.
* Stencil offsets are integer tuples in the same axis order (slowest first).
  The centre point ``(0, .., 0)`` is always listed first.
* Random fields use ``numpy.random.default_rng(seed)`` (PCG64) in FP64.  A
  lower-precision run rounds that FP64 field to its storage type (round to
  nearest even), and the oracle consumes the *rounded* values widened back to
  FP64, so that parity measures arithmetic error only.
"""
from __future__ import annotations

import math
from typing import List, Sequence, Tuple

import numpy as np

__all__ = [
    "uniform_field", "sin_mode", "round_to", "bf16_round", "bf16_bits", "bf16_from_bits",
    "star_offsets", "box_offsets", "heat_weights", "box_mean_weights",
    "star25_weights", "adjust_centre", "batch_shapes", "batch_alphas",
    "varcoef_inputs", "DTYPES",
]

DTYPES = ("f64", "f32", "bf16")


# ----------------------------------------------------------------------------
# fields
# ----------------------------------------------------------------------------
def uniform_field(shape: Sequence[int], seed: int = 0) -> np.ndarray:
    """U[0,1) field in FP64 from PCG64 ``default_rng(seed)``."""
    return np.random.default_rng(seed).random(tuple(int(s) for s in shape))


def sin_mode(shape: Sequence[int]) -> np.ndarray:
    """Product of sin(pi * x_d) over the axes, with x_i = (i+1)/(N_d+1).

    The mode vanishes on the zero ghost layer just outside the grid, so under a
    zero-Dirichlet ghost boundary it is a single eigenvector of every constant
    star stencil (used by the closed-form decay pin).
    """
    out = np.ones(tuple(int(s) for s in shape), dtype=np.float64)
    for axis, n in enumerate(out.shape):
        x = (np.arange(n, dtype=np.float64) + 1.0) / (n + 1.0)
        s = np.sin(np.pi * x)
        view = [1] * out.ndim
        view[axis] = n
        out = out * s.reshape(view)
    return out


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (round to nearest, ties to even) via FP32; return FP32.

    The FP64 input is first rounded to FP32 (RNE), then to the 8-bit-mantissa
    bfloat16 grid (RNE); NaN is preserved.
    """
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    r = r.astype(np.uint32)
    nan = np.isnan(f)
    r[nan] = (f.view(np.uint32)[nan] | 0x00400000) & 0xFFFF0000
    return r.view(np.float32).reshape(f.shape)


def bf16_bits(a_bf16_as_f32: np.ndarray) -> np.ndarray:
    """Storage bits (uint16) of values that are already bfloat16-representable."""
    f = np.ascontiguousarray(a_bf16_as_f32, dtype=np.float32)
    return (f.view(np.uint32) >> 16).astype(np.uint16)


def bf16_from_bits(bits: np.ndarray) -> np.ndarray:
    """Widen uint16 bfloat16 storage to FP32 exactly."""
    b = np.ascontiguousarray(bits, dtype=np.uint16).astype(np.uint32) << 16
    return b.view(np.float32)


def round_to(a: np.ndarray, dtype: str) -> np.ndarray:
    """Round an FP64 array to the storage dtype and widen it back to FP64."""
    if dtype == "f64":
        return np.array(a, dtype=np.float64)
    if dtype == "f32":
        return np.asarray(a, dtype=np.float32).astype(np.float64)
    if dtype == "bf16":
        return bf16_round(a).astype(np.float64)
    raise ValueError(f"unknown dtype {dtype!r}")


# ----------------------------------------------------------------------------
# stencil point lists
# ----------------------------------------------------------------------------
def gaussian_plate(n: int, sigma: float, amplitude: float = 100.0) -> np.ndarray:
    """n x n field amplitude * exp(-r^2 / (2 sigma^2)), r measured from the
    grid's centre point ((n-1)/2, (n-1)/2) in cells (the case study's initial
    temperature: hottest at the centre, cooler towards the edges)."""
    c = (n - 1) / 2.0
    g = np.exp(-((np.arange(n) - c) ** 2) / (2.0 * sigma * sigma))
    return amplitude * np.outer(g, g)


def star_offsets(ndim: int, radius: int) -> List[Tuple[int, ...]]:
    """Centre plus 2*ndim*radius axis points.

    Order: centre; then axis (slowest first), distance 1..radius, sign -,+.
    Heat-2D (5P) is star(2,1), Heat-3D (7P) star(3,1), the order-4 3D star
    (25P) star(3,4); Tab. 1's Star-1D5P is star(1,2) and Star-2D9P star(2,2).
    """
    pts: List[Tuple[int, ...]] = [tuple([0] * ndim)]
    for axis in range(ndim):
        for dist in range(1, radius + 1):
            for sign in (-1, 1):
                o = [0] * ndim
                o[axis] = sign * dist
                pts.append(tuple(o))
    return pts


def box_offsets(ndim: int, radius: int) -> List[Tuple[int, ...]]:
    """All (2r+1)^ndim points, centre first, the rest in lexicographic order."""
    rng = range(-radius, radius + 1)
    grid = [()]
    for _ in range(ndim):
        grid = [g + (d,) for g in grid for d in rng]
    centre = tuple([0] * ndim)
    return [centre] + [g for g in grid if g != centre]


# ----------------------------------------------------------------------------
# weight tables
# ----------------------------------------------------------------------------
def heat_weights(ndim: int, alpha: float, dtype: str = "f64") -> np.ndarray:
    """Weights of the explicit heat step in point order of ``star_offsets(ndim,1)``.

    The heat step u + a*(sum of 2*ndim neighbours - 2*ndim*u) equals the
    weighted form (1 - 2*ndim*a)*u + a*sum (Eq. 3 with mu = a).  For a
    lower-precision dtype the off-centre weight ``a`` is rounded once and the
    centre is set to ``1 - 2*ndim*round(a)`` (computed in FP64, then rounded),
    so that the stored weights are the ones both sides use.
    """
    a = float(round_to(np.array([alpha]), dtype)[0])
    w = np.full(1 + 2 * ndim, a, dtype=np.float64)
    w[0] = float(round_to(np.array([1.0 - 2 * ndim * a]), dtype)[0])
    return w


def adjust_centre(weights: Sequence[float], dtype: str) -> np.ndarray:
    """Round each off-centre weight to ``dtype``; centre = 1 - sum(others).

    The centre is formed in FP64 from the rounded off-centre weights and then
    rounded itself; for the tables used here (1/9 box, the 25-point star) the
    result is exactly representable, so the rounded weights still sum to 1 and
    the periodic mean is not biased by coefficient rounding.
    """
    w = round_to(np.asarray(weights, dtype=np.float64), dtype)
    w[0] = float(round_to(np.array([1.0 - float(np.sum(w[1:]))]), dtype)[0])
    return w


def box_mean_weights(ndim: int, radius: int, dtype: str = "f64") -> np.ndarray:
    """Equal weights 1/(2r+1)^ndim for ``box_offsets``, centre-adjusted."""
    n = (2 * radius + 1) ** ndim
    return adjust_centre(np.full(n, 1.0 / n), dtype)


def star25_weights(seed: int = 0, dtype: str = "f64") -> np.ndarray:
    """Weights for the order-4 3D star in ``star_offsets(3, 4)`` order.

    Centre-dominant and normalised: 24 off-centre weights from
    ``default_rng(seed).random(24)`` scaled to sum 0.5, centre 0.5.  All are
    positive and sum to 1.
    """
    r = np.random.default_rng(seed).random(24)
    w = np.empty(25, dtype=np.float64)
    w[1:] = r * (0.5 / r.sum())
    w[0] = 0.5
    return adjust_centre(w, dtype)


# ----------------------------------------------------------------------------
# batch ensemble
# ----------------------------------------------------------------------------
def batch_shapes(n: int, seed: int = 0, lo: int = 256, hi: int = 4096) -> List[Tuple[int, int]]:
    """n (ny, nx) pairs, each side round(exp(U(ln lo, ln hi))), drawn independently."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(math.log(lo), math.log(hi), size=(n, 2))
    sides = np.rint(np.exp(u)).astype(np.int64)
    return [(int(a), int(b)) for a, b in sides]


def batch_alphas(n: int, seed: int = 0, lo: float = 0.05, hi: float = 0.24) -> np.ndarray:
    """Per-grid diffusion numbers, U[lo, hi) from a stream separate from the sizes."""
    return np.random.default_rng(seed + 7919).uniform(lo, hi, size=n)


# ----------------------------------------------------------------------------
# variable-coefficient (differentiable) workload
# ----------------------------------------------------------------------------
def _box3_replicate(a: np.ndarray) -> np.ndarray:
    """One pass of the 3x3x3 mean filter with edge replication (FP64)."""
    p = np.pad(a, 1, mode="edge")
    out = np.zeros_like(a)
    nz, ny, nx = a.shape
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                out += p[dz:dz + nz, dy:dy + ny, dx:dx + nx]
    return out / 27.0


def varcoef_inputs(shape: Sequence[int], seed: int = 0, passes: int = 3):
    """(u0, k, y): initial field, smoothed conductivity in [0.5, 1.5], target.

    u0 and k come from one ``default_rng(seed)`` stream (u0 first); k starts
    U[0.5, 1.5) and receives ``passes`` 3x3x3 box-mean passes with edge
    replication, so it stays inside [0.5, 1.5].  The target y comes from
    ``default_rng(seed + 1)``.  All FP64.
    """
    shape = tuple(int(s) for s in shape)
    rng = np.random.default_rng(seed)
    u0 = rng.random(shape)
    k = 0.5 + rng.random(shape)
    for _ in range(passes):
        k = _box3_replicate(k)
    y = np.random.default_rng(seed + 1).random(shape)
    return u0, k, y
