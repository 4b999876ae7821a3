"""CPU oracle for the stencil sweep -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package.  It wraps ``stencil_oracle.c`` (plain C, FP64, no FMA
contraction) through ctypes and shares no code with the GPU library.

Functions take and return numpy FP64 arrays in C order, shape (nz, ny, nx)
(or fewer axes), x unit-stride; offsets are lists of integer tuples in the
same axis order.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "stencil_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

BC_ZERO = 0
BC_PERIODIC = 1
_BC = {"zero": BC_ZERO, "periodic": BC_PERIODIC, BC_ZERO: BC_ZERO, BC_PERIODIC: BC_PERIODIC}

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: -O2, no FP contraction, OpenMP."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
               "-shared", "-std=c99", "-Wall", "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        i32, i64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        p_i64 = ctypes.POINTER(ctypes.c_int64)
        p_i32 = ctypes.POINTER(ctypes.c_int32)
        p_dbl = ctypes.POINTER(ctypes.c_double)
        lib.oracle_sweep.argtypes = [i32, p_i64, i32, p_i32, p_dbl, i32, i64, p_dbl, i32]
        lib.oracle_sweep_transpose.argtypes = [i32, p_i64, i32, p_i32, p_dbl, i32, i64, p_dbl]
        lib.oracle_heat.argtypes = [i32, p_i64, dbl, i32, i64, p_dbl, i32]
        lib.oracle_sweep_point.argtypes = [i32, p_i64, i32, p_i32, p_dbl, i32, i64, p_dbl,
                                           p_i64, p_dbl]
        lib.oracle_varcoef_forward.argtypes = [p_i64, p_dbl, dbl, i64, p_dbl, i64, p_dbl, i32]
        lib.oracle_varcoef_adjoint.argtypes = [p_i64, p_dbl, dbl, i64, p_dbl, p_dbl, p_dbl]
        lib.oracle_max_threads.argtypes = []
        for f in (lib.oracle_sweep, lib.oracle_sweep_transpose, lib.oracle_heat,
                  lib.oracle_sweep_point, lib.oracle_varcoef_forward,
                  lib.oracle_varcoef_adjoint, lib.oracle_max_threads, lib.oracle_sweep_flux):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _shape(a: np.ndarray):
    return (ctypes.c_int64 * a.ndim)(*a.shape)


def _pattern(offsets: Sequence[Sequence[int]], weights: Sequence[float], ndim: int):
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int32).reshape(-1, ndim))
    w = np.ascontiguousarray(np.asarray(weights, dtype=np.float64).reshape(-1))
    if off.shape[0] != w.shape[0]:
        raise ValueError("offsets and weights differ in length")
    return off, w


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"{what} rejected its arguments (rc={rc})")


def max_threads() -> int:
    """Threads the oracle's OpenMP loops use by default."""
    return int(_load().oracle_max_threads())


def sweep(u0: np.ndarray, offsets, weights, steps: int, bc="zero",
          threads: int = 0) -> np.ndarray:
    """u_T = S^T u_0 for the weighted-sum stencil S (Alg. 1 form)."""
    u = np.array(u0, dtype=np.float64, order="C", copy=True)
    off, w = _pattern(offsets, weights, u.ndim)
    rc = _load().oracle_sweep(u.ndim, _shape(u), off.shape[0], _ptr(off, ctypes.c_int32),
                              _ptr(w, ctypes.c_double), _BC[bc], int(steps),
                              _ptr(u, ctypes.c_double), int(threads))
    _check(rc, "oracle_sweep")
    return u


def heat_spectral(u0: np.ndarray, alpha: float, steps: int) -> np.ndarray:
    """Closed form of `steps` explicit heat steps (Eq. 3, increment form) under
    the zero rule: the step is diagonal in the DST-I basis, with eigenvalue
    1 - 4*alpha*sum_d sin^2(pi*k_d / (2*(n_d + 1))) for mode k; so transform,
    raise the eigenvalues to the power `steps`, transform back.  scipy's
    orthonormal DST-I is the library step.  Rounding differs from the loop
    oracle (it is a different computation of the same exact result)."""
    import scipy.fft
    u0 = np.asarray(u0, dtype=np.float64)
    lam = np.zeros(u0.shape)
    for axis, n in enumerate(u0.shape):
        k = np.arange(1, n + 1)
        view = [1] * u0.ndim
        view[axis] = n
        lam = lam + (np.sin(np.pi * k / (2.0 * (n + 1))) ** 2).reshape(view)
    lam = 1.0 - 4.0 * alpha * lam
    c = scipy.fft.dstn(u0, type=1, norm="ortho")
    c *= lam ** int(steps)
    return scipy.fft.idstn(c, type=1, norm="ortho")


def sweep_flux(u0: np.ndarray, offsets, weights, steps: int):
    """(u_T, outflow): the zero-rule sweep and the total amount its steps send
    across the grid's boundary (each step sends w_p * u[c] to c - off_p;
    whatever lands outside the grid leaves), summed in FP64."""
    u = np.array(u0, dtype=np.float64, order="C", copy=True)
    off, w = _pattern(offsets, weights, u.ndim)
    flux = ctypes.c_double(0.0)
    rc = _load().oracle_sweep_flux(u.ndim, _shape(u), off.shape[0], _ptr(off, ctypes.c_int32),
                                   _ptr(w, ctypes.c_double), int(steps), _ptr(u, ctypes.c_double),
                                   ctypes.byref(flux))
    _check(rc, "oracle_sweep_flux")
    return u, float(flux.value)


def sweep_transpose(v: np.ndarray, offsets, weights, steps: int, bc="zero") -> np.ndarray:
    """(S^T)^steps v: the transposed weighted-sum operator, by scatter."""
    out = np.array(v, dtype=np.float64, order="C", copy=True)
    off, w = _pattern(offsets, weights, out.ndim)
    rc = _load().oracle_sweep_transpose(out.ndim, _shape(out), off.shape[0],
                                        _ptr(off, ctypes.c_int32), _ptr(w, ctypes.c_double),
                                        _BC[bc], int(steps), _ptr(out, ctypes.c_double))
    _check(rc, "oracle_sweep_transpose")
    return out


def heat(u0: np.ndarray, alpha: float, steps: int, bc="zero", threads: int = 0) -> np.ndarray:
    """Explicit heat steps in increment form u + a*(sum_nbr - 2d*u)."""
    u = np.array(u0, dtype=np.float64, order="C", copy=True)
    rc = _load().oracle_heat(u.ndim, _shape(u), float(alpha), _BC[bc], int(steps),
                             _ptr(u, ctypes.c_double), int(threads))
    _check(rc, "oracle_heat")
    return u


def sweep_point(u0: np.ndarray, offsets, weights, steps: int, at: Sequence[int],
                bc="zero") -> float:
    """One cell of sweep(u0, ...) computed on its dependency cone."""
    u = np.ascontiguousarray(u0, dtype=np.float64)
    off, w = _pattern(offsets, weights, u.ndim)
    pos = (ctypes.c_int64 * u.ndim)(*[int(a) for a in at])
    out = ctypes.c_double(0.0)
    rc = _load().oracle_sweep_point(u.ndim, _shape(u), off.shape[0], _ptr(off, ctypes.c_int32),
                                    _ptr(w, ctypes.c_double), _BC[bc], int(steps),
                                    _ptr(u, ctypes.c_double), pos, ctypes.byref(out))
    _check(rc, "oracle_sweep_point")
    return float(out.value)


def varcoef_forward(u0: np.ndarray, k: np.ndarray, alpha: float, steps: int,
                    every: Optional[int] = None, threads: int = 0):
    """Var-coef heat forward run; returns u_T, or (u_T, checkpoints) if every."""
    u = np.array(u0, dtype=np.float64, order="C", copy=True)
    kk = np.ascontiguousarray(k, dtype=np.float64)
    if u.ndim != 3 or kk.shape != u.shape:
        raise ValueError("var-coef oracle is 3D with k shaped like u")
    ck = None
    if every:
        nck = -(-int(steps) // int(every))
        ck = np.zeros((max(nck, 1),) + u.shape, dtype=np.float64)
    rc = _load().oracle_varcoef_forward(_shape(u), _ptr(kk, ctypes.c_double), float(alpha),
                                        int(steps), _ptr(u, ctypes.c_double),
                                        int(every or 0),
                                        _ptr(ck, ctypes.c_double) if ck is not None else None,
                                        int(threads))
    _check(rc, "oracle_varcoef_forward")
    return (u, ck[: -(-int(steps) // int(every))]) if every else u


def varcoef_adjoint(u0: np.ndarray, k: np.ndarray, alpha: float, steps: int,
                    lam_T: np.ndarray):
    """Reverse mode of varcoef_forward: returns (dL/du0, dL/dk) from dL/du_T."""
    u = np.ascontiguousarray(u0, dtype=np.float64)
    kk = np.ascontiguousarray(k, dtype=np.float64)
    lam = np.array(lam_T, dtype=np.float64, order="C", copy=True)
    gk = np.zeros_like(u)
    rc = _load().oracle_varcoef_adjoint(_shape(u), _ptr(kk, ctypes.c_double), float(alpha),
                                        int(steps), _ptr(u, ctypes.c_double),
                                        _ptr(lam, ctypes.c_double), _ptr(gk, ctypes.c_double))
    _check(rc, "oracle_varcoef_adjoint")
    return lam, gk


def rel_l2(a: np.ndarray, ref: np.ndarray) -> float:
    """||a - ref||_2 / ||ref||_2 in FP64."""
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = float(np.sqrt(np.sum(ref * ref)))
    num = float(np.sqrt(np.sum((a - ref) ** 2)))
    return num / den if den > 0 else num


def stencils_per_second(shape: Sequence[int], steps: int, seconds: float) -> float:
    """Eq. 5: (product of the grid extents) * T / time."""
    n = 1
    for s in shape:
        n *= int(s)
    return n * float(steps) / float(seconds)
