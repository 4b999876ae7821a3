"""MI355X (gfx950) stencil sweep -- Python binding of libstencil.so.

Argument marshalling only: every step of the sweep runs in the library's HIP
kernels.  PyTorch supplies device memory (``tensor.data_ptr()``) and the
stream (``torch.cuda.current_stream().cuda_stream``).  If the built library
is missing, every entry point raises -- there is no CPU fallback.

Names follow include/stencil.h: ``Plan`` wraps ``stencil_plan`` /
``stencil_run``; ``BatchPlan`` wraps ``stencil_batch_plan`` /
``stencil_batch_run``.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, List, Optional, Sequence

__all__ = [
    "StencilError", "Plan", "BatchPlan", "run", "library", "library_path", "build",
    "F64", "F32", "BF16", "BC_ZERO", "BC_PERIODIC", "PLAN_AUTOTUNE", "PLAN_NAIVE",
    "PLAN_VARCOEF", "PLAN_GRAPH", "PLAN_OWN_WORK", "KERNEL_NAIVE", "KERNEL_STREAM2D", "KERNEL_STREAM3D", "KERNEL_VARCOEF3D",
    "KERNEL_STREAM1D", "KERNEL_BOX3D",
    "STATUS", "StencilFn", "varcoef_plan", "copy", "autotune_cache", "batch_run",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libstencil.so")

F64, F32, BF16 = 0, 1, 2
BC_ZERO, BC_PERIODIC = 0, 1
PLAN_AUTOTUNE, PLAN_NAIVE, PLAN_VARCOEF, PLAN_GRAPH, PLAN_OWN_WORK = 0x1, 0x2, 0x4, 0x8, 0x10
KERNEL_NAIVE, KERNEL_STREAM2D, KERNEL_STREAM3D, KERNEL_VARCOEF3D, KERNEL_STREAM1D, KERNEL_BOX3D = 0, 1, 2, 3, 4, 5
STATUS = {0: "ST_OK", -1: "ST_ERR_ARG", -2: "ST_ERR_UNSUPPORTED", -3: "ST_ERR_MISMATCH",
          -4: "ST_ERR_NOMEM", -5: "ST_ERR_HIP", -6: "ST_ERR_CAPTURE"}
_DTYPES = {"f64": F64, "f32": F32, "bf16": BF16, F64: F64, F32: F32, BF16: BF16}
_BCS = {"zero": BC_ZERO, "periodic": BC_PERIODIC, BC_ZERO: BC_ZERO, BC_PERIODIC: BC_PERIODIC}


class StencilError(RuntimeError):
    """A libstencil call returned a status other than ST_OK."""

    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.message = message


class PlanInfo(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("tb", ctypes.c_int32), ("radius", ctypes.c_int32),
                ("shape_class", ctypes.c_int32), ("tile_x", ctypes.c_int32),
                ("tile_y", ctypes.c_int32), ("tile_z", ctypes.c_int32), ("block", ctypes.c_int32),
                ("workgroups", ctypes.c_int64), ("lds_bytes", ctypes.c_int64),
                ("variant", ctypes.c_int32), ("ncandidates", ctypes.c_int32), ("pipeline", ctypes.c_int32),
                ("tessellated", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class _Pattern(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("npoints", ctypes.c_int32),
                ("offsets", ctypes.POINTER(ctypes.c_int32))]


_lib = None


def library_path() -> str:
    return _LIB_PATH


def build(force: bool = False) -> str:
    """Compile the HIP library in-tree (see buildlib.py)."""
    from . import buildlib
    return buildlib.build(force=force)


def library():
    """The loaded libstencil.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"libstencil.so is not built at {_LIB_PATH}; run build() first")
        # One HIP runtime per process: PyTorch ships its own libamdhip64 (same
        # soname as the system one the library links).  Loading torch first
        # makes the library bind to that copy; loading the system copy first
        # would leave torch with a second runtime that finds no GPU.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i32, i64, u32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
        p_i64 = ctypes.POINTER(ctypes.c_int64)
        p_dbl = ctypes.POINTER(ctypes.c_double)
        sig = {
            "stencil_plan": [ctypes.POINTER(P), ctypes.POINTER(_Pattern), p_i64, i32, i32, u32],
            "stencil_plan_destroy": [P],
            "stencil_plan_info": [P, ctypes.POINTER(PlanInfo)],
            "stencil_plan_candidate": [P, i32, ctypes.POINTER(PlanInfo)],
            "stencil_plan_select": [P, i32, i32, i32],
            "stencil_run": [P, P, P, p_dbl, p_i64, i64, i32, P],
            "stencil_run_flux": [P, P, P, p_dbl, p_i64, i64, i32, P, P],
            "stencil_run_noalloc": [P, P, p_dbl, p_i64, i64, i32, P],
            "stencil_batch_plan": [ctypes.POINTER(P), ctypes.POINTER(_Pattern), i32, p_i64, i32, i32, u32],
            "stencil_batch_run": [P, i32, ctypes.POINTER(P), ctypes.POINTER(P), p_dbl, p_i64, P],
            "stencil_batch_run_flux": [P, i32, ctypes.POINTER(P), ctypes.POINTER(P), p_dbl, p_i64, P, P],
            "stencil_run_ckpt": [P, P, P, P, ctypes.c_double, i64, i64, ctypes.POINTER(P), P],
            "stencil_adjoint_run": [P, P, ctypes.c_double, p_dbl, ctypes.POINTER(P), i64, i64, P, P, P,
                                    P, P],
            "stencil_copy": [P, P, i64, P],
            "stencil_autotune_cache": [ctypes.c_char_p],
        }
        for name, args in sig.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        lib.stencil_last_error.argtypes = []
        lib.stencil_last_error.restype = ctypes.c_char_p
        lib.stencil_version.argtypes = []
        lib.stencil_version.restype = ctypes.c_char_p
        _lib = lib
    return _lib


def _check(status: int):
    if status != 0:
        msg = library().stencil_last_error().decode(errors="replace")
        raise StencilError(status, msg)


def _pattern(offsets: Sequence[Sequence[int]]):
    offs = [tuple(int(v) for v in o) for o in offsets]
    if not offs:
        raise ValueError("empty point list")
    ndim = len(offs[0])
    flat = (ctypes.c_int32 * (len(offs) * ndim))(*[v for o in offs for v in o])
    pat = _Pattern(ndim, len(offs), ctypes.cast(flat, ctypes.POINTER(ctypes.c_int32)))
    return pat, flat


def _doubles(vals: Iterable[float]):
    v = [float(x) for x in vals]
    return (ctypes.c_double * len(v))(*v)


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _tensor_dtype(t) -> int:
    import torch
    m = {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16}
    if t.dtype not in m:
        raise TypeError(f"unsupported tensor dtype {t.dtype}")
    return m[t.dtype]


def _on_one_gpu(*named):
    """Every tensor the kernels will read or write must be GPU memory of one
    device: a host pointer handed to a kernel would fault the GPU (no XNACK).
    `named` holds (tensor or None, what) pairs; None entries are skipped."""
    dev = None
    for t, what in named:
        if t is None:
            continue
        if not getattr(t, "is_cuda", False):
            raise ValueError(f"{what} must be a GPU tensor (got device {getattr(t, 'device', '?')})")
        if dev is None:
            dev = t.device
        elif t.device != dev:
            raise ValueError(f"{what} is on {t.device}, the other tensors on {dev}")
    return dev


class Plan:
    """A plan for one grid shape (``stencil_plan``)."""

    def __init__(self, offsets, shape, dtype="f64", bc="zero", autotune=False, naive=False,
                 varcoef=False, graph=False, own_work=False):
        lib = library()
        self.offsets = [tuple(int(v) for v in o) for o in offsets]
        self.shape = tuple(int(s) for s in shape)
        self.dtype = _DTYPES[dtype]
        self.bc = _BCS[bc]
        self.own_work = bool(own_work)
        self._work = None
        flags = ((PLAN_AUTOTUNE if autotune else 0) | (PLAN_NAIVE if naive else 0) |
                 (PLAN_VARCOEF if varcoef else 0) | (PLAN_GRAPH if graph else 0) |
                 (PLAN_OWN_WORK if own_work else 0))
        pat, self._flat = _pattern(self.offsets)
        shp = (ctypes.c_int64 * len(self.shape))(*self.shape)
        h = ctypes.c_void_p()
        _check(lib.stencil_plan(ctypes.byref(h), ctypes.byref(pat), shp, self.dtype, self.bc, flags))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            library().stencil_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        i = PlanInfo()
        _check(library().stencil_plan_info(self._h, ctypes.byref(i)))
        return i.as_dict()

    def candidates(self) -> List[dict]:
        n = self.info()["ncandidates"]
        out = []
        for k in range(n):
            i = PlanInfo()
            _check(library().stencil_plan_candidate(self._h, k, ctypes.byref(i)))
            out.append(i.as_dict())
        return out

    def select(self, kernel: int = -1, tb: int = 0, variant: int = -1):
        _check(library().stencil_plan_select(self._h, int(kernel), int(tb), int(variant)))
        return self

    def run(self, grid, coeffs, steps: int, work=None, stream=None):
        """Run `steps` steps in place on the device tensor `grid`."""
        if tuple(grid.shape) != self.shape:
            raise ValueError(f"grid shape {tuple(grid.shape)} != plan shape {self.shape}")
        if not grid.is_contiguous() or _tensor_dtype(grid) != self.dtype:
            raise ValueError("grid must be a contiguous tensor of the plan's dtype")
        if work is not None and (work.numel() != grid.numel() or work.dtype != grid.dtype):
            raise ValueError("work must match grid in size and dtype")
        _on_one_gpu((grid, "grid"), (work, "work"))
        work = self._work_for(grid, work)
        w = _doubles(coeffs)
        if len(w) != len(self.offsets):
            raise ValueError("one coefficient per point")
        shp = (ctypes.c_int64 * len(self.shape))(*self.shape)
        _check(library().stencil_run(self._h, grid.data_ptr(),
                                     work.data_ptr() if work is not None else None, w, shp,
                                     int(steps), self.bc, _stream_handle(stream)))
        return grid

    def run_noalloc(self, grid, coeffs, steps: int, stream=None):
        """``stencil_run_noalloc``: `steps` steps in place on `grid` with the
        library's static work space (no work tensor, nothing allocated)."""
        if tuple(grid.shape) != self.shape:
            raise ValueError(f"grid shape {tuple(grid.shape)} != plan shape {self.shape}")
        if not grid.is_contiguous() or _tensor_dtype(grid) != self.dtype:
            raise ValueError("grid must be a contiguous tensor of the plan's dtype")
        _on_one_gpu((grid, "grid"))
        w = _doubles(coeffs)
        if len(w) != len(self.offsets):
            raise ValueError("one coefficient per point")
        shp = (ctypes.c_int64 * len(self.shape))(*self.shape)
        _check(library().stencil_run_noalloc(self._h, grid.data_ptr(), w, shp, int(steps), self.bc,
                                             _stream_handle(stream)))
        return grid

    def run_flux(self, grid, coeffs, steps: int, flux, work=None, stream=None):
        """``stencil_run_flux``: `steps` steps in place on `grid`, adding the
        outflow across the zero-rule boundary to `flux` (a one-element FP64
        device tensor)."""
        if tuple(grid.shape) != self.shape:
            raise ValueError(f"grid shape {tuple(grid.shape)} != plan shape {self.shape}")
        if not grid.is_contiguous() or _tensor_dtype(grid) != self.dtype:
            raise ValueError("grid must be a contiguous tensor of the plan's dtype")
        if work is not None and (work.numel() != grid.numel() or work.dtype != grid.dtype):
            raise ValueError("work must match grid in size and dtype")
        if flux.numel() != 1 or str(flux.dtype) != "torch.float64" or flux.device != grid.device:
            raise ValueError("flux must be a one-element float64 tensor on the grid's device")
        _on_one_gpu((grid, "grid"), (work, "work"), (flux, "flux"))
        work = self._work_for(grid, work)
        w = _doubles(coeffs)
        if len(w) != len(self.offsets):
            raise ValueError("one coefficient per point")
        shp = (ctypes.c_int64 * len(self.shape))(*self.shape)
        _check(library().stencil_run_flux(self._h, grid.data_ptr(),
                                          work.data_ptr() if work is not None else None, w, shp,
                                          int(steps), self.bc, flux.data_ptr(), _stream_handle(stream)))
        return grid

    def _work_for(self, grid, work):
        """The work buffer to pass: the caller's, NULL for a plan that owns
        one, or a torch tensor this object keeps for later calls."""
        if work is not None or self.own_work:
            return work
        if self._work is None or self._work.device != grid.device:
            import torch
            self._work = torch.empty_like(grid)
        return self._work

    def _same(self, t, what):
        if tuple(t.shape) != self.shape or not t.is_contiguous() or _tensor_dtype(t) != self.dtype:
            raise ValueError(f"{what} must be a contiguous tensor of the plan's shape and dtype")

    def run_ckpt(self, grid, k, alpha: float, steps: int, work, every: int = 0, ckpts=None,
                 stream=None):
        """Variable-coefficient run (``stencil_run_ckpt``) in place on `grid`.

        With `every` > 0, `ckpts` holds ceil(steps/every) tensors that receive
        u^(c*every)."""
        self._same(grid, "grid")
        self._same(k, "k")
        self._same(work, "work")
        if int(every) < 0:
            raise ValueError("every must be >= 0")
        cp = None
        need = 0
        if every:
            need = -(-int(steps) // int(every))
            if ckpts is None or len(ckpts) < need:
                raise ValueError(f"{need} checkpoint tensors are required")
            for c in ckpts[:need]:
                self._same(c, "checkpoint")
            cp = (ctypes.c_void_p * max(need, 1))(*[c.data_ptr() for c in ckpts[:need]])
        _on_one_gpu((grid, "grid"), (k, "k"), (work, "work"),
                    *[(c, "checkpoint") for c in (ckpts or [])[:need]])
        _check(library().stencil_run_ckpt(self._h, grid.data_ptr(), work.data_ptr(), k.data_ptr(),
                                          float(alpha), int(steps), int(every), cp,
                                          _stream_handle(stream)))
        return grid

    def adjoint(self, lam, steps: int, work, k=None, alpha: float = 0.0, coeffs=None, ckpts=None,
                every: int = 0, grad_k=None, seg=None, stream=None):
        """Reverse sweep (``stencil_adjoint_run``): `lam` goes from dL/du_T to dL/du_0."""
        self._same(lam, "lambda")
        self._same(work, "work")
        steps, every = int(steps), int(every)
        w = None
        if coeffs is not None:
            w = _doubles(coeffs)
            if len(w) != len(self.offsets):
                raise ValueError("one coefficient per point")
        if k is not None:
            self._same(k, "k")
        cp = None
        need = 0
        if k is not None and steps > 0:
            # variable coefficients: ceil(steps/every) checkpoints of the
            # grid's shape and min(every, steps) - 1 recomputed states in seg
            if every < 1:
                raise ValueError("every must be >= 1 with variable coefficients")
            need = -(-steps // every)
            if ckpts is None or len(ckpts) < need:
                raise ValueError(f"{need} checkpoint tensors are required")
            for c in ckpts[:need]:
                self._same(c, "checkpoint")
            cp = (ctypes.c_void_p * need)(*[c.data_ptr() for c in ckpts[:need]])
            nseg = min(every, steps) - 1
            if nseg > 0:
                if seg is None:
                    raise ValueError(f"seg must hold {nseg} states of the grid's shape")
                if not seg.is_contiguous() or _tensor_dtype(seg) != self.dtype:
                    raise ValueError("seg must be contiguous and of the plan's dtype")
                if seg.numel() < nseg * lam.numel():
                    raise ValueError(f"seg holds {seg.numel()} values, {nseg} states need {nseg * lam.numel()}")
        if grad_k is not None:
            self._same(grad_k, "grad_k")
        _on_one_gpu((lam, "lambda"), (work, "work"), (k, "k"), (grad_k, "grad_k"),
                    (seg if need else None, "seg"), *[(c, "checkpoint") for c in (ckpts or [])[:need]])
        _check(library().stencil_adjoint_run(
            self._h, k.data_ptr() if k is not None else None, float(alpha), w, cp, int(every),
            int(steps), lam.data_ptr(), grad_k.data_ptr() if grad_k is not None else None,
            seg.data_ptr() if seg is not None else None, work.data_ptr(), _stream_handle(stream)))
        return lam


class BatchPlan:
    """A plan for a batch of 2D grids (``stencil_batch_plan``)."""

    def __init__(self, offsets, shapes, dtype="f32", bc="zero", autotune=False, graph=False):
        lib = library()
        self.offsets = [tuple(int(v) for v in o) for o in offsets]
        self.shapes = [tuple(int(s) for s in sh) for sh in shapes]
        self.dtype = _DTYPES[dtype]
        self.bc = _BCS[bc]
        pat, self._flat = _pattern(self.offsets)
        flat = [s for sh in self.shapes for s in sh]
        shp = (ctypes.c_int64 * len(flat))(*flat)
        h = ctypes.c_void_p()
        flags = (PLAN_AUTOTUNE if autotune else 0) | (PLAN_GRAPH if graph else 0)
        _check(lib.stencil_batch_plan(ctypes.byref(h), ctypes.byref(pat), len(self.shapes), shp,
                                      self.dtype, self.bc, flags))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            library().stencil_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        i = PlanInfo()
        _check(library().stencil_plan_info(self._h, ctypes.byref(i)))
        return i.as_dict()

    def select(self, kernel: int = -1, tb: int = 0, variant: int = -1):
        _check(library().stencil_plan_select(self._h, int(kernel), int(tb), int(variant)))
        return self

    def run(self, grids, works, coeffs, steps, stream=None, flux=None):
        """``stencil_batch_run``; with `flux` (n doubles on the device)
        ``stencil_batch_run_flux``, adding each grid's outflow to its entry."""
        n = len(self.shapes)
        if len(grids) != n or len(works) != n or len(coeffs) != n or len(steps) != n:
            raise ValueError("one grid, work buffer, coefficient row and step count per batch entry")
        for g, w, sh in zip(grids, works, self.shapes):
            if tuple(g.shape) != sh or not g.is_contiguous() or _tensor_dtype(g) != self.dtype:
                raise ValueError("grid shape/dtype/contiguity differs from the plan")
            if w.numel() != g.numel() or w.dtype != g.dtype:
                raise ValueError("work must match its grid")
        _on_one_gpu(*[(g, f"grid {i}") for i, g in enumerate(grids)],
                    *[(w, f"work {i}") for i, w in enumerate(works)], (flux, "flux"))
        gp = (ctypes.c_void_p * n)(*[g.data_ptr() for g in grids])
        wp = (ctypes.c_void_p * n)(*[w.data_ptr() for w in works])
        cf = _doubles([c for row in coeffs for c in row])
        st = (ctypes.c_int64 * n)(*[int(s) for s in steps])
        if flux is None:
            _check(library().stencil_batch_run(self._h, n, gp, wp, cf, st, _stream_handle(stream)))
        else:
            if flux.numel() != n or str(flux.dtype) != "torch.float64" or not flux.is_contiguous():
                raise ValueError("flux must be a contiguous float64 device tensor with one entry per grid")
            _check(library().stencil_batch_run_flux(self._h, n, gp, wp, cf, st, flux.data_ptr(),
                                                    _stream_handle(stream)))
        return grids


def autotune_cache(path: Optional[str]):
    """``stencil_autotune_cache``: keep autotuning choices in `path` (a text
    file read now and rewritten after every new tuning); None stops writing."""
    _check(library().stencil_autotune_cache(None if path is None else os.fsencode(path)))


def copy(dst, src, stream=None):
    """Device copy with the library's streaming kernel (bandwidth reference)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("dst and src differ in size")
    _on_one_gpu((dst, "dst"), (src, "src"))
    _check(library().stencil_copy(dst.data_ptr(), src.data_ptr(), nbytes, _stream_handle(stream)))
    return dst


def run(grid, coeffs, offsets, steps: int, bc="zero", plan: Optional[Plan] = None, work=None,
        stream=None):
    """One-shot sweep: plan (unless given) and run in place on `grid`."""
    if plan is None:
        plan = Plan(offsets, tuple(grid.shape), _tensor_dtype(grid), bc)
    return plan.run(grid, coeffs, steps, work=work, stream=stream)


def batch_run(grids, coeffs, offsets, steps, bc="zero", plan: Optional[BatchPlan] = None, works=None,
              stream=None):
    """One-shot batch: plan (unless given) and run every grid in place.
    `coeffs` holds one weight row per grid, `steps` one count per grid (or
    one count for all); `works` defaults to fresh buffers like the grids."""
    import torch
    n = len(grids)
    steps = list(steps) if hasattr(steps, "__len__") else [int(steps)] * n
    if plan is None:
        dts = {_tensor_dtype(g) for g in grids}
        if len(dts) != 1:
            raise ValueError("all grids of a batch share one dtype")
        plan = BatchPlan(offsets, [tuple(g.shape) for g in grids], dts.pop(), bc)
    if works is None:
        works = [torch.empty_like(g) for g in grids]
    return plan.run(grids, works, coeffs, steps, stream=stream)


_VC_PLANS = {}


def varcoef_plan(shape, dtype="f32", naive=False) -> Plan:
    """Cached variable-coefficient plan (3D radius-1 star, zero boundary).
    naive=True keeps the one-thread-per-cell kernels instead of the
    z-streaming ones."""
    key = (tuple(int(v) for v in shape), _DTYPES[dtype], bool(naive))
    if key not in _VC_PLANS:
        star = [(0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
        _VC_PLANS[key] = Plan(star, key[0], key[1], "zero", varcoef=True, naive=naive)
    return _VC_PLANS[key]


def _make_stencil_fn():
    import torch

    class _StencilFn(torch.autograd.Function):
        """u_T = (A_k)^steps u_0 for the variable-coefficient heat step A_k.

        forward(u0, k, alpha, steps, every) keeps u^(c*every) checkpoints;
        backward recomputes each segment from its checkpoint and steps the
        adjoint back, returning (dL/du0, dL/dk)."""

        @staticmethod
        def forward(ctx, u0, k, alpha, steps, every):
            plan = varcoef_plan(u0.shape, _tensor_dtype(u0))
            u0c = u0.detach().contiguous()
            kc = k.detach().contiguous()
            nck = max(1, -(-int(steps) // int(every)))
            ckpts = [torch.empty_like(u0c) for _ in range(nck)]
            out = u0c.clone()
            work = torch.empty_like(u0c)
            plan.run_ckpt(out, kc, alpha, steps, work, every=every, ckpts=ckpts)
            ctx.save_for_backward(kc, *ckpts)
            ctx.alpha, ctx.steps, ctx.every, ctx.plan = float(alpha), int(steps), int(every), plan
            return out

        @staticmethod
        def backward(ctx, grad_out):
            kc, *ckpts = ctx.saved_tensors
            lam = grad_out.detach().contiguous().clone()
            gk = torch.zeros_like(kc)
            work = torch.empty_like(lam)
            nseg = min(ctx.every, ctx.steps) - 1
            seg = torch.empty((max(nseg, 1),) + tuple(lam.shape), dtype=lam.dtype, device=lam.device)
            ctx.plan.adjoint(lam, ctx.steps, work, k=kc, alpha=ctx.alpha, ckpts=ckpts,
                             every=ctx.every, grad_k=gk, seg=seg)
            return lam, gk, None, None, None

    return _StencilFn


class _LazyFn:
    """``StencilFn.apply(u0, k, alpha, steps, every)`` (imports torch on first use)."""

    _fn = None

    def apply(self, *args):
        if _LazyFn._fn is None:
            _LazyFn._fn = _make_stencil_fn()
        return _LazyFn._fn.apply(*args)


StencilFn = _LazyFn()
