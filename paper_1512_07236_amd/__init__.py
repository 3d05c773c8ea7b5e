"""GPU generalized canonical purification on AMD Instinct MI355X (gfx950).

Thin ctypes binding over ``lib/libgcp.so`` (C ABI: ``include/gcp.h``).  This
module only marshals arguments: every step of the purification runs in the
library's HIP kernels.  PyTorch supplies device memory and the stream.  If the
library is missing or cannot be loaded, importing the binding's entry points
raises; there is no CPU fallback.

Typical use::

    import torch, paper_1512_07236_amd as gcp
    H = torch.as_tensor(H_np, device="cuda")            # FP64, symmetric
    D, info = gcp.purify(H, N, emin=-1.0, emax=1.0, precision="fp16x3")
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass
from enum import IntEnum
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libgcp.so")


class Precision(IntEnum):
    FP64 = 0
    FP32 = 1
    BF16 = 2
    FP16 = 3
    BF16X3 = 4
    FP16X3 = 5
    BF16X6 = 6

    @classmethod
    def parse(cls, p) -> "Precision":
        if isinstance(p, cls):
            return p
        if isinstance(p, int):
            return cls(p)
        return cls[str(p).upper()]


# products per matrix multiplication (split encodings issue several)
PRODUCTS = {Precision.FP64: 1, Precision.FP32: 1, Precision.BF16: 1, Precision.FP16: 1,
            Precision.BF16X3: 3, Precision.FP16X3: 3, Precision.BF16X6: 6}
# MFMA data type each precision issues
MFMA_DTYPE = {Precision.FP64: "fp64", Precision.FP32: "fp32", Precision.BF16: "bf16",
              Precision.FP16: "fp16", Precision.BF16X3: "bf16", Precision.FP16X3: "fp16",
              Precision.BF16X6: "bf16"}

OK, ERR_INVALID_ARG, ERR_HIP, ERR_NO_MEMORY, ERR_NOT_CONVERGED, ERR_BREAKDOWN, ERR_STATE, \
    ERR_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
# not an error: the rounding floor of the encoding was reached above tol_ddbar
STOPPED_AT_FLOOR = 1
SUCCESS = (OK, STOPPED_AT_FLOOR)
STATUS_NAMES = {OK: "OK", STOPPED_AT_FLOOR: "STOPPED_AT_FLOOR", ERR_INVALID_ARG: "INVALID_ARG", ERR_HIP: "HIP", ERR_NO_MEMORY: "NO_MEMORY",
                ERR_NOT_CONVERGED: "NOT_CONVERGED", ERR_BREAKDOWN: "BREAKDOWN",
                ERR_STATE: "STATE", ERR_UNSUPPORTED: "UNSUPPORTED"}
DTYPE_F64, DTYPE_F32 = 0, 1
HIST_COLS = 9
HIST_FIELDS = ("n", "t1", "t2", "t3", "c", "omega", "gamma", "lagrangian", "step")


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("tol_ddbar", ctypes.c_double), ("tol_idem", ctypes.c_double),
                ("fold_every", ctypes.c_int32), ("profile", ctypes.c_int32),
                ("keep_iterates", ctypes.c_int32), ("bwd_precision", ctypes.c_int32),
                ("late_precision", ctypes.c_int32), ("final_precision", ctypes.c_int32),
                ("switch_ddbar", ctypes.c_double), ("method", ctypes.c_int32),
                ("init_mode", ctypes.c_int32), ("alpha", ctypes.c_double),
                ("delta", ctypes.c_double), ("hole", ctypes.c_int32),
                ("checkpoint_every", ctypes.c_int32), ("sync_every", ctypes.c_int32),
                ("ksplit", ctypes.c_int32), ("floor_ddbar", ctypes.c_double),
                ("final_ddbar", ctypes.c_double)]


METHODS = {"hpcp": 0, "pmcp": 1}           # the recursion
INITS = {"pmcp": 0, "hp": 1, "search": 2}  # the initial guess


class CResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("t1", ctypes.c_double), ("t2", ctypes.c_double), ("c_last", ctypes.c_double),
                ("idem", ctypes.c_double), ("ms_total", ctypes.c_double),
                ("gemm_ms", ctypes.c_double), ("gemm_launches", ctypes.c_int32),
                ("host_syncs", ctypes.c_int32), ("gemm_flops", ctypes.c_double),
                ("mfma_flops", ctypes.c_double)]


class CVerify(ctypes.Structure):
    _fields_ = [("trace", ctypes.c_double), ("fro2", ctypes.c_double), ("idem", ctypes.c_double),
                ("energy", ctypes.c_double), ("comm", ctypes.c_double), ("ms", ctypes.c_double)]


class GCPError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load_library() -> ctypes.CDLL:
    """Load libgcp.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libgcp.so not found at {LIB_PATH}; build it with "
                          "`python -m paper_1512_07236_amd._build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.gcp_options_default.argtypes = [ctypes.POINTER(Options)]
    L.gcp_options_default.restype = ctypes.c_int
    L.gcp_create.argtypes = [ctypes.POINTER(vp), i64, ctypes.POINTER(Options), vp]
    L.gcp_create.restype = ctypes.c_int
    L.gcp_destroy.argtypes = [vp]
    L.gcp_destroy.restype = None
    L.gcp_init.argtypes = [vp, vp, i64, i64, dbl, dbl]
    L.gcp_init.restype = ctypes.c_int
    L.gcp_purify.argtypes = [vp, vp, i32, i64, ctypes.POINTER(CResult)]
    L.gcp_purify.restype = ctypes.c_int
    L.gcp_backward.argtypes = [vp, vp, i64, vp, i64, i32, ctypes.POINTER(CResult)]
    L.gcp_backward.restype = ctypes.c_int
    L.gcp_verify.argtypes = [vp, vp, i32, i64, vp, i64, ctypes.POINTER(CVerify)]
    L.gcp_verify.restype = ctypes.c_int
    L.gcp_get_history.argtypes = [vp, ctypes.POINTER(ctypes.c_double), i32, ctypes.POINTER(i32)]
    L.gcp_get_history.restype = ctypes.c_int
    L.gcp_get_init_scalars.argtypes = [vp] + [ctypes.POINTER(ctypes.c_double)] * 5
    L.gcp_get_init_scalars.restype = ctypes.c_int
    L.gcp_last_error.argtypes = [vp]
    L.gcp_last_error.restype = ctypes.c_char_p
    L.gcp_purify_static.argtypes = [vp, i64, i64, i64, dbl, dbl, ctypes.POINTER(Options), vp, i32,
                                    i64, vp, ctypes.POINTER(CResult)]
    L.gcp_purify_static.restype = ctypes.c_int
    L.gcp_stream_lds.argtypes = [vp, i64, vp]
    L.gcp_stream_lds.restype = ctypes.c_int
    _lib = L
    return L


def default_options() -> Options:
    o = Options()
    load_library().gcp_options_default(ctypes.byref(o))
    return o


@dataclass
class Result:
    status: int
    iters: int
    t1: float
    t2: float
    c_last: float
    idem: float
    ms_total: float
    gemm_ms: float
    gemm_launches: int
    gemm_flops: float
    mfma_flops: float
    history: np.ndarray
    host_syncs: int = 0

    @property
    def ok(self) -> bool:
        """Converged to the tolerance, or stopped at the encoding's rounding floor."""
        return self.status in SUCCESS

    def col(self, name: str) -> np.ndarray:
        return self.history[:, HIST_FIELDS.index(name)]


def _stream_handle(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


class Context:
    """A purification context for M x M problems (owns the device workspace)."""

    def __init__(self, M: int, precision="fp64", max_iter: int = 100, tol_ddbar: float = 1e-6,
                 tol_idem: float = 0.0, fold_every: int = 0, profile: bool = False,
                 keep_iterates: bool = False, bwd_precision="fp64", late_precision=None,
                 switch_ddbar: float = 0.0, final_precision=None, final_ddbar: float = 0.0,
                 method: str = "hpcp", init: str = "pmcp",
                 alpha: float = 0.5, delta: float = 2.0 / 3.0, hole: bool = False,
                 checkpoint_every: int = 0, sync_every: int = 4, ksplit: int = 0,
                 floor_ddbar: float = math.nan, stream=None):
        L = load_library()
        self._L = L
        self.M = int(M)
        self.precision = Precision.parse(precision)
        o = default_options()
        o.precision = int(self.precision)
        o.max_iter = int(max_iter)
        o.tol_ddbar = float(tol_ddbar)
        o.tol_idem = float(tol_idem)
        o.fold_every = int(fold_every)
        o.profile = 1 if profile else 0
        o.keep_iterates = 1 if keep_iterates else 0
        o.bwd_precision = int(Precision.parse(bwd_precision))
        o.late_precision = -1 if late_precision is None else int(Precision.parse(late_precision))
        o.switch_ddbar = float(switch_ddbar)
        o.final_precision = -1 if final_precision is None else int(Precision.parse(final_precision))
        o.final_ddbar = float(final_ddbar)
        o.method = METHODS[method]
        o.init_mode = INITS[init]
        o.alpha = float(alpha)
        o.delta = float(delta)
        o.hole = 1 if hole else 0
        o.checkpoint_every = int(checkpoint_every)
        o.sync_every = int(sync_every)
        o.ksplit = int(ksplit)
        o.floor_ddbar = float(floor_ddbar)
        self.options = o
        import torch
        # the library works on this stream; calls made while another stream is
        # current first make it wait for that stream (inputs written there)
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        st = L.gcp_create(ctypes.byref(h), self.M, ctypes.byref(o),
                          ctypes.c_void_p(_stream_handle(self._stream)))
        if st != OK:
            raise GCPError(st, L.gcp_last_error(None).decode())
        self._h = h
        self._H = None

    def _check(self, st: int, allow=(OK,)):
        if st not in allow:
            raise GCPError(st, self._L.gcp_last_error(self._h).decode())
        return st

    def _handle(self):
        if not getattr(self, "_h", None):
            raise GCPError(ERR_STATE, "the context is closed")
        import torch
        cur = torch.cuda.current_stream()
        if cur != self._stream:
            self._stream.wait_stream(cur)
        return self._h

    def init(self, H, N: int, emin: float = math.nan, emax: float = math.nan) -> None:
        import torch
        if not (isinstance(H, torch.Tensor) and H.is_cuda and H.dtype == torch.float64):
            raise TypeError("H must be a CUDA float64 tensor")
        if H.dim() != 2 or H.shape[0] != self.M or H.shape[1] != self.M or H.stride(1) != 1:
            raise ValueError(f"H must be {self.M} x {self.M} with unit column stride")
        self._check(self._L.gcp_init(self._handle(), ctypes.c_void_p(H.data_ptr()), H.stride(0), int(N),
                                     float(emin), float(emax)))
        self.N = int(N)

    def purify(self, out=None, dtype=None, raise_on_failure: bool = False):
        """Returns (D, Result).  D is a new (or the given) CUDA tensor."""
        import torch
        if out is None:
            dtype = dtype or torch.float64
            out = torch.empty((self.M, self.M), dtype=dtype, device="cuda")
        if out.dtype not in (torch.float64, torch.float32) or out.stride(1) != 1 or \
                tuple(out.shape) != (self.M, self.M):
            raise ValueError("out must be an M x M float64/float32 CUDA tensor with unit column stride")
        dt = DTYPE_F64 if out.dtype == torch.float64 else DTYPE_F32
        r = CResult()
        st = self._L.gcp_purify(self._handle(), ctypes.c_void_p(out.data_ptr()), dt, out.stride(0),
                                ctypes.byref(r))
        allowed = SUCCESS if raise_on_failure else SUCCESS + (ERR_NOT_CONVERGED, ERR_BREAKDOWN)
        self._check(st, allowed)
        return out, Result(r.status, r.iters, r.t1, r.t2, r.c_last, r.idem, r.ms_total, r.gemm_ms,
                           r.gemm_launches, r.gemm_flops, r.mfma_flops, self.history(),
                           r.host_syncs)

    def backward(self, dL_dD, out=None):
        """dL/dH for the loss gradient dL_dD of the last purify's result
        (needs keep_iterates=True).  Returns (dL_dH, Result)."""
        import torch
        if not (isinstance(dL_dD, torch.Tensor) and dL_dD.is_cuda and
                dL_dD.dtype in (torch.float64, torch.float32) and dL_dD.stride(1) == 1 and
                tuple(dL_dD.shape) == (self.M, self.M)):
            raise ValueError("dL_dD must be an M x M float64/float32 CUDA tensor with unit "
                             "column stride")
        if out is None:
            out = torch.empty((self.M, self.M), dtype=dL_dD.dtype, device=dL_dD.device)
        if out.dtype != dL_dD.dtype or out.stride(1) != 1 or tuple(out.shape) != (self.M, self.M):
            raise ValueError("out must match dL_dD's dtype and shape with unit column stride")
        dt = DTYPE_F64 if out.dtype == torch.float64 else DTYPE_F32
        r = CResult()
        self._check(self._L.gcp_backward(self._handle(), ctypes.c_void_p(dL_dD.data_ptr()),
                                         dL_dD.stride(0), ctypes.c_void_p(out.data_ptr()),
                                         out.stride(0), dt, ctypes.byref(r)))
        return out, Result(r.status, r.iters, r.t1, r.t2, r.c_last, r.idem, r.ms_total, r.gemm_ms,
                           r.gemm_launches, r.gemm_flops, r.mfma_flops, np.zeros((0, HIST_COLS)))

    def verify(self, D, H) -> dict:
        """FP64 checks of D against H on the GPU: Tr D, ||D||_F^2, ||D^2 - D||_F,
        Tr(DH), ||HD - DH||_F (and the call's wall time in ms)."""
        import torch
        for name, X, dts in (("D", D, (torch.float64, torch.float32)), ("H", H, (torch.float64,))):
            if not (isinstance(X, torch.Tensor) and X.is_cuda and X.dtype in dts and
                    X.stride(1) == 1 and tuple(X.shape) == (self.M, self.M)):
                raise ValueError(f"{name} must be an M x M CUDA tensor of {dts} with unit column stride")
        dt = DTYPE_F64 if D.dtype == torch.float64 else DTYPE_F32
        r = CVerify()
        self._check(self._L.gcp_verify(self._handle(), ctypes.c_void_p(D.data_ptr()), dt, D.stride(0),
                                       ctypes.c_void_p(H.data_ptr()), H.stride(0), ctypes.byref(r)))
        return {k: getattr(r, k) for k, _ in CVerify._fields_}

    def history(self) -> np.ndarray:
        n = ctypes.c_int32()
        self._check(self._L.gcp_get_history(self._h, None, 0, ctypes.byref(n)))
        rows = np.full((max(n.value, 0), HIST_COLS), np.nan)
        if n.value > 0:
            self._check(self._L.gcp_get_history(
                self._h, rows.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n.value,
                ctypes.byref(n)))
        return rows

    def init_scalars(self) -> dict:
        v = [ctypes.c_double() for _ in range(5)]
        self._check(self._L.gcp_get_init_scalars(self._h, *[ctypes.byref(x) for x in v]))
        return dict(zip(("mu", "beta", "emin", "emax", "alpha"), (x.value for x in v)))

    def close(self) -> None:
        if getattr(self, "_h", None):
            self._L.gcp_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def purify(H, N: int, emin: float = math.nan, emax: float = math.nan, precision="fp64",
           out=None, **options):
    """One-shot solve: returns (D, Result)."""
    with Context(H.shape[0], precision=precision, **options) as ctx:
        ctx.init(H, N, emin, emax)
        return ctx.purify(out=out)


STATIC_MAX_M = 1024


def purify_static(H, N: int, emin: float = math.nan, emax: float = math.nan, out=None,
                  precision="fp64", **options):
    """gcp_purify_static: the whole solve without any device allocation by the
    library (workspace in its static per-GPU array, M <= STATIC_MAX_M).
    Returns (D, status, iters) where D is `out` (or a new tensor allocated
    here by torch, before the call)."""
    import torch
    L = load_library()
    M = H.shape[0]
    if out is None:
        out = torch.empty((M, M), dtype=torch.float64, device=H.device)
    o = default_options()
    o.precision = int(Precision.parse(precision))
    for k, v in options.items():
        setattr(o, k, v)
    r = CResult()
    st = L.gcp_purify_static(ctypes.c_void_p(H.data_ptr()), H.stride(0), M, int(N), float(emin),
                             float(emax), ctypes.byref(o), ctypes.c_void_p(out.data_ptr()),
                             DTYPE_F64 if out.dtype == torch.float64 else DTYPE_F32,
                             out.stride(0), ctypes.c_void_p(_stream_handle(None)), ctypes.byref(r))
    return out, st, r


def _autograd_function():
    import torch

    class _Purify(torch.autograd.Function):
        """D = purify(H): forward and backward both run in libgcp."""

        @staticmethod
        def forward(ctx, H, N, emin, emax, options):
            options = dict(options)
            retain = bool(options.pop("retain_iterates", False))
            c = Context(H.shape[0], keep_iterates=True, **options)
            c.init(H.detach().contiguous(), N, emin, emax)
            D, res = c.purify(dtype=H.dtype, raise_on_failure=True)
            ctx.gcp = c
            ctx.retain = retain
            ctx.result = res
            return D

        @staticmethod
        def backward(ctx, gD):
            if ctx.gcp is None:
                raise RuntimeError(
                    "purify_autograd: backward ran already and released the stored iterates; "
                    "pass retain_iterates=True to differentiate the same solve more than once")
            dH, _ = ctx.gcp.backward(gD.contiguous())
            if not ctx.retain:
                ctx.gcp.close()   # the p stored iterates are released now
                ctx.gcp = None
            return dH, None, None, None, None

    return _Purify


_PURIFY_FN = None


def purify_autograd(H, N: int, emin: float = math.nan, emax: float = math.nan, **options):
    """Differentiable D(H): a torch.autograd.Function whose backward is the
    library's adjoint (gcp_backward).  The context, with its stored iterates,
    lives until the backward has run (or, with retain_iterates=True, until the
    graph is freed, so that backward may run more than once).  Other options
    are those of Context (FP64 H)."""
    global _PURIFY_FN
    if _PURIFY_FN is None:
        _PURIFY_FN = _autograd_function()
    return _PURIFY_FN.apply(H, int(N), float(emin), float(emax), dict(options))
