"""ctypes binding of libgpchol (include/gpchol.h): argument marshalling only.

Tensors are torch float64 CUDA (HIP) tensors, 2-D, row-major with unit column
stride (``t.stride(1) == 1``); the row stride is passed as the leading
dimension, so sub-matrix views work.  Every call enqueues on torch's current
stream of the tensor's device and returns without waiting.  All arithmetic runs
in the library's HIP kernels; there is no fallback: if ``libgpchol.so`` is
missing or the device is not gfx950, the calls raise.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgpchol.so")

(GPC_OK, GPC_ERR_ARG, GPC_ERR_NO_DEVICE, GPC_ERR_ARCH, GPC_ERR_HIP, GPC_ERR_REFINE, GPC_ERR_ALLOC,
 GPC_ERR_SWEEP, GPC_ERR_CAPTURE) = range(9)
GPC_FP64, GPC_MIXED = 0, 1
GPC_NOTRANS, GPC_TRANS = 0, 1

# Every symbol the header declares, in declaration order.
EXPORTS = (
    "gpc_create", "gpc_destroy", "gpc_set_stream", "gpc_check", "gpc_set_options", "gpc_get_options",
    "gpc_factor", "gpc_factor_noalloc", "gpc_get_fallback", "gpc_adjoint", "gpc_trsm", "gpc_logdet",
    "gpc_solve_refined", "gpc_gp_kgen_se", "gpc_gp_value", "gpc_gp_value_refined", "gpc_gp_lbar", "gpc_gp_hypergrad_se",
    "gpc_factor_batched", "gpc_adjoint_batched", "gpc_factor_adjoint_batched", "gpc_autotune_batched",
    "gpc_get_tuning",
    "gpc_trace_enable", "gpc_trace_reset", "gpc_trace_read",
    "gpc_status_string", "gpc_last_error",
)

# Kernel classes of the launch trace (gpc_kernel_class).
KERNEL_CLASSES = ("diag_factor", "panel_solve", "trailing_update", "diag_inverse", "adj_panel_solve",
                  "adj_left_update", "adj_diag_product", "adj_diag_block", "adj_row_update", "reduce",
                  "batched", "trailing_narrow", "ops")


class GpcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(msg)
        self.status = status


class gpc_options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("block", ctypes.c_int32),
                ("lookahead", ctypes.c_int32), ("refine_maxit", ctypes.c_int32),
                ("refine_tol", ctypes.c_double), ("mixed_fallback", ctypes.c_int32),
                ("test_flags", ctypes.c_int32), ("gemm_max_splits", ctypes.c_int32),
                ("batched_schedule", ctypes.c_int32), ("adjoint_group", ctypes.c_int32)]


_i64, _i32, _vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
_lib = None


def load_library(path: str = LIB_PATH):
    """Load libgpchol.so and declare the C signatures (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run `python -m paper_1907_01063_amd.build`")
    lib = ctypes.CDLL(path)
    sig = {
        "gpc_create": [ctypes.POINTER(_vp), _vp],
        "gpc_destroy": [_vp],
        "gpc_set_stream": [_vp, _vp],
        "gpc_check": [_vp],
        "gpc_set_options": [_vp, ctypes.POINTER(gpc_options)],
        "gpc_get_options": [_vp, ctypes.POINTER(gpc_options)],
        "gpc_factor": [_vp, _i64, _vp, _i64, _vp],
        "gpc_factor_noalloc": [_vp, _i64, _vp, _i64, _vp],
        "gpc_adjoint": [_vp, _i64, _vp, _i64, _vp, _i64],
        "gpc_trsm": [_vp, _i32, _i64, _i64, _vp, _i64, _vp, _i64],
        "gpc_logdet": [_vp, _i64, _vp, _i64, _vp],
        "gpc_solve_refined": [_vp, _i64, _vp, _i64, _vp, _i64, _vp, _vp, _vp, _vp],
        "gpc_gp_kgen_se": [_vp, _i64, _i32, _vp, _vp, _vp, _i64],
        "gpc_gp_value": [_vp, _i64, _vp, _i64, _vp, _vp, _vp, _vp, _vp],
        "gpc_gp_value_refined": [_vp, _i64, _vp, _i64, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp],
        "gpc_gp_lbar": [_vp, _i64, _vp, _i64, _vp, _vp, _vp, _i64],
        "gpc_gp_hypergrad_se": [_vp, _i64, _i32, _vp, _vp, _vp, _i64, _vp, _vp],
        "gpc_factor_batched": [_vp, _i32, _vp, _vp, _vp, _vp],
        "gpc_adjoint_batched": [_vp, _i32, _vp, _vp, _vp, _vp],
        "gpc_factor_adjoint_batched": [_vp, _i32, _vp, _vp, _vp, _vp, _vp],
        "gpc_autotune_batched": [_vp, ctypes.c_char_p],
        "gpc_get_tuning": [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32)],
        "gpc_get_fallback": [_vp, ctypes.POINTER(_i32)],
        "gpc_trace_enable": [_vp, _i32],
        "gpc_trace_reset": [_vp],
        "gpc_trace_read": [_vp, _i32, ctypes.POINTER(_i64), ctypes.POINTER(ctypes.c_double),
                           ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.gpc_status_string.argtypes = [ctypes.c_int]
    lib.gpc_status_string.restype = ctypes.c_char_p
    lib.gpc_last_error.argtypes = [_vp]
    lib.gpc_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _ptr(t) -> int:
    return 0 if t is None else t.data_ptr()


def _mat(t: torch.Tensor, name: str):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or t.dim() != 2 or not t.is_cuda:
        raise TypeError(f"{name}: expected a 2-D float64 GPU tensor")
    if t.numel() == 0:   # no element is addressed: the smallest valid row stride
        return max(1, t.shape[1])
    if t.shape[1] > 1 and t.stride(1) != 1:
        raise ValueError(f"{name}: needs unit column stride (row-major)")
    return t.stride(0) if t.shape[0] > 1 else max(1, t.shape[1])


class Handle:
    """One library handle per (device, host thread).  Calls follow torch's
    current stream at call time."""

    def __init__(self, device=None, precision: int = GPC_FP64, block: int = 0):
        self.lib = load_library()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else
                                   torch.device(device).index or 0)
        h = _vp()
        with torch.cuda.device(self.device):
            st = self.lib.gpc_create(ctypes.byref(h), _vp(torch.cuda.current_stream().cuda_stream))
        if st != GPC_OK:
            raise GpcError(st, f"gpc_create: {self.lib.gpc_status_string(st).decode()}")
        self.h = h
        if precision != GPC_FP64 or block != 0:
            self.set_options(precision=precision, block=block)

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self.lib.gpc_destroy(h)
            self.h = None

    def _check(self, st: int, what: str):
        if st != GPC_OK:
            msg = self.lib.gpc_last_error(self.h).decode() if self.h else ""
            raise GpcError(st, f"{what}: {self.lib.gpc_status_string(st).decode()} {msg}".strip())

    def _sync_stream(self):
        self.lib.gpc_set_stream(self.h, _vp(torch.cuda.current_stream(self.device).cuda_stream))

    def check(self):
        """Wait for the stream; raise GpcError(GPC_ERR_SWEEP) if a one-launch
        solve sweep of this handle ran out of time since the last check."""
        self._sync_stream()
        self._check(self.lib.gpc_check(self.h), "gpc_check")

    def options(self) -> gpc_options:
        o = gpc_options()
        self._check(self.lib.gpc_get_options(self.h, ctypes.byref(o)), "gpc_get_options")
        return o

    def set_options(self, **kw):
        o = self.options()
        for k, v in kw.items():
            setattr(o, k, v)
        self._check(self.lib.gpc_set_options(self.h, ctypes.byref(o)), "gpc_set_options")

    # --- entry points (same names as the C ABI, without the prefix) ---
    def factor(self, A: torch.Tensor, info: torch.Tensor | None = None) -> torch.Tensor:
        """In place: tril(A) <- L, strict upper <- 0.  Returns the device int32 info."""
        lda = _mat(A, "A")
        n = A.shape[0]
        if A.shape[1] != n:
            raise ValueError("A must be square")
        if info is None:
            info = torch.empty((), dtype=torch.int32, device=A.device)
        self._sync_stream()
        self._check(self.lib.gpc_factor(self.h, n, _ptr(A), lda, _ptr(info)), "gpc_factor")
        return info

    def factor_noalloc(self, A: torch.Tensor, info: torch.Tensor) -> torch.Tensor:
        """gpc_factor_noalloc: the FP64 factor in place with no device
        allocation (the caller passes info as well)."""
        lda = _mat(A, "A")
        n = A.shape[0]
        if A.shape[1] != n:
            raise ValueError("A must be square")
        self._sync_stream()
        self._check(self.lib.gpc_factor_noalloc(self.h, n, _ptr(A), lda, _ptr(info)), "gpc_factor_noalloc")
        return info

    def fell_back(self) -> bool:
        """True if the last factor call was a mixed-precision one that lost
        definiteness in its FP32 updates and was redone in FP64."""
        f = _i32(0)
        self._check(self.lib.gpc_get_fallback(self.h, ctypes.byref(f)), "gpc_get_fallback")
        return bool(f.value)

    def adjoint(self, L: torch.Tensor, Lbar: torch.Tensor) -> torch.Tensor:
        """In place: tril(Lbar) <- Abar, strict upper <- 0.  Returns Lbar."""
        ldl, ldb = _mat(L, "L"), _mat(Lbar, "Lbar")
        n = L.shape[0]
        if L.shape != (n, n) or Lbar.shape != (n, n):
            raise ValueError("L and Lbar must be n x n")
        self._sync_stream()
        self._check(self.lib.gpc_adjoint(self.h, n, _ptr(L), ldl, _ptr(Lbar), ldb), "gpc_adjoint")
        return Lbar

    def trsm(self, L: torch.Tensor, B: torch.Tensor, trans: bool = False) -> torch.Tensor:
        """In place: B <- L^-1 B (or L^-T B).  B is n x nrhs (a 1-D B is one column)."""
        ldl = _mat(L, "L")
        B2 = B.unsqueeze(1) if B.dim() == 1 else B
        ldb = _mat(B2, "B")
        n = L.shape[0]
        if B2.shape[0] != n:
            raise ValueError("B must have n rows")
        self._sync_stream()
        self._check(self.lib.gpc_trsm(self.h, GPC_TRANS if trans else GPC_NOTRANS, n, B2.shape[1],
                                      _ptr(L), ldl, _ptr(B2), ldb), "gpc_trsm")
        return B

    def solve_refined(self, K: torch.Tensor, L: torch.Tensor, y: torch.Tensor, x: torch.Tensor | None = None,
                      check: bool = True):
        """x solving K x = y by FP64 refinement with the factor L.  Returns
        (x, iters, eta) with iters/eta as device scalars.  With check=True a
        non-converged refinement raises GpcError(GPC_ERR_REFINE)."""
        ldk, ldl = _mat(K, "K"), _mat(L, "L")
        n = K.shape[0]
        if x is None:
            x = torch.empty_like(y)
        iters = torch.empty((), dtype=torch.int32, device=K.device)
        eta = torch.empty((), dtype=torch.float64, device=K.device)
        self._sync_stream()
        st = self.lib.gpc_solve_refined(self.h, n, _ptr(K), ldk, _ptr(L), ldl, _ptr(y), _ptr(x),
                                        _ptr(iters), _ptr(eta))
        if not (st == GPC_ERR_REFINE and not check):
            self._check(st, "gpc_solve_refined")
        return x, iters, eta

    def gp_kgen_se(self, X: torch.Tensor, theta: torch.Tensor, K: torch.Tensor | None = None) -> torch.Tensor:
        n, d = X.shape
        if K is None:
            K = torch.empty((n, n), dtype=torch.float64, device=X.device)
        self._sync_stream()
        self._check(self.lib.gpc_gp_kgen_se(self.h, n, d, _ptr(X.contiguous()), _ptr(theta.contiguous()),
                                            _ptr(K), _mat(K, "K")), "gpc_gp_kgen_se")
        return K

    def gp_value(self, L: torch.Tensor, y: torch.Tensor):
        """(f, z, alpha, logdet) of the GP log-density from the factor L."""
        n = L.shape[0]
        z, alpha = torch.empty_like(y), torch.empty_like(y)
        ld = torch.empty((), dtype=torch.float64, device=L.device)
        f = torch.empty((), dtype=torch.float64, device=L.device)
        self._sync_stream()
        self._check(self.lib.gpc_gp_value(self.h, n, _ptr(L), _mat(L, "L"), _ptr(y), _ptr(z), _ptr(alpha),
                                          _ptr(ld), _ptr(f)), "gpc_gp_value")
        return f, z, alpha, ld

    def gp_value_refined(self, K: torch.Tensor, L: torch.Tensor, y: torch.Tensor, check: bool = True):
        """(f, z, alpha, logdet, iters, eta) with alpha from FP64 refinement
        against K and z = L^T alpha.  With check=False a refinement that did
        not reach its tolerance still returns its outputs."""
        n = L.shape[0]
        z, alpha = torch.empty_like(y), torch.empty_like(y)
        ld = torch.empty((), dtype=torch.float64, device=L.device)
        f = torch.empty((), dtype=torch.float64, device=L.device)
        iters = torch.empty((), dtype=torch.int32, device=L.device)
        eta = torch.empty((), dtype=torch.float64, device=L.device)
        self._sync_stream()
        st = self.lib.gpc_gp_value_refined(self.h, n, _ptr(K), _mat(K, "K"), _ptr(L), _mat(L, "L"), _ptr(y),
                                           _ptr(z), _ptr(alpha), _ptr(ld), _ptr(f), _ptr(iters), _ptr(eta))
        if not (st == GPC_ERR_REFINE and not check):
            self._check(st, "gpc_gp_value_refined")
        return f, z, alpha, ld, iters, eta

    def gp_lbar(self, L: torch.Tensor, alpha: torch.Tensor, z: torch.Tensor, Lbar: torch.Tensor | None = None):
        n = L.shape[0]
        if Lbar is None:
            Lbar = torch.empty_like(L)
        self._sync_stream()
        self._check(self.lib.gpc_gp_lbar(self.h, n, _ptr(L), _mat(L, "L"), _ptr(alpha), _ptr(z), _ptr(Lbar),
                                         _mat(Lbar, "Lbar")), "gpc_gp_lbar")
        return Lbar

    def gp_hypergrad_se(self, X: torch.Tensor, theta: torch.Tensor, Abar: torch.Tensor,
                        scale: torch.Tensor | None = None) -> torch.Tensor:
        n, d = X.shape
        grad = torch.empty(d + 2, dtype=torch.float64, device=X.device)
        self._sync_stream()
        self._check(self.lib.gpc_gp_hypergrad_se(self.h, n, d, _ptr(X.contiguous()), _ptr(theta.contiguous()),
                                                 _ptr(Abar), _mat(Abar, "Abar"), _ptr(scale), _ptr(grad)),
                    "gpc_gp_hypergrad_se")
        return grad

    def _batch_args(self, n, off):
        import numpy as np
        n_arr = np.ascontiguousarray(np.asarray(n, dtype=np.int32))
        off_arr = np.ascontiguousarray(np.asarray(off, dtype=np.int64))
        if n_arr.shape != off_arr.shape or n_arr.ndim != 1:
            raise ValueError("n and off must be 1-D of equal length")
        self._keep = (n_arr, off_arr)
        return len(n_arr), n_arr.ctypes.data_as(_vp), off_arr.ctypes.data_as(_vp)

    def factor_batched(self, n, off, base: torch.Tensor, info: torch.Tensor | None = None) -> torch.Tensor:
        """Factor every matrix of a packed batch in place (one persistent launch)."""
        nb, pn, po = self._batch_args(n, off)
        if info is None:
            info = torch.empty(nb, dtype=torch.int32, device=base.device)
        self._sync_stream()
        self._check(self.lib.gpc_factor_batched(self.h, nb, pn, po, _ptr(base), _ptr(info)), "gpc_factor_batched")
        return info

    def adjoint_batched(self, n, off, Lbase: torch.Tensor, Lbarbase: torch.Tensor) -> torch.Tensor:
        nb, pn, po = self._batch_args(n, off)
        self._sync_stream()
        self._check(self.lib.gpc_adjoint_batched(self.h, nb, pn, po, _ptr(Lbase), _ptr(Lbarbase)),
                    "gpc_adjoint_batched")
        return Lbarbase

    def factor_adjoint_batched(self, n, off, base: torch.Tensor, Lbarbase: torch.Tensor,
                               info: torch.Tensor | None = None) -> torch.Tensor:
        nb, pn, po = self._batch_args(n, off)
        if info is None:
            info = torch.empty(nb, dtype=torch.int32, device=base.device)
        self._sync_stream()
        self._check(self.lib.gpc_factor_adjoint_batched(self.h, nb, pn, po, _ptr(base), _ptr(Lbarbase),
                                                        _ptr(info)), "gpc_factor_adjoint_batched")
        return info

    def autotune_batched(self, cache_path: str | None = None):
        self._sync_stream()
        self._check(self.lib.gpc_autotune_batched(self.h, cache_path.encode() if cache_path else None),
                    "gpc_autotune_batched")

    def tuning(self):
        blocks = (_i32 * 5)()
        tuned = _i32()
        self._check(self.lib.gpc_get_tuning(self.h, blocks, ctypes.byref(tuned)), "gpc_get_tuning")
        return list(blocks), bool(tuned.value)

    def trace_enable(self, on: bool = True):
        self._check(self.lib.gpc_trace_enable(self.h, 1 if on else 0), "gpc_trace_enable")

    def trace_reset(self):
        self._sync_stream()
        self._check(self.lib.gpc_trace_reset(self.h), "gpc_trace_reset")

    def trace_read(self) -> dict:
        """{class name: (launches, ms, flops, bytes)} for every kernel class."""
        out = {}
        for k, name in enumerate(KERNEL_CLASSES):
            n, ms, fl, by = _i64(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
            self._check(self.lib.gpc_trace_read(self.h, k, ctypes.byref(n), ctypes.byref(ms),
                                                ctypes.byref(fl), ctypes.byref(by)), "gpc_trace_read")
            out[name] = (n.value, ms.value, fl.value, by.value)
        return out

    def logdet(self, L: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        ldl = _mat(L, "L")
        if out is None:
            out = torch.empty((), dtype=torch.float64, device=L.device)
        self._sync_stream()
        self._check(self.lib.gpc_logdet(self.h, L.shape[0], _ptr(L), ldl, _ptr(out)), "gpc_logdet")
        return out


_handles: dict = {}


def default_handle(device=None) -> Handle:
    dev = torch.cuda.current_device() if device is None else torch.device(device).index or 0
    if dev not in _handles:
        _handles[dev] = Handle(device=dev)
    return _handles[dev]
