"""Autograd operations over the library's other entry points: the triangular
solve and the lower-triangular inverse (section 3.2), matrix products and
C = A A^T (section 3.1), and the Bernoulli-logit GLM log-likelihood
(section 3.4).  Forward and backward both run in the library's HIP kernels;
this module only moves tensors between the calls.
"""
from __future__ import annotations

import ctypes

import torch

from .gpchol import GPC_NOTRANS, GPC_TRANS, Handle, _mat, _ptr, default_handle, load_library

_i64, _i32, _vp, _dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_double

# Every symbol include/gpchol_ops.h declares, in declaration order.
OPS_EXPORTS = ("gpc_trtri", "gpc_trtri_adjoint", "gpc_trsm_adjoint", "gpc_gemm", "gpc_get_last_splits",
               "gpc_gemm_adjoint", "gpc_multiply_transpose", "gpc_multiply_transpose_adjoint",
               "gpc_glm_bernoulli_logit")

_SIG = {
    "gpc_trtri": [_vp, _i64, _vp, _i64, _vp, _i64],
    "gpc_trtri_adjoint": [_vp, _i64, _vp, _i64, _vp, _i64, _vp, _i64],
    "gpc_trsm_adjoint": [_vp, _i32, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _i64],
    "gpc_gemm": [_vp, _i32, _i32, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _dbl, _vp, _i64],
    "gpc_get_last_splits": [_vp, ctypes.POINTER(_i32)],
    "gpc_gemm_adjoint": [_vp, _i32, _i32, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _dbl, _vp, _i64,
                         _vp, _i64],
    "gpc_multiply_transpose": [_vp, _i64, _i64, _vp, _i64, _vp, _i64],
    "gpc_multiply_transpose_adjoint": [_vp, _i64, _i64, _vp, _i64, _vp, _i64, _dbl, _vp, _i64],
    "gpc_glm_bernoulli_logit": [_vp, _i64, _i64, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i64],
}
_lib = None


def lib():
    """The library with the signatures of gpchol_ops.h declared (raises if not built)."""
    global _lib
    if _lib is None:
        L = load_library()
        for name, args in _SIG.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        _lib = L
    return _lib


def _h(handle):
    return handle or default_handle()


def _call(H: Handle, name: str, *args):
    H._sync_stream()
    H._check(getattr(lib(), name)(H.h, *args), name)


def _square(t, name):
    ld = _mat(t, name)
    if t.shape[0] != t.shape[1]:
        raise ValueError(f"{name} must be square")
    return ld


# ---- entry points (same names as the C ABI, without the prefix) ----------------

def trtri(H: Handle, L: torch.Tensor, X: torch.Tensor | None = None) -> torch.Tensor:
    """X = L^-1 (lower)."""
    ldl = _square(L, "L")
    n = L.shape[0]
    if X is None:
        X = torch.empty_like(L)
    _call(H, "gpc_trtri", n, _ptr(L), ldl, _ptr(X), _square(X, "X"))
    return X


def trtri_adjoint(H: Handle, X: torch.Tensor, Xbar: torch.Tensor, Lbar: torch.Tensor | None = None):
    n = X.shape[0]
    if Lbar is None:
        Lbar = torch.empty_like(X)
    _call(H, "gpc_trtri_adjoint", n, _ptr(X), _square(X, "X"), _ptr(Xbar), _square(Xbar, "Xbar"), _ptr(Lbar),
          _square(Lbar, "Lbar"))
    return Lbar


def trsm_adjoint(H: Handle, L: torch.Tensor, C: torch.Tensor, Cbar: torch.Tensor, trans: bool = False,
                 Lbar: torch.Tensor | None = None) -> torch.Tensor:
    """In place Cbar <- Bbar; returns Lbar.  C, Cbar: n x nrhs (1-D: one column)."""
    n = L.shape[0]
    C2 = C.unsqueeze(1) if C.dim() == 1 else C
    Cb2 = Cbar.unsqueeze(1) if Cbar.dim() == 1 else Cbar
    if Lbar is None:
        Lbar = torch.empty_like(L)
    _call(H, "gpc_trsm_adjoint", GPC_TRANS if trans else GPC_NOTRANS, n, C2.shape[1], _ptr(L), _square(L, "L"),
          _ptr(C2), _mat(C2, "C"), _ptr(Cb2), _mat(Cb2, "Cbar"), _ptr(Lbar), _square(Lbar, "Lbar"))
    return Lbar


def gemm(H: Handle, A: torch.Tensor, B: torch.Tensor, ta: bool = False, tb: bool = False, beta: float = 0.0,
         C: torch.Tensor | None = None) -> torch.Tensor:
    """C = op(A) op(B) + beta C (beta 0 or 1)."""
    M, K = (A.shape[1], A.shape[0]) if ta else A.shape
    N = B.shape[0] if tb else B.shape[1]
    if C is None:
        C = torch.empty((M, N), dtype=torch.float64, device=A.device)
    _call(H, "gpc_gemm", int(ta), int(tb), M, N, K, _ptr(A), _mat(A, "A"), _ptr(B), _mat(B, "B"), float(beta),
          _ptr(C), _mat(C, "C"))
    return C


def last_splits(H: Handle) -> int:
    s = _i32()
    H._check(lib().gpc_get_last_splits(H.h, ctypes.byref(s)), "gpc_get_last_splits")
    return s.value


def gemm_adjoint(H: Handle, A, B, Cbar, ta=False, tb=False, beta=0.0, Abar=None, Bbar=None,
                 want_a=True, want_b=True):
    M, K = (A.shape[1], A.shape[0]) if ta else A.shape
    N = B.shape[0] if tb else B.shape[1]
    if want_a and Abar is None:
        Abar = torch.empty_like(A)
    if want_b and Bbar is None:
        Bbar = torch.empty_like(B)
    _call(H, "gpc_gemm_adjoint", int(ta), int(tb), M, N, K, _ptr(A), _mat(A, "A"), _ptr(B), _mat(B, "B"),
          _ptr(Cbar), _mat(Cbar, "Cbar"), float(beta), _ptr(Abar if want_a else None),
          _mat(Abar, "Abar") if want_a else 1, _ptr(Bbar if want_b else None), _mat(Bbar, "Bbar") if want_b else 1)
    return (Abar if want_a else None), (Bbar if want_b else None)


def multiply_transpose(H: Handle, A: torch.Tensor, C: torch.Tensor | None = None) -> torch.Tensor:
    M, K = A.shape
    if C is None:
        C = torch.empty((M, M), dtype=torch.float64, device=A.device)
    _call(H, "gpc_multiply_transpose", M, K, _ptr(A), _mat(A, "A"), _ptr(C), _mat(C, "C"))
    return C


def multiply_transpose_adjoint(H: Handle, A, Cbar, beta=0.0, Abar=None):
    M, K = A.shape
    if Abar is None:
        Abar = torch.empty_like(A)
    _call(H, "gpc_multiply_transpose_adjoint", M, K, _ptr(A), _mat(A, "A"), _ptr(Cbar), _mat(Cbar, "Cbar"),
          float(beta), _ptr(Abar), _mat(Abar, "Abar"))
    return Abar


def glm_bernoulli_logit(H: Handle, X, y, alpha, beta, with_dX=False):
    """(lp, dalpha, dbeta, dX or None) as device tensors; y: int32 0/1."""
    n, k = X.shape
    if y.dtype != torch.int32:
        raise TypeError("y must be int32")
    if alpha.dtype != torch.float64 or beta.dtype != torch.float64:
        raise TypeError("alpha and beta must be float64")
    alpha = alpha.reshape(()).contiguous()
    beta = beta.contiguous()
    lp = torch.empty((), dtype=torch.float64, device=X.device)
    da = torch.empty((), dtype=torch.float64, device=X.device)
    db = torch.empty(k, dtype=torch.float64, device=X.device)
    dX = torch.empty_like(X) if with_dX else None
    _call(H, "gpc_glm_bernoulli_logit", n, k, _ptr(X), _mat(X, "X"), _ptr(y.contiguous()), _ptr(alpha),
          _ptr(beta), _ptr(lp), _ptr(da), _ptr(db), _ptr(dX), _mat(dX, "dX") if with_dX else 1)
    return lp, da, db, dX


class TriangularSolve(torch.autograd.Function):
    """apply(L, B, trans=False, handle=None) -> C = L^-1 B (or L^-T B); L lower
    (its strict upper part is not read and gets no gradient)."""

    @staticmethod
    def forward(ctx, L, B, trans=False, handle=None):
        H = _h(handle)
        C = B.detach().clone().contiguous()
        H.trsm(L.detach(), C, trans=trans)
        ctx.H, ctx.trans = H, trans
        ctx.save_for_backward(L.detach(), C)
        return C

    @staticmethod
    def backward(ctx, Cbar):
        L, C = ctx.saved_tensors
        Bbar = Cbar.detach().clone().contiguous()
        Lbar = trsm_adjoint(ctx.H, L, C, Bbar, trans=ctx.trans)
        return Lbar, Bbar, None, None


class LowerTriangularInverse(torch.autograd.Function):
    """apply(L, handle=None) -> X = L^-1 (lower)."""

    @staticmethod
    def forward(ctx, L, handle=None):
        H = _h(handle)
        X = trtri(H, L.detach())
        ctx.H = H
        ctx.save_for_backward(X)
        return X

    @staticmethod
    def backward(ctx, Xbar):
        (X,) = ctx.saved_tensors
        return trtri_adjoint(ctx.H, X, Xbar.detach().contiguous()), None


class MatMul(torch.autograd.Function):
    """apply(A, B, handle=None) -> A B."""

    @staticmethod
    def forward(ctx, A, B, handle=None):
        H = _h(handle)
        C = gemm(H, A.detach(), B.detach())
        ctx.H = H
        ctx.save_for_backward(A.detach(), B.detach())
        return C

    @staticmethod
    def backward(ctx, Cbar):
        A, B = ctx.saved_tensors
        Ab, Bb = gemm_adjoint(ctx.H, A, B, Cbar.detach().contiguous(),
                              want_a=ctx.needs_input_grad[0], want_b=ctx.needs_input_grad[1])
        return Ab, Bb, None


class MultiplyTranspose(torch.autograd.Function):
    """apply(A, handle=None) -> A A^T."""

    @staticmethod
    def forward(ctx, A, handle=None):
        H = _h(handle)
        C = multiply_transpose(H, A.detach())
        ctx.H = H
        ctx.save_for_backward(A.detach())
        return C

    @staticmethod
    def backward(ctx, Cbar):
        (A,) = ctx.saved_tensors
        return multiply_transpose_adjoint(ctx.H, A, Cbar.detach().contiguous()), None


class BernoulliLogitGLM(torch.autograd.Function):
    """apply(X, y, alpha, beta, handle=None) -> the log-likelihood
    sum_i y_i log s(X_i beta + alpha) + (1 - y_i) log(1 - s(X_i beta + alpha))
    (0-d tensor); gradients for X, alpha and beta (y is data)."""

    @staticmethod
    def forward(ctx, X, y, alpha, beta, handle=None):
        H = _h(handle)
        want_x = ctx.needs_input_grad[0]
        lp, da, db, dX = glm_bernoulli_logit(H, X.detach(), y, alpha.detach().reshape(()),
                                             beta.detach().contiguous(), with_dX=want_x)
        ctx.save_for_backward(da, db, dX if want_x else None)
        ctx.alpha_shape = alpha.shape
        return lp

    @staticmethod
    def backward(ctx, g):
        da, db, dX = ctx.saved_tensors
        g = g.detach()
        return (None if dX is None else g * dX), None, (g * da).reshape(ctx.alpha_shape), g * db, None
