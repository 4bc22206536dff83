"""GP marginal log-likelihood as a torch.autograd.Function over the library.

f(theta) = -1/2 y^T K^-1 y - 1/2 log|K|   (the constant -n/2 log 2 pi omitted)
with K the squared-exponential ARD covariance of X plus noise,
theta = (s2, l_1..l_d, sn2).  Forward: K -> factor L -> z, alpha, log|K| -> f.
Backward: Lbar = tril(alpha z^T) - diag(1/L_ii) -> Abar (reverse-mode adjoint of
the factor, section 3.3.2) -> df/dtheta.  In the mixed form (FP32 trailing
updates) alpha comes from FP64 iterative refinement against K and
z = L^T alpha, f = -1/2 y^T alpha - 1/2 log|K|: the data term and its
gradient carry FP64 accuracy, the log-determinant term the mixed factor's.  Every step runs in the library's HIP
kernels; this module only moves tensors between the calls.
"""
from __future__ import annotations

import torch

from .gpchol import GPC_FP64, GPC_MIXED, GpcError, Handle, default_handle


class NotPositiveDefiniteError(ValueError):
    def __init__(self, col: int):
        super().__init__(f"covariance is not positive definite (first failing column {col})")
        self.col = col


def _factor(H: Handle, X, theta, precision):
    K = H.gp_kgen_se(X, theta)
    H.set_options(precision=precision)
    info = H.factor(K)
    return K, info


class GPMarginalLogLik(torch.autograd.Function):
    """apply(X, y, theta, precision=GPC_FP64, recompute_L=False, handle=None, check=True) -> f

    recompute_L: do not keep L between forward and backward; refactor it
    (same kernels, same inputs, so the gradient is bitwise the same).
    check: read the factor's info flag (one device sync) and raise
    NotPositiveDefiniteError on failure; in the mixed form a lost pivot first
    makes the covariance be generated again and factored in FP64 (backward
    then uses FP64 too).  Also raises GpcError if a solve sweep ran out of
    time.
    """

    @staticmethod
    def forward(ctx, X, y, theta, precision=GPC_FP64, recompute_L=False, handle=None, check=True):
        H = handle or default_handle(X.device)
        X = X.detach().contiguous()
        y = y.detach().contiguous()
        th = theta.detach().contiguous()
        L, info = _factor(H, X, th, precision)
        if check:
            col = int(info.item())
            if col != 0 and precision == GPC_MIXED:
                # the FP32-updated Schur complement lost definiteness: the
                # covariance is generated again and factored in FP64
                precision = GPC_FP64
                L, info = _factor(H, X, th, precision)
                col = int(info.item())
            if col != 0:
                raise NotPositiveDefiniteError(col)
        if precision == GPC_MIXED:
            # alpha by FP64 refinement against the covariance (generated
            # again: the factor overwrote the first copy), z = L^T alpha
            K = H.gp_kgen_se(X, th)
            f, z, alpha, _, _, _ = H.gp_value_refined(K, L, y, check=check)
            del K
        else:
            f, z, alpha, _ = H.gp_value(L, y)
        if check:
            H.check()   # raises if a solve sweep ran out of time
        ctx.H, ctx.precision, ctx.recompute = H, precision, recompute_L
        ctx.save_for_backward(X, th, z, alpha, None if recompute_L else L)
        return f

    @staticmethod
    def backward(ctx, grad_f):
        X, th, z, alpha, L = ctx.saved_tensors
        H = ctx.H
        if L is None:
            L, _ = _factor(H, X, th, ctx.precision)
        H.set_options(precision=ctx.precision)
        Lbar = H.gp_lbar(L, alpha, z)
        H.adjoint(L, Lbar)
        g = H.gp_hypergrad_se(X, th, Lbar, scale=grad_f.detach().to(torch.float64).contiguous())
        return None, None, g, None, None, None, None


def gp_mll(X, y, theta, precision=GPC_FP64, recompute_L=False, handle=None, check=True):
    return GPMarginalLogLik.apply(X, y, theta, precision, recompute_L, handle, check)
