"""NumPy front end of the plain CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product library never imports this
package, and this package imports nothing from the product.

Every function takes and returns float64 NumPy arrays in row-major order; only
the lower triangle of symmetric inputs is read.  The arithmetic lives in C (see
``oracle.c`` for the definitions and the paper passages they follow).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_i64 = ctypes.c_int64
_dp = ctypes.POINTER(ctypes.c_double)


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` (gcc, -O2, OpenMP, no BLAS)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
             _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        lib.orc_potrf.restype = ctypes.c_int
        lib.orc_potrf.argtypes = [_i64, _dp, _i64, _dp, _i64]
        lib.orc_potrf_ref.restype = ctypes.c_int
        lib.orc_potrf_ref.argtypes = [_i64, _dp, _i64, _dp, _i64]
        for f in (lib.orc_potrf_adjoint, lib.orc_potrf_adjoint_ref):
            f.restype = None
            f.argtypes = [_i64, _dp, _i64, _dp, _i64, _dp, _i64]
        lib.orc_trsm.restype = None
        lib.orc_trsm.argtypes = [ctypes.c_int, _i64, _i64, _dp, _i64, _dp, _i64]
        lib.orc_logdet.restype = ctypes.c_double
        lib.orc_logdet.argtypes = [_i64, _dp, _i64]
        lib.orc_gp_kgen_se.restype = None
        lib.orc_gp_kgen_se.argtypes = [_i64, _i64, _dp, ctypes.c_double, _dp,
                                       ctypes.c_double, _dp, _i64]
        lib.orc_gp_lbar.restype = None
        lib.orc_gp_lbar.argtypes = [_i64, _dp, _i64, _dp, _dp, _dp, _i64]
        lib.orc_trtri.restype = None
        lib.orc_trtri.argtypes = [_i64, _dp, _i64, _dp, _i64]
        lib.orc_trsm_adjoint.restype = None
        lib.orc_trsm_adjoint.argtypes = [ctypes.c_int, _i64, _i64, _dp, _i64, _dp, _i64, _dp, _i64,
                                         _dp, _i64, _dp, _i64]
        lib.orc_trtri_adjoint.restype = None
        lib.orc_trtri_adjoint.argtypes = [_i64, _dp, _i64, _dp, _i64, _dp, _i64]
        lib.orc_gemm.restype = None
        lib.orc_gemm.argtypes = [ctypes.c_int, ctypes.c_int, _i64, _i64, _i64, _dp, _i64, _dp, _i64,
                                 ctypes.c_double, _dp, _i64]
        lib.orc_multiply_transpose.restype = None
        lib.orc_multiply_transpose.argtypes = [_i64, _i64, _dp, _i64, _dp, _i64]
        lib.orc_glm_bernoulli_logit.restype = None
        lib.orc_glm_bernoulli_logit.argtypes = [_i64, _i64, _dp, _i64, ctypes.POINTER(ctypes.c_int32),
                                                ctypes.c_double, _dp, _dp, _dp, _dp, _dp, _i64]
        lib.orc_max_threads.restype = ctypes.c_int
        lib.orc_max_threads.argtypes = []
        lib.orc_set_threads.restype = None
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        lib.orc_gp_hypergrad_se.restype = None
        lib.orc_gp_hypergrad_se.argtypes = [_i64, _i64, _dp, ctypes.c_double, _dp,
                                            _dp, _i64, _dp]
        _lib = lib
    return _lib


def threads() -> int:
    """Threads the oracle's parallel loops use (OpenMP)."""
    return int(_load().orc_max_threads())


def set_threads(t: int) -> None:
    """Set the oracle's thread count (its results do not depend on it)."""
    _load().orc_set_threads(int(t))


def _c(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def potrf(A: np.ndarray, referee: bool = False):
    """Cholesky factor of the SPD matrix whose lower triangle is in ``A``.

    Returns ``(L, info)``: ``info`` is 0, or j+1 for the first column j whose
    pivot is not positive (L is then unspecified from column j on).
    """
    A = _c(A)
    n = A.shape[0]
    L = np.zeros((n, n))
    f = _load().orc_potrf_ref if referee else _load().orc_potrf
    info = f(n, _p(A), n, _p(L), n)
    return L, int(info)


def potrf_adjoint(L: np.ndarray, Lbar: np.ndarray, referee: bool = False) -> np.ndarray:
    """Adjoint Abar (lower triangle, independent-entry convention) of the factor."""
    L = _c(L)
    Lbar = _c(Lbar)
    n = L.shape[0]
    Abar = np.zeros((n, n))
    f = _load().orc_potrf_adjoint_ref if referee else _load().orc_potrf_adjoint
    f(n, _p(L), n, _p(Lbar), n, _p(Abar), n)
    return Abar


def trsm(L: np.ndarray, B: np.ndarray, trans: bool = False) -> np.ndarray:
    """``L^-1 B`` (trans False) or ``L^-T B`` (trans True); B is n or n x nrhs."""
    L = _c(L)
    vec = B.ndim == 1
    X = _c(B.reshape(B.shape[0], -1)).copy()
    n, nrhs = X.shape
    _load().orc_trsm(1 if trans else 0, n, nrhs, _p(L), n, _p(X), nrhs)
    return X[:, 0].copy() if vec else X


def logdet(L: np.ndarray) -> float:
    L = _c(L)
    return float(_load().orc_logdet(L.shape[0], _p(L), L.shape[0]))


def gp_kgen_se(X: np.ndarray, sigma2: float, ell, noise: float) -> np.ndarray:
    X = _c(X)
    n, d = X.shape
    ell = _c(np.asarray(ell, dtype=np.float64).reshape(d))
    K = np.zeros((n, n))
    _load().orc_gp_kgen_se(n, d, _p(X), float(sigma2), _p(ell), float(noise), _p(K), n)
    return K


def gp_lbar(L: np.ndarray, alpha: np.ndarray, z: np.ndarray) -> np.ndarray:
    L = _c(L)
    alpha = _c(alpha)
    z = _c(z)
    n = L.shape[0]
    Lbar = np.zeros((n, n))
    _load().orc_gp_lbar(n, _p(L), n, _p(alpha), _p(z), _p(Lbar), n)
    return Lbar


def gp_hypergrad_se(X: np.ndarray, sigma2: float, ell, Abar: np.ndarray) -> np.ndarray:
    X = _c(X)
    n, d = X.shape
    ell = _c(np.asarray(ell, dtype=np.float64).reshape(d))
    Abar = _c(Abar)
    g = np.zeros(d + 2)
    _load().orc_gp_hypergrad_se(n, d, _p(X), float(sigma2), _p(ell), _p(Abar), n, _p(g))
    return g


def gp_mll(L: np.ndarray, y: np.ndarray):
    """Value pieces of the GP log-density: returns (f, z, alpha, logdet) with
    f = -1/2 z^T z - 1/2 log|K| (the constant -n/2 log 2 pi left out)."""
    z = trsm(L, y, trans=False)
    alpha = trsm(L, z, trans=True)
    ld = logdet(L)
    zz = 0.0
    for v in z:          # fixed order, i increasing
        zz += float(v) * float(v)
    return -0.5 * zz - 0.5 * ld, z, alpha, ld


def trtri(L: np.ndarray) -> np.ndarray:
    """``L^-1`` of a lower-triangular L (lower, strict upper zero)."""
    L = _c(L)
    n = L.shape[0]
    X = np.zeros((n, n))
    _load().orc_trtri(n, _p(L), n, _p(X), n)
    return X


def trsm_adjoint(L: np.ndarray, C: np.ndarray, Cbar: np.ndarray, trans: bool = False):
    """Adjoints of C = L^-1 B (or L^-T B): returns (Bbar, Lbar)."""
    L = _c(L)
    vec = C.ndim == 1
    C2 = _c(C.reshape(C.shape[0], -1))
    Cb2 = _c(Cbar.reshape(Cbar.shape[0], -1))
    n, nrhs = C2.shape
    Bbar = np.zeros((n, nrhs))
    Lbar = np.zeros((n, n))
    _load().orc_trsm_adjoint(1 if trans else 0, n, nrhs, _p(L), n, _p(C2), nrhs, _p(Cb2), nrhs,
                             _p(Bbar), nrhs, _p(Lbar), n)
    return (Bbar[:, 0].copy() if vec else Bbar), Lbar


def trtri_adjoint(X: np.ndarray, Xbar: np.ndarray) -> np.ndarray:
    """Lbar of X = L^-1 given the adjoint Xbar of its lower triangle."""
    X = _c(X)
    Xbar = _c(Xbar)
    n = X.shape[0]
    Lbar = np.zeros((n, n))
    _load().orc_trtri_adjoint(n, _p(X), n, _p(Xbar), n, _p(Lbar), n)
    return Lbar


def gemm(A: np.ndarray, B: np.ndarray, ta: bool = False, tb: bool = False, beta: float = 0.0,
         C: np.ndarray | None = None) -> np.ndarray:
    """``op(A) op(B) + beta C``."""
    A = _c(A)
    B = _c(B)
    M, K = (A.shape[1], A.shape[0]) if ta else A.shape
    N = B.shape[0] if tb else B.shape[1]
    out = np.zeros((M, N)) if C is None else _c(C).copy()
    _load().orc_gemm(1 if ta else 0, 1 if tb else 0, M, N, K, _p(A), A.shape[1], _p(B), B.shape[1],
                     float(beta), _p(out), N)
    return out


def multiply_transpose(A: np.ndarray) -> np.ndarray:
    """``A A^T`` (full symmetric)."""
    A = _c(A)
    M, K = A.shape
    C = np.zeros((M, M))
    _load().orc_multiply_transpose(M, K, _p(A), K, _p(C), M)
    return C


def glm_bernoulli_logit(X: np.ndarray, y: np.ndarray, alpha: float, beta: np.ndarray, with_dX: bool = False):
    """Bernoulli-logit GLM: returns (lp, dalpha, dbeta, dX or None)."""
    X = _c(X)
    n, k = X.shape
    yi = np.ascontiguousarray(y, dtype=np.int32)
    beta = _c(np.asarray(beta).reshape(k))
    lp, da = ctypes.c_double(), ctypes.c_double()
    db = np.zeros(k)
    dX = np.zeros((n, k)) if with_dX else None
    _load().orc_glm_bernoulli_logit(n, k, _p(X), k, yi.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                    float(alpha), _p(beta), ctypes.byref(lp), ctypes.byref(da), _p(db),
                                    _p(dX) if with_dX else None, k)
    return lp.value, da.value, db, dX
