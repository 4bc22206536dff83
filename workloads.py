"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws random numbers and assembles covariance matrices from
them; it holds none of the factorisation, adjoint, solve or GP-gradient
arithmetic, and neither the oracle nor the HIP library imports it.  Every
generator draws with ``numpy.random.default_rng(seed)`` in the order
points -> Lbar -> y -> (jitter), all in float64, so that the same seed gives the
same bytes on every machine.

Workloads (n is the matrix order):

* ``toeplitz``: the paper's Cholesky timing matrix (section 3.3.3),
  A_ij = n - |i - j| off the diagonal and A_ii = n^2.
* ``c1``: n = 256, x ~ U(-10, 10) in 1-D, squared-exponential (variance 1,
  lengthscale 1) plus 0.1 I  (the 1-D GP regression inputs of section 4.2).
* ``c2``: n = 4096, x ~ N(0, I_4), SE (variance 2, lengthscale 1.5) + 0.05 I.
* ``c3``: n = 16384, x ~ U([0, 50]^2), Matern-3/2 (variance 1, lengthscale 3)
  + 0.01 I, y ~ N(0, I).
* ``c4``: a batch of 512 matrices with n_b ~ U{32..1024}, x ~ N(0, I_3),
  lengthscale log-uniform on [0.3, 3], SE (variance 1) + 0.1 I, packed
  row-major with 256-byte aligned offsets.
* ``c5``: n = 30000 GP marginal-likelihood inputs, x ~ N(0, I_8), y ~ N(0, I),
  SE-ARD base hyperparameters (1, ell_d = 2, 0.1) and 100 jittered copies
  theta_e = theta_base * exp(0.1 xi_e), xi_e ~ N(0, I_10).
* ``tri``: a lower-triangular factor with diagonal |N(0,1)| + 1 and N(0, 1/n)
  entries below it, a right-hand side block B ~ N(0,1) and adjoint seeds
  ~ N(0,1) (triangular solve and inverse, and their reverse modes).
* ``gemm``: A, B and an output adjoint ~ N(0,1) of given shapes (matrix
  products and their reverse mode).
* ``glm``: the logistic-regression data of section 4.1: X ~ N(0,1) of n x k,
  mu_i = 3 X_i1 - 2 X_i2 + 1, y_i ~ Bernoulli(1 / (1 + exp(-mu_i))); the
  likelihood is evaluated at (alpha, beta) = (1, 3, -2, 0, ..., 0) + 0.1 xi.

Lbar, the adjoint fed to the reverse pass, has N(0, 1) entries on and below the
diagonal and zeros above it.
"""
from __future__ import annotations

import math

import numpy as np

SEEDS = {"toeplitz": 1000, "c1": 1001, "c2": 1002, "c3": 1003, "c4": 1004, "c5": 1005,
         "tri": 1006, "gemm": 1007, "glm": 1008}

_ROWS = 1024   # rows per chunk when assembling large covariances


def toeplitz(n: int) -> np.ndarray:
    i = np.arange(n, dtype=np.float64)
    A = n - np.abs(i[:, None] - i[None, :])
    A[np.diag_indices(n)] = float(n) * float(n)
    return A


def _sq_dist_rows(x: np.ndarray, r0: int, r1: int, scale=None) -> np.ndarray:
    """Squared distances between rows r0:r1 of x and all rows (exact per pair:
    sum over coordinates of the squared difference)."""
    xs = x if scale is None else x / scale
    diff = xs[r0:r1, None, :] - xs[None, :, :]
    return np.einsum("ijk,ijk->ij", diff, diff)


def se_cov(x: np.ndarray, variance: float, lengthscale, noise: float) -> np.ndarray:
    """variance * exp(-1/2 sum_d (x_id - x_jd)^2 / l_d^2) + noise * I (full matrix)."""
    n = x.shape[0]
    ls = np.broadcast_to(np.asarray(lengthscale, dtype=np.float64), (x.shape[1],))
    K = np.empty((n, n))
    for r0 in range(0, n, _ROWS):
        r1 = min(n, r0 + _ROWS)
        K[r0:r1] = variance * np.exp(-0.5 * _sq_dist_rows(x, r0, r1, ls))
    K[np.diag_indices(n)] += noise
    return K


def matern32_cov(x: np.ndarray, variance: float, lengthscale: float, noise: float) -> np.ndarray:
    """variance * (1 + sqrt(3) r / l) exp(-sqrt(3) r / l) + noise * I."""
    n = x.shape[0]
    K = np.empty((n, n))
    c = math.sqrt(3.0) / lengthscale
    for r0 in range(0, n, _ROWS):
        r1 = min(n, r0 + _ROWS)
        s = c * np.sqrt(_sq_dist_rows(x, r0, r1))
        K[r0:r1] = variance * (1.0 + s) * np.exp(-s)
    K[np.diag_indices(n)] += noise
    return K


def lower_normal(rng: np.random.Generator, n: int) -> np.ndarray:
    """N(0, 1) on and below the diagonal, zero above (drawn row by row)."""
    M = rng.standard_normal((n, n))
    return np.tril(M)


def toeplitz_case(n: int, seed: int = SEEDS["toeplitz"]) -> dict:
    rng = np.random.default_rng(seed)
    A = toeplitz(n)
    Lbar = lower_normal(rng, n)
    y = rng.standard_normal(n)
    return {"name": f"toeplitz-n{n}", "A": A, "Lbar": Lbar, "y": y}


def c1(seed: int = SEEDS["c1"], n: int = 256) -> dict:
    rng = np.random.default_rng(seed)
    x = rng.uniform(-10.0, 10.0, size=(n, 1))
    Lbar = lower_normal(rng, n)
    y = rng.standard_normal(n)
    A = se_cov(x, 1.0, 1.0, 0.1)
    return {"name": f"se1d-n{n}", "x": x, "A": A, "Lbar": Lbar, "y": y}


def c2(seed: int = SEEDS["c2"], n: int = 4096) -> dict:
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, 4))
    Lbar = lower_normal(rng, n)
    y = rng.standard_normal(n)
    A = se_cov(x, 2.0, 1.5, 0.05)
    return {"name": f"se4d-n{n}", "x": x, "A": A, "Lbar": Lbar, "y": y}


def c3(seed: int = SEEDS["c3"], n: int = 16384, with_lbar: bool = True) -> dict:
    """Matern-3/2 on 2-D points with the point density of the n = 16384 case:
    the square's side scales as 50 * sqrt(n / 16384), so a smaller n is a
    same-density sample of the full workload."""
    rng = np.random.default_rng(seed)
    side = 50.0 * math.sqrt(n / 16384.0)
    x = rng.uniform(0.0, side, size=(n, 2))
    Lbar = lower_normal(rng, n) if with_lbar else None
    y = rng.standard_normal(n)
    A = matern32_cov(x, 1.0, 3.0, 0.01)
    return {"name": f"matern32-2d-n{n}", "x": x, "A": A, "Lbar": Lbar, "y": y}


def matern_duplicates(n: int = 1024, dup: int = 64, noise: float = 1e-10, seed: int = SEEDS["c3"]) -> dict:
    """The n-point Matern-3/2 workload at the same point density, with points
    n/2 .. n/2 + dup - 1 copies of points 0 .. dup - 1 and a nugget of `noise`:
    each copied pair leaves a Schur-complement pivot of about `noise`, far
    below FP32 rounding of the trailing updates (about 6e-8 here) but well
    above FP64's, so the matrix is SPD in FP64 yet loses definiteness when its
    updates are done in FP32."""
    rng = np.random.default_rng(seed)
    side = 50.0 * math.sqrt(n / 16384.0)
    x = rng.uniform(0.0, side, size=(n, 2))
    h = n // 2
    x[h:h + dup] = x[:dup]
    return {"name": f"matern32-dup{dup}-n{n}", "x": x, "A": matern32_cov(x, 1.0, 3.0, noise)}


def c4(seed: int = SEEDS["c4"], count: int = 512, nmin: int = 32, nmax: int = 1024,
       with_lbar: bool = True) -> dict:
    """Batch of SE covariances of uneven order, packed row-major one after the
    other (each with leading dimension n_b), offsets aligned to 256 bytes."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(nmin, nmax + 1, size=count)
    offs = np.zeros(count, dtype=np.int64)
    pos = 0
    for b in range(count):
        offs[b] = pos
        pos += int(ns[b]) * int(ns[b])
        pos = (pos + 31) // 32 * 32          # 32 doubles = 256 bytes
    total = pos
    base = np.zeros(total)
    lbar = np.zeros(total) if with_lbar else None
    ells = np.empty(count)
    for b in range(count):
        n = int(ns[b])
        x = rng.standard_normal((n, 3))
        ell = math.exp(rng.uniform(math.log(0.3), math.log(3.0)))
        ells[b] = ell
        A = se_cov(x, 1.0, ell, 0.1)
        base[offs[b]:offs[b] + n * n] = A.reshape(-1)
        if with_lbar:
            lbar[offs[b]:offs[b] + n * n] = lower_normal(rng, n).reshape(-1)
    return {"name": f"se3d-batch{count}", "n": ns.astype(np.int32), "off": offs,
            "base": base, "Lbar": lbar, "ell": ells}


def c5(seed: int = SEEDS["c5"], n: int = 30000, evals: int = 100, d: int = 8) -> dict:
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, d))
    y = rng.standard_normal(n)
    base = np.concatenate([[1.0], np.full(d, 2.0), [0.1]])
    xi = rng.standard_normal((evals, d + 2))
    thetas = base[None, :] * np.exp(0.1 * xi)
    return {"name": f"se-ard{d}d-n{n}", "x": x, "y": y, "theta_base": base,
            "thetas": thetas}


def spd_from_factor(rng: np.random.Generator, n: int):
    """A = L0 L0^T for a random lower-triangular L0 with diagonal |N(0,1)| + 1 and
    N(0, 1/n) entries below it (scaled so that L0 stays well conditioned)."""
    L0 = np.tril(rng.standard_normal((n, n)), -1) / math.sqrt(max(n, 1))
    L0[np.diag_indices(n)] = np.abs(rng.standard_normal(n)) + 1.0
    return L0 @ L0.T, L0


def tri(n: int, nrhs: int = 1, seed: int = SEEDS["tri"]) -> dict:
    rng = np.random.default_rng(seed)
    L = np.tril(rng.standard_normal((n, n)), -1) / math.sqrt(max(n, 1))
    L[np.diag_indices(n)] = np.abs(rng.standard_normal(n)) + 1.0
    B = rng.standard_normal((n, nrhs))
    Cbar = rng.standard_normal((n, nrhs))
    Xbar = lower_normal(rng, n)
    return {"name": f"tri-n{n}-r{nrhs}", "L": L, "B": B, "Cbar": Cbar, "Xbar": Xbar}


def gemm_case(M: int, N: int, K: int, seed: int = SEEDS["gemm"]) -> dict:
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((M, K))
    B = rng.standard_normal((K, N))
    Cbar = rng.standard_normal((M, N))
    return {"name": f"gemm-{M}x{N}x{K}", "A": A, "B": B, "Cbar": Cbar}


def glm(n: int, k: int, seed: int = SEEDS["glm"]) -> dict:
    """Logistic-regression data (section 4.1) and one parameter point."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, k))
    mu = 3.0 * X[:, 0] - 2.0 * X[:, 1] + 1.0 if k >= 2 else X[:, 0] + 1.0
    y = (rng.random(n) < 1.0 / (1.0 + np.exp(-mu))).astype(np.int32)
    theta = np.zeros(k + 1)
    theta[0] = 1.0
    theta[1:3] = (3.0, -2.0)[:min(2, k)]
    theta += 0.1 * rng.standard_normal(k + 1)
    return {"name": f"glm-n{n}-k{k}", "X": X, "y": y, "alpha": float(theta[0]), "beta": theta[1:]}


def flops_factor(n: int) -> float:
    """LAPACK potrf convention: n^3/3 + n^2/2 + n/6."""
    return n ** 3 / 3.0 + n ** 2 / 2.0 + n / 6.0


def flops_adjoint(n: int) -> float:
    """Leading term of the blocked reverse sweep: 2 n^3 / 3."""
    return 2.0 * n ** 3 / 3.0
