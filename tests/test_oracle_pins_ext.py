"""Pins of the oracle's triangular inverse, triangular-solve and inverse
reverse modes (section 3.2), matrix products (section 3.1) and the
Bernoulli-logit GLM likelihood (section 3.4), against what mathematics and
independent libraries fix: residual identities, LAPACK through NumPy, torch-CPU
autograd, central finite differences, closed forms and exact integer cases."""
import math

import numpy as np
import pytest
import torch

import oracle


def lower(rng, n, diag=2.0):
    L = np.tril(rng.standard_normal((n, n)), -1) / math.sqrt(n)
    L[np.diag_indices(n)] = np.abs(rng.standard_normal(n)) + diag
    return L


# ---- lower-triangular inverse ----------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 7, 64, 131])
def test_trtri_residual_and_lapack(n):
    rng = np.random.default_rng(n)
    L = lower(rng, n)
    X = oracle.trtri(L)
    assert np.all(np.triu(X, 1) == 0.0)
    assert np.linalg.norm(L @ X - np.eye(n)) <= 1e-13 * math.sqrt(n)
    Xl = np.linalg.inv(L)
    assert np.linalg.norm(X - Xl) <= 1e-13 * np.linalg.norm(Xl)


def test_trtri_closed_forms():
    a, b, c = 2.0, 3.0, 5.0
    X = oracle.trtri(np.array([[a, 0.0], [b, c]]))
    assert np.array_equal(X, np.array([[1 / a, 0.0], [-b / (a * c), 1 / c]]))
    d = np.array([1.0, 4.0, 0.5, 8.0])
    assert np.array_equal(oracle.trtri(np.diag(d)), np.diag(1.0 / d))
    # unit bidiagonal with -1 below the diagonal: the inverse is all ones below
    n = 6
    B = np.eye(n) - np.eye(n, k=-1)
    assert np.array_equal(oracle.trtri(B), np.tril(np.ones((n, n))))


def test_trtri_ignores_upper_triangle():
    rng = np.random.default_rng(3)
    L = lower(rng, 20)
    G = L + np.triu(rng.standard_normal((20, 20)), 1) * 1e3
    assert np.array_equal(oracle.trtri(G), oracle.trtri(L))


# ---- reverse modes of the solve and of the inverse ---------------------------

def fd_lower(f, L, h=1e-6):
    """Central differences of f with respect to each lower entry of L."""
    n = L.shape[0]
    G = np.zeros_like(L)
    for i in range(n):
        for j in range(i + 1):
            Lp, Lm = L.copy(), L.copy()
            Lp[i, j] += h
            Lm[i, j] -= h
            G[i, j] = (f(Lp) - f(Lm)) / (2 * h)
    return G


@pytest.mark.parametrize("trans", [False, True])
@pytest.mark.parametrize("nrhs", [1, 3])
def test_trsm_adjoint_finite_differences(trans, nrhs):
    rng = np.random.default_rng(10 + nrhs + 2 * trans)
    n = 7
    L = lower(rng, n)
    B = rng.standard_normal((n, nrhs))
    Cbar = rng.standard_normal((n, nrhs))
    C = oracle.trsm(L, B, trans=trans)
    Bbar, Lbar = oracle.trsm_adjoint(L, C, Cbar, trans=trans)
    f = lambda LL, BB=B: float(np.sum(Cbar * oracle.trsm(LL, BB, trans=trans)))
    G = fd_lower(f, L)
    assert np.linalg.norm(Lbar - G) <= 1e-6 * np.linalg.norm(G)
    assert np.all(np.triu(Lbar, 1) == 0.0)
    GB = np.zeros_like(B)
    for i in range(n):
        for c in range(nrhs):
            Bp, Bm = B.copy(), B.copy()
            Bp[i, c] += 1e-6
            Bm[i, c] -= 1e-6
            GB[i, c] = (f(L, Bp) - f(L, Bm)) / 2e-6
    assert np.linalg.norm(Bbar - GB) <= 1e-6 * np.linalg.norm(GB)


@pytest.mark.parametrize("trans", [False, True])
def test_trsm_adjoint_torch_autograd(trans):
    rng = np.random.default_rng(21 + trans)
    n, nrhs = 40, 5
    L = lower(rng, n)
    B = rng.standard_normal((n, nrhs))
    Cbar = rng.standard_normal((n, nrhs))
    Lt = torch.tensor(L, requires_grad=True)
    Bt = torch.tensor(B, requires_grad=True)
    M = torch.tril(Lt)
    Ct = torch.linalg.solve_triangular(M.T if trans else M, Bt, upper=trans)
    (Ct * torch.tensor(Cbar)).sum().backward()
    C = oracle.trsm(L, B, trans=trans)
    Bbar, Lbar = oracle.trsm_adjoint(L, C, Cbar, trans=trans)
    assert np.linalg.norm(C - Ct.detach().numpy()) <= 1e-13 * np.linalg.norm(C)
    assert np.linalg.norm(Bbar - Bt.grad.numpy()) <= 1e-12 * np.linalg.norm(Bbar)
    assert np.linalg.norm(Lbar - np.tril(Lt.grad.numpy())) <= 1e-12 * np.linalg.norm(Lbar)


def test_trsm_adjoint_linear_in_seed():
    rng = np.random.default_rng(5)
    n = 30
    L = lower(rng, n)
    C = rng.standard_normal((n, 2))
    S1, S2 = rng.standard_normal((n, 2)), rng.standard_normal((n, 2))
    b1, l1 = oracle.trsm_adjoint(L, C, S1)
    b2, l2 = oracle.trsm_adjoint(L, C, S2)
    b3, l3 = oracle.trsm_adjoint(L, C, 2.0 * S1 - 3.0 * S2)
    assert np.allclose(b3, 2 * b1 - 3 * b2, rtol=0, atol=1e-12 * np.abs(b3).max())
    assert np.allclose(l3, 2 * l1 - 3 * l2, rtol=0, atol=1e-12 * np.abs(l3).max())


def test_trtri_adjoint_finite_differences_and_torch():
    rng = np.random.default_rng(31)
    n = 6
    L = lower(rng, n)
    Xbar = np.tril(rng.standard_normal((n, n)))
    X = oracle.trtri(L)
    Lbar = oracle.trtri_adjoint(X, Xbar)
    G = fd_lower(lambda LL: float(np.sum(Xbar * oracle.trtri(LL))), L)
    assert np.linalg.norm(Lbar - G) <= 1e-6 * np.linalg.norm(G)
    Lt = torch.tensor(L, requires_grad=True)
    (torch.linalg.inv(torch.tril(Lt)) * torch.tensor(Xbar)).sum().backward()
    assert np.linalg.norm(Lbar - np.tril(Lt.grad.numpy())) <= 1e-12 * np.linalg.norm(Lbar)


def test_trtri_adjoint_ignores_upper_seed_and_matches_solve_with_identity():
    rng = np.random.default_rng(32)
    n = 25
    L = lower(rng, n)
    X = oracle.trtri(L)
    Xbar = np.tril(rng.standard_normal((n, n)))
    full = Xbar + np.triu(rng.standard_normal((n, n)), 1)
    Lbar = oracle.trtri_adjoint(X, Xbar)
    assert np.array_equal(oracle.trtri_adjoint(X, full), Lbar)
    # the inverse is the solve with B = I: its reverse mode gives the same Lbar
    _, Lbar2 = oracle.trsm_adjoint(L, X, Xbar)
    assert np.linalg.norm(Lbar - Lbar2) <= 1e-12 * np.linalg.norm(Lbar)


# ---- matrix products ---------------------------------------------------------

@pytest.mark.parametrize("ta", [False, True])
@pytest.mark.parametrize("tb", [False, True])
def test_gemm_against_numpy(ta, tb):
    rng = np.random.default_rng(40 + 2 * ta + tb)
    M, N, K = 13, 9, 21
    A = rng.standard_normal((K, M) if ta else (M, K))
    B = rng.standard_normal((N, K) if tb else (K, N))
    C0 = rng.standard_normal((M, N))
    ref = (A.T if ta else A) @ (B.T if tb else B)
    assert np.allclose(oracle.gemm(A, B, ta, tb), ref, rtol=1e-14, atol=1e-13)
    assert np.allclose(oracle.gemm(A, B, ta, tb, beta=1.0, C=C0), ref + C0, rtol=1e-14, atol=1e-13)


def test_gemm_exact_on_integers_and_identity():
    rng = np.random.default_rng(44)
    A = rng.integers(-50, 50, size=(17, 33)).astype(np.float64)
    B = rng.integers(-50, 50, size=(33, 11)).astype(np.float64)
    assert np.array_equal(oracle.gemm(A, B), A @ B)          # integer sums are exact
    assert np.array_equal(oracle.gemm(A, np.eye(33)), A)
    assert np.array_equal(oracle.multiply_transpose(A), A @ A.T)


def test_multiply_transpose_symmetric():
    rng = np.random.default_rng(45)
    A = rng.standard_normal((30, 70))
    C = oracle.multiply_transpose(A)
    assert np.array_equal(C, C.T)
    assert np.allclose(C, A @ A.T, rtol=1e-13, atol=1e-12)


def test_gemm_reverse_mode_finite_differences():
    # the reverse mode of C = A B (section 3.1): Abar = Cbar B^T, Bbar = A^T Cbar
    rng = np.random.default_rng(46)
    A, B, Cb = rng.standard_normal((5, 4)), rng.standard_normal((4, 3)), rng.standard_normal((5, 3))
    Ab = oracle.gemm(Cb, B, tb=True)
    Bb = oracle.gemm(A, Cb, ta=True)
    f = lambda AA, BB: float(np.sum(Cb * oracle.gemm(AA, BB)))
    GA, GB = np.zeros_like(A), np.zeros_like(B)
    for idx in np.ndindex(A.shape):
        P, Q = A.copy(), A.copy()
        P[idx] += 1e-6
        Q[idx] -= 1e-6
        GA[idx] = (f(P, B) - f(Q, B)) / 2e-6
    for idx in np.ndindex(B.shape):
        P, Q = B.copy(), B.copy()
        P[idx] += 1e-6
        Q[idx] -= 1e-6
        GB[idx] = (f(A, P) - f(A, Q)) / 2e-6
    assert np.allclose(Ab, GA, atol=1e-8) and np.allclose(Bb, GB, atol=1e-8)


# ---- Bernoulli-logit GLM -------------------------------------------------------

def test_glm_closed_forms():
    # one observation with mu = log 3: s = 3/4
    lp, da, db, _ = oracle.glm_bernoulli_logit(np.zeros((1, 1)), np.array([1]), math.log(3.0), np.zeros(1))
    assert abs(lp - math.log(0.75)) <= 1e-15 and abs(da - 0.25) <= 1e-15
    lp, da, _, _ = oracle.glm_bernoulli_logit(np.zeros((1, 1)), np.array([0]), math.log(3.0), np.zeros(1))
    assert abs(lp - math.log(0.25)) <= 1e-15 and abs(da + 0.75) <= 1e-15
    # beta = 0, alpha = 0: every probability is 1/2
    rng = np.random.default_rng(50)
    X = rng.standard_normal((200, 6))
    y = (rng.random(200) < 0.3).astype(np.int32)
    lp, da, db, _ = oracle.glm_bernoulli_logit(X, y, 0.0, np.zeros(6))
    assert abs(lp + 200 * math.log(2.0)) <= 1e-12
    assert abs(da - float(np.sum(y - 0.5))) <= 1e-12
    assert np.allclose(db, X.T @ (y - 0.5), rtol=1e-13, atol=1e-12)


def test_glm_against_scipy_and_extremes():
    from scipy.special import expit, log_expit
    rng = np.random.default_rng(51)
    n, k = 500, 7
    X = rng.standard_normal((n, k))
    beta = rng.standard_normal(k)
    alpha = 0.3
    y = (rng.random(n) < 0.5).astype(np.int32)
    mu = alpha + X @ beta
    ref = float(np.sum(y * log_expit(mu) + (1 - y) * log_expit(-mu)))
    lp, da, db, dX = oracle.glm_bernoulli_logit(X, y, alpha, beta, with_dX=True)
    assert abs(lp - ref) <= 1e-12 * abs(ref)
    d = y - expit(mu)
    assert abs(da - d.sum()) <= 1e-12 * n
    assert np.allclose(db, X.T @ d, rtol=1e-12, atol=1e-11)
    assert np.allclose(dX, np.outer(d, beta), rtol=1e-13, atol=1e-14)
    # |mu| far beyond exp's range stays finite
    lp, da, _, _ = oracle.glm_bernoulli_logit(np.array([[1.0], [1.0]]), np.array([1, 0]), 0.0, np.array([800.0]))
    assert lp == -800.0 and da == -1.0


def test_glm_finite_differences():
    rng = np.random.default_rng(52)
    n, k = 40, 4
    X = rng.standard_normal((n, k))
    beta = rng.standard_normal(k)
    y = (rng.random(n) < 0.6).astype(np.int32)
    alpha = -0.7
    lp, da, db, dX = oracle.glm_bernoulli_logit(X, y, alpha, beta, with_dX=True)
    f = lambda XX, a, b: oracle.glm_bernoulli_logit(XX, y, a, b)[0]
    h = 1e-6
    assert abs((f(X, alpha + h, beta) - f(X, alpha - h, beta)) / (2 * h) - da) <= 1e-6 * max(1, abs(da))
    for j in range(k):
        bp, bm = beta.copy(), beta.copy()
        bp[j] += h
        bm[j] -= h
        assert abs((f(X, alpha, bp) - f(X, alpha, bm)) / (2 * h) - db[j]) <= 1e-6 * max(1, abs(db[j]))
    for (i, j) in [(0, 0), (7, 3), (39, 1)]:
        Xp, Xm = X.copy(), X.copy()
        Xp[i, j] += h
        Xm[i, j] -= h
        assert abs((f(Xp, alpha, beta) - f(Xm, alpha, beta)) / (2 * h) - dX[i, j]) <= 1e-6
