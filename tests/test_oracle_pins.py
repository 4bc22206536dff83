"""Pins of the CPU oracle against what the mathematics fixes (no GPU needed).

Each test checks the oracle against something other than itself: exact
constructions, closed forms, finite differences of an independent forward
(LAPACK through NumPy), torch-CPU autograd, the paper's blocked reverse sweep
re-derived in NumPy, and invariants.  A plausible slip in the oracle (a dropped
term, a wrong sign, a transposed operand, a missing halving of the diagonal)
fails at least one of them.
"""
import json
import math
import os

import numpy as np
import torch
import pytest
import scipy.linalg as sla

import oracle
import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def relf(a, b):
    d = np.linalg.norm(np.asarray(a) - np.asarray(b))
    s = np.linalg.norm(np.asarray(b))
    return d / s if s > 0 else d


def phi(M):
    """Lower triangle with the diagonal halved."""
    return np.tril(M) - 0.5 * np.diag(np.diag(M))


# ---------------------------------------------------------------- factor --

@pytest.mark.parametrize("n", [1, 2, 5, 33, 100])
def test_factor_recovers_constructed_factor(n):
    rng = np.random.default_rng(10 + n)
    A, L0 = W.spd_from_factor(rng, n)
    L, info = oracle.potrf(A)
    assert info == 0
    assert relf(L, L0) < 1e-12


def test_factor_golden_integer_case():
    fx = json.load(open(os.path.join(GOLD, "chol_int3.json")))
    Lx = np.array([[math.sqrt(3.0) if v == "sqrt3" else float(v) for v in r] for r in fx["L"]])
    L, info = oracle.potrf(np.array(fx["A"], dtype=float))
    assert info == 0
    assert np.max(np.abs(L - Lx)) < 1e-15 * 8


def test_factor_invariant_and_upper_zero():
    for case in (W.c1(), W.toeplitz_case(300)):
        A = case["A"]
        L, info = oracle.potrf(A)
        assert info == 0
        assert np.all(np.triu(L, 1) == 0.0)
        assert relf(L @ L.T, A) <= 1e-13


def test_factor_never_reads_upper():
    case = W.c1(n=64)
    A = case["A"].copy()
    L1, _ = oracle.potrf(A)
    A[np.triu_indices(64, 1)] = np.nan
    L2, info = oracle.potrf(A)
    assert info == 0
    assert np.array_equal(L1, L2)


def test_factor_matches_lapack():
    for case in (W.c1(), W.c3(n=512, with_lbar=False)):
        L, _ = oracle.potrf(case["A"])
        assert relf(L, np.linalg.cholesky(case["A"])) < 1e-13


def test_factor_closed_forms_small():
    rng = np.random.default_rng(3)
    for _ in range(20):
        a = rng.uniform(0.5, 3.0)
        b = rng.uniform(-1.0, 1.0)
        c = b * b / a + rng.uniform(0.1, 2.0)
        L, info = oracle.potrf(np.array([[a, b], [b, c]]))
        assert info == 0
        ref = np.array([[math.sqrt(a), 0.0], [b / math.sqrt(a), math.sqrt(c - b * b / a)]])
        assert np.max(np.abs(L - ref)) < 1e-14
    d = rng.uniform(0.1, 9.0, size=40)
    L, _ = oracle.potrf(np.diag(d))
    assert np.max(np.abs(L - np.diag(np.sqrt(d)))) == 0.0


def test_factor_info_codes():
    A = np.eye(8)
    A[3, 3] = -1.0
    assert oracle.potrf(A)[1] == 4
    assert oracle.potrf(np.array([[1.0, 2.0], [2.0, 1.0]]))[1] == 2
    A = np.eye(8)
    A[5, 5] = np.nan
    assert oracle.potrf(A)[1] == 6
    A = np.eye(8)
    A[6, 2] = np.nan           # poisons L_62, hence the pivot of column 6
    assert oracle.potrf(A)[1] == 7
    A = np.eye(5)
    A[0, 0] = 0.0
    assert oracle.potrf(A)[1] == 1
    assert oracle.potrf(np.zeros((0, 0)))[1] == 0


def test_factor_paper_toeplitz_is_spd():
    # section 3.3.3 matrix: diagonally dominant, so SPD
    L, info = oracle.potrf(W.toeplitz(200))
    assert info == 0
    assert relf(L @ L.T, W.toeplitz(200)) < 1e-15 * 200


# --------------------------------------------------------------- adjoint --

def _fd_adjoint(A, Lbar, h=1e-6):
    """Central differences of f(A) = <Lbar, chol(A)> over the lower entries,
    moving A_ij and A_ji together; forward by LAPACK (independent of the oracle)."""
    n = A.shape[0]
    G = np.zeros((n, n))
    for i in range(n):
        for j in range(i + 1):
            E = np.zeros((n, n))
            E[i, j] = E[j, i] = 1.0
            fp = np.sum(Lbar * np.linalg.cholesky(A + h * E))
            fm = np.sum(Lbar * np.linalg.cholesky(A - h * E))
            G[i, j] = (fp - fm) / (2 * h)
    return G


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
def test_adjoint_central_differences(n):
    rng = np.random.default_rng(100 + n)
    A, _ = W.spd_from_factor(rng, n)
    L, _ = oracle.potrf(A)
    Lbar = np.tril(rng.standard_normal((n, n)))
    Ab = oracle.potrf_adjoint(L, Lbar)
    assert np.all(np.triu(Ab, 1) == 0.0)
    assert relf(Ab, _fd_adjoint(A, Lbar)) <= 1e-6


def test_adjoint_golden_2x2():
    fx = json.load(open(os.path.join(GOLD, "adjoint_2x2.json")))
    Ab = oracle.potrf_adjoint(np.array(fx["L"], float), np.array(fx["Lbar"], float))
    assert np.max(np.abs(Ab - np.array(fx["Abar"]))) < 1e-15


def test_adjoint_closed_form_2x2_random():
    rng = np.random.default_rng(4)
    for _ in range(20):
        a = rng.uniform(0.5, 3.0)
        b = rng.uniform(-1.0, 1.0)
        c = b * b / a + rng.uniform(0.1, 2.0)
        l11, l21 = math.sqrt(a), b / math.sqrt(a)
        l22 = math.sqrt(c - b * b / a)
        Lb = np.tril(rng.standard_normal((2, 2)))
        ref = np.array([
            [Lb[0, 0] / (2 * l11) - Lb[1, 0] * b / (2 * a ** 1.5) + Lb[1, 1] * b * b / (2 * a * a * l22), 0.0],
            [Lb[1, 0] / l11 - Lb[1, 1] * b / (a * l22), Lb[1, 1] / (2 * l22)]])
        L = np.array([[l11, 0], [l21, l22]])
        assert np.max(np.abs(oracle.potrf_adjoint(L, Lb) - ref)) < 1e-13


def test_adjoint_identity_lbar_equals_l():
    # With Lbar held at L: <L, dL> = d tr(L L^T) / 2 = tr(dA) / 2, so the
    # gradient w.r.t. the lower entries is 1/2 on the diagonal and 0 below it.
    case = W.c1()
    L, _ = oracle.potrf(case["A"])
    Ab = oracle.potrf_adjoint(L, L)
    assert np.max(np.abs(Ab - 0.5 * np.eye(L.shape[0]))) < 1e-12


def test_adjoint_closed_form_inverse():
    # Lbar = diag(1/L_ii): f = sum log L_ii = log|A| / 2, gradient Phi(A^-1)
    case = W.c1(n=128)
    A = case["A"]
    L, _ = oracle.potrf(A)
    Ab = oracle.potrf_adjoint(L, np.diag(1.0 / np.diag(L)))
    assert relf(Ab, phi(np.linalg.inv(A))) < 1e-11


def test_adjoint_closed_form_diagonal_matrix():
    rng = np.random.default_rng(5)
    a = rng.uniform(0.2, 5.0, size=30)
    L = np.diag(np.sqrt(a))
    Lb = np.tril(rng.standard_normal((30, 30)))
    ref = Lb / np.sqrt(a)[None, :]
    ref[np.diag_indices(30)] = np.diag(Lb) / (2 * np.sqrt(a))
    assert np.max(np.abs(oracle.potrf_adjoint(L, Lb) - ref)) < 1e-15


def test_adjoint_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    case = W.c1(n=96)
    A, Lb = case["A"], case["Lbar"][:96, :96]
    At = torch.tensor(A, dtype=torch.float64, requires_grad=True)
    Lt = torch.linalg.cholesky(At)
    Lt.backward(torch.tensor(Lb))
    g = At.grad.numpy()
    mapped = 2.0 * np.tril(g) - np.diag(np.diag(g))
    L, _ = oracle.potrf(A)
    assert relf(oracle.potrf_adjoint(L, Lb), mapped) < 1e-11


def _chol_blocked(S, b):
    """Right-looking blocked factor of section 3.3.1 in torch-CPU ops: factor
    the leading diagonal block, solve the panel against it, then factor the
    Schur complement the same way (blocks of b columns)."""
    n = S.shape[0]
    k = min(b, n)
    L11 = torch.linalg.cholesky(S[:k, :k])
    if k == n:
        return L11
    L21 = torch.linalg.solve_triangular(L11, S[k:, :k].T, upper=False).T
    L22 = _chol_blocked(S[k:, k:] - L21 @ L21.T, b)
    top = torch.cat([L11, torch.zeros(k, n - k, dtype=S.dtype)], 1)
    return torch.cat([top, torch.cat([L21, L22], 1)], 0)


def _blocked_forward_gradient(A, Lbar, b):
    """A second derivation of the adjoint: torch autograd of the blocked
    forward factor, with the symmetric input built from its independent
    lower-triangle entries (so the gradient is taken with respect to them)."""
    T = torch.tensor(np.tril(A), requires_grad=True)
    S = torch.tril(T) + torch.tril(T, -1).T
    L = _chol_blocked(S, b)
    (torch.tensor(np.tril(Lbar)) * L).sum().backward()
    return np.tril(T.grad.numpy())


@pytest.mark.parametrize("b", [1, 2, 3, 7, 64, 100])
def test_adjoint_matches_autograd_of_blocked_factor(b):
    case = W.c1(n=100)
    L, _ = oracle.potrf(case["A"])
    Lb = case["Lbar"][:100, :100]
    assert relf(oracle.potrf_adjoint(L, Lb), _blocked_forward_gradient(case["A"], Lb, b)) < 1e-11


def test_adjoint_linear_in_lbar():
    rng = np.random.default_rng(6)
    A, _ = W.spd_from_factor(rng, 40)
    L, _ = oracle.potrf(A)
    L1 = np.tril(rng.standard_normal((40, 40)))
    L2 = np.tril(rng.standard_normal((40, 40)))
    lhs = oracle.potrf_adjoint(L, 2.5 * L1 - 0.75 * L2)
    rhs = 2.5 * oracle.potrf_adjoint(L, L1) - 0.75 * oracle.potrf_adjoint(L, L2)
    assert relf(lhs, rhs) < 1e-13


def test_adjoint_tangent_identity():
    # forward mode of the factor: dL = L * Phi(L^-1 dA L^-T); reverse mode must
    # satisfy <Lbar, dL> = sum_{i>=j} Abar_ij dA_ij for every symmetric dA.
    case = W.c3(n=300)
    A, Lb = case["A"], case["Lbar"]
    L, _ = oracle.potrf(A)
    Ab = oracle.potrf_adjoint(L, Lb)
    rng = np.random.default_rng(7)
    for _ in range(3):
        E = rng.standard_normal((300, 300))
        dA = E + E.T
        Li = sla.solve_triangular(L, np.eye(300), lower=True)
        dL = L @ phi(Li @ dA @ Li.T)
        lhs = np.sum(Lb * dL)
        rhs = np.sum(np.tril(Ab) * np.tril(dA))
        assert abs(lhs - rhs) <= 1e-10 * (abs(lhs) + np.linalg.norm(Lb) * np.linalg.norm(dL))


def test_referee_floor():
    case = W.c2(n=256)
    L, _ = oracle.potrf(case["A"])
    Lr, _ = oracle.potrf(case["A"], referee=True)
    assert relf(L, Lr) < 1e-13
    Lb = case["Lbar"][:256, :256]
    assert relf(oracle.potrf_adjoint(L, Lb), oracle.potrf_adjoint(Lr, Lb, referee=True)) < 1e-11


# ------------------------------------------------------- solves, log-det --

def test_trsm_against_scipy_and_residual():
    rng = np.random.default_rng(8)
    A, L0 = W.spd_from_factor(rng, 60)
    L, _ = oracle.potrf(A)
    B = rng.standard_normal((60, 3))
    X = oracle.trsm(L, B)
    assert relf(X, sla.solve_triangular(L, B, lower=True)) < 1e-13
    Y = oracle.trsm(L, B, trans=True)
    assert relf(Y, sla.solve_triangular(L.T, B, lower=False)) < 1e-13
    assert relf(L @ X, B) < 1e-14 and relf(L.T @ Y, B) < 1e-14
    d = rng.uniform(0.5, 2.0, size=10)
    v = rng.standard_normal(10)
    assert np.max(np.abs(oracle.trsm(np.diag(d), v) - v / d)) < 1e-15


def test_logdet_against_slogdet():
    for case in (W.c1(), W.toeplitz_case(100)):
        L, _ = oracle.potrf(case["A"])
        s, ld = np.linalg.slogdet(case["A"])
        assert s > 0 and abs(oracle.logdet(L) - ld) <= 1e-12 * abs(ld) + 1e-12


# --------------------------------------------------------------- GP ------

def test_kgen_special_values():
    x = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 2.0]])
    K = oracle.gp_kgen_se(x, 1.7, [0.5, 2.0], 0.3)
    assert np.all(np.triu(K, 1) == 0.0)
    assert np.allclose(np.diag(K), 1.7 + 0.3, rtol=0, atol=1e-15)
    assert abs(K[1, 0] - 1.7 * math.exp(-0.5 * 1.0 / 0.25)) < 1e-15
    assert abs(K[2, 0] - 1.7 * math.exp(-0.5 * 4.0 / 4.0)) < 1e-15
    assert abs(K[2, 1] - 1.7 * math.exp(-0.5 * (1.0 / 0.25 + 4.0 / 4.0))) < 1e-15


def _mll_numpy(x, y, theta):
    d = x.shape[1]
    K = W.se_cov(x, theta[0], theta[1:1 + d], theta[-1])
    s, ld = np.linalg.slogdet(K)
    return -0.5 * y @ np.linalg.solve(K, y) - 0.5 * ld


def _oracle_mll_grad(x, y, theta):
    d = x.shape[1]
    K = oracle.gp_kgen_se(x, theta[0], theta[1:1 + d], theta[-1])
    L, info = oracle.potrf(K)
    assert info == 0
    f, z, alpha, _ = oracle.gp_mll(L, y)
    Ab = oracle.potrf_adjoint(L, oracle.gp_lbar(L, alpha, z))
    Kfull = K + np.tril(K, -1).T          # the oracle writes the lower triangle only
    return f, oracle.gp_hypergrad_se(x, theta[0], theta[1:1 + d], Ab), Ab, Kfull, alpha


def test_gp_value_and_lbar():
    rng = np.random.default_rng(9)
    x = rng.standard_normal((40, 3))
    y = rng.standard_normal(40)
    theta = np.array([1.3, 0.8, 1.1, 2.0, 0.2])
    f, _, _, K, alpha = _oracle_mll_grad(x, y, theta)
    assert abs(f - _mll_numpy(x, y, theta)) < 1e-11 * max(1.0, abs(f))
    # Lbar by finite differences of f(L) = -1/2 |L^-1 y|^2 - sum log L_ii
    L = np.linalg.cholesky(K)
    def fL(L):
        z = sla.solve_triangular(L, y, lower=True)
        return -0.5 * z @ z - np.sum(np.log(np.diag(L)))
    z = sla.solve_triangular(L, y, lower=True)
    a = sla.solve_triangular(L.T, z, lower=False)
    Lb = oracle.gp_lbar(L, a, z)
    h = 1e-6
    for (i, j) in [(0, 0), (5, 2), (39, 39), (39, 0), (20, 19)]:
        E = np.zeros_like(L)
        E[i, j] = h
        fd = (fL(L + E) - fL(L - E)) / (2 * h)
        assert abs(fd - Lb[i, j]) < 1e-6 * max(1.0, abs(fd))
    assert np.all(np.triu(Lb, 1) == 0.0)


def test_gp_adjoint_closed_form():
    # GP adjoint equals Phi(alpha alpha^T - K^-1) (Rasmussen & Williams eq. 5.9)
    rng = np.random.default_rng(11)
    x = rng.standard_normal((80, 2))
    y = rng.standard_normal(80)
    theta = np.array([1.0, 1.2, 0.7, 0.1])
    _, _, Ab, K, alpha = _oracle_mll_grad(x, y, theta)
    ref = phi(np.outer(alpha, alpha) - np.linalg.inv(K))
    assert relf(Ab, ref) < 1e-10


def test_gp_hypergrad_fd_and_trace_form():
    rng = np.random.default_rng(12)
    x = rng.standard_normal((50, 3))
    y = rng.standard_normal(50)
    theta = np.array([1.4, 0.9, 1.6, 1.1, 0.15])
    _, g, _, K, alpha = _oracle_mll_grad(x, y, theta)
    h = 1e-6
    for q in range(len(theta)):
        tp, tm = theta.copy(), theta.copy()
        tp[q] += h
        tm[q] -= h
        fd = (_mll_numpy(x, y, tp) - _mll_numpy(x, y, tm)) / (2 * h)
        assert abs(fd - g[q]) < 1e-6 * max(1.0, abs(fd)), q
    # 1/2 tr((alpha alpha^T - K^-1) dK/dsigma2)
    Kse = W.se_cov(x, theta[0], theta[1:4], 0.0)
    Mm = np.outer(alpha, alpha) - np.linalg.inv(K)
    assert abs(0.5 * np.sum(Mm * (Kse / theta[0])) - g[0]) < 1e-10 * max(1.0, abs(g[0]))
    assert abs(0.5 * np.trace(Mm) - g[-1]) < 1e-10 * max(1.0, abs(g[-1]))
