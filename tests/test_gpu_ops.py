"""The operations beside the Cholesky path against the oracle: the
lower-triangular inverse and the reverse modes of the triangular solve and of
the inverse (section 3.2), general products, their reverse mode and A A^T
(section 3.1, including the split-K form of long inner dimensions), and the
Bernoulli-logit GLM likelihood and gradient (section 3.4); autograd through
each; full-size properties at the benchmark's shapes."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpu_util import TOL, dev, host, relf, say, with_upper_garbage

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    from paper_1907_01063_amd import Handle
    return Handle()


def ops():
    from paper_1907_01063_amd import ops as O
    return O


# ---- inverse ---------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 5, 127, 128, 129, 255, 300, 513, 1000, 2100])
def test_trtri_parity(H, n):
    c = W.tri(n)
    Lt = dev(with_upper_garbage(c["L"], seed=n))
    X = ops().trtri(H, Lt)
    Xo = oracle.trtri(c["L"])
    e = relf(host(X), Xo)
    say(f"trtri n={n}: {e:.2e}")
    assert e <= TOL
    assert np.all(np.triu(host(X), 1) == 0.0)


@pytest.mark.parametrize("n", [1, 100, 129, 300, 700])
def test_trtri_adjoint_parity(H, n):
    c = W.tri(n)
    Xo = oracle.trtri(c["L"])
    Lb = ops().trtri_adjoint(H, dev(Xo), dev(with_upper_garbage(c["Xbar"], seed=n + 1)))
    e = relf(host(Lb), oracle.trtri_adjoint(Xo, c["Xbar"]))
    say(f"trtri adjoint n={n}: {e:.2e}")
    assert e <= TOL
    assert np.all(np.triu(host(Lb), 1) == 0.0)


# ---- reverse mode of the solve ----------------------------------------------------

@pytest.mark.parametrize("trans", [False, True])
@pytest.mark.parametrize("n,nrhs", [(1, 1), (100, 1), (300, 3), (1000, 1), (1000, 40), (2100, 9)])
def test_trsm_adjoint_parity(H, trans, n, nrhs):
    c = W.tri(n, nrhs)
    C = oracle.trsm(c["L"], c["B"], trans=trans)
    Cb = dev(c["Cbar"])
    Lb = ops().trsm_adjoint(H, dev(with_upper_garbage(c["L"], seed=3)), dev(C), Cb, trans=trans)
    H.check()
    Bbo, Lbo = oracle.trsm_adjoint(c["L"], C, c["Cbar"], trans=trans)
    eb, el = relf(host(Cb), Bbo), relf(host(Lb), Lbo)
    say(f"trsm adjoint trans={trans} n={n} nrhs={nrhs}: Bbar {eb:.2e} Lbar {el:.2e}")
    assert eb <= TOL and el <= TOL
    assert np.all(np.triu(host(Lb), 1) == 0.0)


# ---- products ----------------------------------------------------------------------

@pytest.mark.parametrize("ta", [False, True])
@pytest.mark.parametrize("tb", [False, True])
@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (1, 300, 5), (257, 129, 1000), (130, 70, 0), (128, 128, 16)])
def test_gemm_parity(H, ta, tb, M, N, K):
    c = W.gemm_case(M, N, K)
    A = c["A"].T.copy() if ta else c["A"]
    B = c["B"].T.copy() if tb else c["B"]
    C0 = c["Cbar"]
    for beta in (0.0, 1.0):
        Ct = dev(C0)
        ops().gemm(H, dev(A), dev(B), ta, tb, beta, Ct)
        ref = oracle.gemm(A, B, ta, tb, beta, C0)
        e = relf(host(Ct), ref)
        assert e <= TOL, (beta, e)


def test_gemm_exact_on_integers(H):
    rng = np.random.default_rng(5)
    A = rng.integers(-64, 64, size=(300, 777)).astype(np.float64)
    B = rng.integers(-64, 64, size=(777, 200)).astype(np.float64)
    C = ops().gemm(H, dev(A), dev(B))
    assert np.array_equal(host(C), oracle.gemm(A, B))   # every partial sum is an exact integer


@pytest.mark.parametrize("ta,tb", [(False, False), (True, False), (False, True), (True, True)])
def test_gemm_split_k_long_inner_dimension(H, ta, tb):
    M, N, K = 96, 200, 60000
    c = W.gemm_case(M, N, K)
    A = c["A"].T.copy() if ta else c["A"]
    B = c["B"].T.copy() if tb else c["B"]
    Ct = ops().gemm(H, dev(A), dev(B), ta, tb)
    sp = ops().last_splits(H)
    C2 = ops().gemm(H, dev(A), dev(B), ta, tb)
    e = relf(host(Ct), oracle.gemm(A, B, ta, tb))
    say(f"gemm {M}x{N}x{K} ta={ta} tb={tb}: splits {sp}, err {e:.2e}")
    assert sp > 1
    assert e <= TOL
    assert torch.equal(Ct, C2)   # fixed-order sums: bit for bit


@pytest.mark.parametrize("ta", [False, True])
@pytest.mark.parametrize("tb", [False, True])
def test_gemm_adjoint_parity(H, ta, tb):
    M, N, K = 150, 90, 260
    c = W.gemm_case(M, N, K)
    A = c["A"].T.copy() if ta else c["A"]
    B = c["B"].T.copy() if tb else c["B"]
    Cb = c["Cbar"]
    Ab, Bb = ops().gemm_adjoint(H, dev(A), dev(B), dev(Cb), ta, tb)
    # d<Cbar, op(A) op(B)>/d op(A) = Cbar op(B)^T, mapped back through the transposes
    opB = B.T if tb else B
    opA = A.T if ta else A
    GA = oracle.gemm(Cb, np.ascontiguousarray(opB), tb=True)
    GB = oracle.gemm(np.ascontiguousarray(opA), Cb, ta=True)
    GA = GA.T if ta else GA
    GB = GB.T if tb else GB
    assert relf(host(Ab), GA) <= TOL and relf(host(Bb), GB) <= TOL


@pytest.mark.parametrize("M,K", [(1, 1), (129, 70), (300, 1000)])
def test_multiply_transpose_parity(H, M, K):
    A = W.gemm_case(M, 1, K)["A"]
    C = host(ops().multiply_transpose(H, dev(A)))
    assert np.array_equal(C, C.T)
    assert relf(C, oracle.multiply_transpose(A)) <= TOL
    Cb = W.gemm_case(M, M, 1)["Cbar"]
    Ab = host(ops().multiply_transpose_adjoint(H, dev(A), dev(Cb)))
    ref = oracle.gemm(Cb, A) + oracle.gemm(Cb, A, ta=True)
    assert relf(Ab, ref) <= TOL


# ---- GLM ------------------------------------------------------------------------------

def alpha_of(c):
    return torch.tensor(c["alpha"], dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("n,k", [(0, 5), (1, 1), (37, 3), (1000, 10), (333, 31), (5000, 100), (4001, 300),
                                 (777, 600), (3000, 2048), (2000, 3000)])
def test_glm_parity(H, n, k):
    c = W.glm(n, k)
    lp, da, db, dX = ops().glm_bernoulli_logit(H, dev(c["X"]), dev(c["y"]), alpha_of(c), dev(c["beta"]),
                                               with_dX=True)
    lpo, dao, dbo, dXo = oracle.glm_bernoulli_logit(c["X"], c["y"], c["alpha"], c["beta"], with_dX=True)
    got = float(host(lp))
    e_lp = abs(got - lpo) / max(abs(lpo), 1.0)
    e_da = abs(float(host(da)) - dao) / max(abs(dao), 1.0)
    e_db = relf(host(db), dbo) if k else 0.0
    e_dx = relf(host(dX), dXo) if n * k else 0.0
    say(f"glm n={n} k={k}: lp {e_lp:.2e} dalpha {e_da:.2e} dbeta {e_db:.2e} dX {e_dx:.2e}")
    assert max(e_lp, e_da, e_db, e_dx) <= TOL
    # bit-for-bit repetition (fixed reduction orders)
    lp2, _, db2, _ = ops().glm_bernoulli_logit(H, dev(c["X"]), dev(c["y"]), alpha_of(c), dev(c["beta"]))
    assert float(host(lp2)) == got and np.array_equal(host(db2), host(db))


def test_glm_full_size(H):
    c = W.glm(1 << 22, 10)
    Xt = dev(c["X"])
    lp, da, db, _ = ops().glm_bernoulli_logit(H, Xt, dev(c["y"]), alpha_of(c), dev(c["beta"]))
    lpo, dao, dbo, _ = oracle.glm_bernoulli_logit(c["X"], c["y"], c["alpha"], c["beta"])
    e = abs(float(host(lp)) - lpo) / abs(lpo)
    say(f"glm n=2^22 k=10: lp {e:.2e} dbeta {relf(host(db), dbo):.2e}")
    assert e <= TOL and relf(host(db), dbo) <= TOL and abs(float(host(da)) - dao) <= TOL * abs(dao) + 1e-9


# ---- autograd -------------------------------------------------------------------------

def test_autograd_gradcheck(H):
    from paper_1907_01063_amd.ops import (BernoulliLogitGLM, LowerTriangularInverse, MatMul, MultiplyTranspose,
                                          TriangularSolve)
    rng = np.random.default_rng(9)
    n = 12
    L = torch.tensor(W.tri(n)["L"], device="cuda", requires_grad=True)
    B = torch.tensor(rng.standard_normal((n, 3)), device="cuda", requires_grad=True)
    for trans in (False, True):
        # the strict upper part of L is not an input of the operation: test through tril
        assert torch.autograd.gradcheck(lambda l, b: TriangularSolve.apply(torch.tril(l), b, trans, H), (L, B))
    assert torch.autograd.gradcheck(lambda l: torch.tril(LowerTriangularInverse.apply(torch.tril(l), H)), (L,))
    A = torch.tensor(rng.standard_normal((7, 5)), device="cuda", requires_grad=True)
    Bm = torch.tensor(rng.standard_normal((5, 4)), device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(lambda a, b: MatMul.apply(a, b, H), (A, Bm))
    assert torch.autograd.gradcheck(lambda a: MultiplyTranspose.apply(a, H), (A,))
    c = W.glm(50, 4)
    X = torch.tensor(c["X"], device="cuda", requires_grad=True)
    y = torch.tensor(c["y"], device="cuda")
    al = torch.tensor([c["alpha"]], dtype=torch.float64, device="cuda", requires_grad=True)
    be = torch.tensor(c["beta"], device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(lambda x, a, b: BernoulliLogitGLM.apply(x, y, a, b, H), (X, al, be))


# ---- full size -------------------------------------------------------------------------

def test_trtri_full_size_columns(H):
    # n = 16384: L X = I on sampled columns (the oracle's inverse would take minutes)
    c = W.tri(16384)
    Lt = dev(c["L"])
    X = ops().trtri(H, Lt)
    cols = np.random.default_rng(3).choice(16384, size=8, replace=False)
    Xc = host(X[:, cols])
    R = c["L"] @ Xc
    R[cols, np.arange(8)] -= 1.0
    e = np.linalg.norm(R) / np.sqrt(8)
    say(f"trtri n=16384: |L X - I| on 8 columns {e:.2e}")
    assert e <= 1e-12
    assert np.all(np.triu(host(X[:2048, :2048]), 1) == 0.0)
