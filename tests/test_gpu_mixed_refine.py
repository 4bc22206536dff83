"""Mixed form (FP32 MFMA trailing updates, FP64 diagonal blocks and panels) and
FP64 iterative refinement, against the FP64 oracle.

The mixed factor and adjoint have no oracle of their own (parity unpinned):
their error against the FP64 oracle is reported and bounded by a budget
derived from the arithmetic: FP32 products carry unit roundoff 2^-24 = 6e-8
per trailing update, amplified by the conditioning of the matrix (about 1e3 to
1e4 here), so errors of order 1e-4 and below are expected; the tests allow
1e-3 (L) and 1e-2 (Abar).  The refined solve is pinned: its normwise backward
error must reach 1e-12 and its solution must match the oracle's FP64 solve to
the conditioning-limited accuracy.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpu_util import TOL, dev, host, relf, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    from paper_1907_01063_amd import Handle
    return Handle()


def mixed(H):
    from paper_1907_01063_amd import GPC_MIXED
    H.set_options(precision=GPC_MIXED)


def fp64(H):
    from paper_1907_01063_amd import GPC_FP64
    H.set_options(precision=GPC_FP64)


@pytest.mark.parametrize("n", [100, 129, 300, 700, 1000])
def test_mixed_factor_and_adjoint_error_budget(H, n):
    case = W.c3(n=n)
    say(f"mixed factor+adjoint n={n}")
    mixed(H)
    At = dev(case["A"])
    info = H.factor(At)
    Lbt = dev(case["Lbar"])
    H.adjoint(At, Lbt)
    fp64(H)
    Lo, _ = oracle.potrf(case["A"])
    Ao = oracle.potrf_adjoint(Lo, case["Lbar"])
    eL, eA = relf(host(At), Lo), relf(host(Lbt), Ao)
    say(f"  mixed n={n}: L err {eL:.2e}, Abar err {eA:.2e}")
    assert int(host(info)) == 0
    assert np.all(np.triu(host(At), 1) == 0.0) and np.all(np.triu(host(Lbt), 1) == 0.0)
    assert eL <= 1e-3 and eA <= 1e-2
    if n <= 128:          # a single diagonal block: no FP32 update at all
        assert eL <= TOL


@pytest.mark.parametrize("form", ["fp64", "mixed"])
@pytest.mark.parametrize("n", [257, 1000])
def test_refined_solve(H, form, n):
    case = W.c3(n=n)
    say(f"refine {form} n={n}")
    (mixed if form == "mixed" else fp64)(H)
    L = dev(case["A"])
    H.factor(L)
    fp64(H)
    K = dev(case["A"])
    y = dev(case["y"])
    x, iters, eta = H.solve_refined(K, L, y)
    it, e = int(host(iters)), float(host(eta))
    Lo, _ = oracle.potrf(case["A"])
    xo = oracle.trsm(Lo, oracle.trsm(Lo, case["y"]), trans=True)
    err = relf(host(x), xo)
    say(f"  {form}: iters {it}, eta {e:.2e}, |x - x_oracle|/|x_oracle| {err:.2e}")
    assert e <= 1e-12
    assert 1 <= it <= (2 if form == "fp64" else 6)
    # the oracle's own solve is exact up to cond * 1e-16; allow that slack
    assert err <= 1e-9


def test_refined_solve_reports_nonconvergence(H):
    from paper_1907_01063_amd.gpchol import GPC_ERR_REFINE, GpcError
    case = W.c3(n=300)
    mixed(H)
    L = dev(case["A"])
    H.factor(L)
    H.set_options(precision=0, refine_maxit=1, refine_tol=1e-300)
    try:
        with pytest.raises(GpcError) as ei:
            H.solve_refined(dev(case["A"]), L, dev(case["y"]))
        assert ei.value.status == GPC_ERR_REFINE
        x, iters, eta = H.solve_refined(dev(case["A"]), L, dev(case["y"]), check=False)
        assert int(host(iters)) == 1
        # after one step with the mixed factor the residual is far above
        # rounding, so eta (and the row sums of |K| it uses, formed in the
        # same pass as the residual) can be checked against its definition
        A, yv, xv = case["A"], case["y"], host(x)
        r = yv - A @ xv
        eta_h = np.abs(r).max() / (np.abs(A).sum(axis=1).max() * np.abs(xv).max() + np.abs(yv).max())
        assert eta_h > 1e-13
        assert abs(float(host(eta)) - eta_h) <= 1e-6 * eta_h
    finally:
        H.set_options(precision=0, refine_maxit=10, refine_tol=1e-12)


@pytest.mark.parametrize("n,group", [(400, 0), (1100, 1), (1100, 2), (2600, 4)])
def test_mixed_adjoint_given_factor_matches_fp64_closely(H, n, group):
    # the mixed adjoint only rounds its two trailing products to FP32; at
    # n = 1100 (five 256-blocks) and 2600 (eleven) the Bbar updates of a group
    # of steps share products whose FP32 panel copies share one buffer
    rng = np.random.default_rng(33)
    _, L0 = W.spd_from_factor(rng, n)
    Lb = W.lower_normal(rng, n)
    mixed(H)
    H.set_options(adjoint_group=group)
    try:
        Lbt = dev(Lb)
        H.adjoint(dev(L0), Lbt)
    finally:
        H.set_options(adjoint_group=0)
        fp64(H)
    e = relf(host(Lbt), oracle.potrf_adjoint(L0, Lb))
    say(f"mixed adjoint given factor n={n} group={group}: {e:.2e}")
    assert e <= 1e-4


def test_mixed_fallback_to_fp64():
    """FP32 trailing updates lose definiteness on copied points with a tiny
    nugget; the mixed factor then redoes the factorisation in FP64 (flag set),
    giving exactly the FP64 path's L."""
    from paper_1907_01063_amd import GPC_FP64, GPC_MIXED, Handle
    case = W.matern_duplicates(1024, 64, 1e-10)
    A = case["A"]
    assert oracle.potrf(A)[1] == 0                      # SPD in FP64
    say("mixed fallback n=1024")
    Hm = Handle()
    Hm.set_options(precision=GPC_MIXED, mixed_fallback=0)
    At = dev(A)
    info = int(host(Hm.factor(At)))
    assert info != 0 and not Hm.fell_back()              # the FP32 form really breaks down
    Hm.set_options(mixed_fallback=1)
    At = dev(A)
    info = int(host(Hm.factor(At)))
    assert info == 0 and Hm.fell_back()
    Hd = Handle()
    Hd.set_options(precision=GPC_FP64)
    Ad = dev(A)
    assert int(host(Hd.factor(Ad))) == 0
    assert torch.equal(At, Ad)
    L = host(At)
    rows = np.arange(0, 1024, 37)
    assert np.linalg.norm(L[rows] @ L.T - A[rows]) / np.linalg.norm(A[rows]) <= 1e-13


def test_mixed_no_fallback_when_definite(H):
    case = W.c3(n=700)
    mixed(H)
    try:
        At = dev(case["A"])
        assert int(host(H.factor(At))) == 0
        assert not H.fell_back()
    finally:
        fp64(H)
    Lo, _ = oracle.potrf(case["A"])
    e = relf(host(At), Lo)
    assert 0.0 < e <= 1e-3                               # the FP32 result, not a silent FP64 redo
