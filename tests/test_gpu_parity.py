"""Parity of the HIP path (through the C ABI) with the CPU oracle, FP64.

Bar: relative Frobenius error <= 1e-11 for L, Abar, solves and log-det; the
strict upper triangle of every triangular output is exactly zero; info codes
equal the oracle's.  Sizes span one and several 128-blocks with ragged tails;
non-default block sizes exercise more block steps on the same inputs.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpu_util import TOL, dev, host, relf, say, with_upper_garbage

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 3, 17, 31, 64, 127, 128, 129, 200, 255, 256, 257, 383, 511, 700, 1000]


@pytest.fixture(scope="module")
def H():
    from paper_1907_01063_amd import Handle
    return Handle()


def _case(kind, n):
    if kind == "matern":
        return W.c3(n=n)
    if kind == "toeplitz":
        return W.toeplitz_case(n)
    return W.c1(n=n)


def gpu_factor(H, A, block=0):
    H.set_options(block=block)
    At = dev(with_upper_garbage(A))
    info = H.factor(At)
    return host(At), int(host(info))


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("kind", ["se1d", "matern"])
def test_factor_parity(H, kind, n):
    case = _case(kind, n)
    say(f"factor {kind} n={n}")
    Lg, info = gpu_factor(H, case["A"])
    Lo, info_o = oracle.potrf(case["A"])
    assert info == info_o == 0
    assert np.all(np.triu(Lg, 1) == 0.0)
    assert relf(Lg, Lo) <= TOL


@pytest.mark.parametrize("block", [32, 64])
@pytest.mark.parametrize("n", [97, 300, 513])
def test_factor_parity_small_blocks(H, block, n):
    case = W.c3(n=n)
    say(f"factor block={block} n={n}")
    Lg, info = gpu_factor(H, case["A"], block=block)
    H.set_options(block=0)
    Lo, _ = oracle.potrf(case["A"])
    assert info == 0
    assert relf(Lg, Lo) <= TOL


def test_factor_paper_toeplitz(H):
    case = W.toeplitz_case(1000)
    say("factor toeplitz n=1000")
    Lg, info = gpu_factor(H, case["A"])
    Lo, _ = oracle.potrf(case["A"])
    assert info == 0 and relf(Lg, Lo) <= TOL


def test_factor_n0(H):
    A = torch.zeros((0, 0), dtype=torch.float64, device="cuda")
    info = H.factor(A)
    assert int(host(info)) == 0


@pytest.mark.parametrize("bad", [0, 5, 127, 128, 129, 250, 299])
def test_factor_info_matches_oracle(H, bad):
    A = W.c3(n=300)["A"].copy()
    A[bad, bad] = -1.0 if bad % 2 else np.nan
    say(f"info bad={bad}")
    _, info = gpu_factor(H, A)
    _, info_o = oracle.potrf(A)
    assert info == info_o == bad + 1


def test_factor_info_indefinite_schur(H):
    # positive diagonal, but the Schur complement loses definiteness at column 200
    rng = np.random.default_rng(21)
    A, L0 = W.spd_from_factor(rng, 260)
    v = L0[200, :200].copy()
    A[200, 200] = float(v @ v) - 0.5
    say("info schur")
    _, info = gpu_factor(H, A)
    _, info_o = oracle.potrf(A)
    assert info == info_o == 201


@pytest.mark.parametrize("n", SIZES)
def test_adjoint_parity_given_factor(H, n):
    rng = np.random.default_rng(500 + n)
    _, L0 = W.spd_from_factor(rng, n)
    Lb = W.lower_normal(rng, n)
    say(f"adjoint n={n}")
    Lt = dev(with_upper_garbage(L0, 1))
    Lbt = dev(with_upper_garbage(Lb, 2))
    H.adjoint(Lt, Lbt)
    Ag = host(Lbt)
    Ao = oracle.potrf_adjoint(L0, Lb)
    assert np.all(np.triu(Ag, 1) == 0.0)
    assert np.array_equal(np.tril(host(Lt)), L0)          # L not modified
    assert relf(Ag, Ao) <= TOL


@pytest.mark.parametrize("block", [32, 64])
def test_adjoint_parity_small_blocks(H, block):
    case = W.c3(n=333)
    L, _ = oracle.potrf(case["A"])
    H.set_options(block=block)
    say(f"adjoint block={block}")
    Lbt = dev(case["Lbar"])
    H.adjoint(dev(L), Lbt)
    H.set_options(block=0)
    assert relf(host(Lbt), oracle.potrf_adjoint(L, case["Lbar"])) <= TOL


@pytest.mark.parametrize("kind,n", [("se1d", 256), ("matern", 1000), ("toeplitz", 700)])
def test_factor_then_adjoint_parity(H, kind, n):
    case = _case(kind, n)
    say(f"factor+adjoint {kind} n={n}")
    At = dev(case["A"])
    info = H.factor(At)
    Lbt = dev(case["Lbar"])
    H.adjoint(At, Lbt)
    Lo, _ = oracle.potrf(case["A"])
    Ao = oracle.potrf_adjoint(Lo, case["Lbar"])
    assert int(host(info)) == 0
    assert relf(host(At), Lo) <= TOL
    assert relf(host(Lbt), Ao) <= TOL


# n = 511 / 512 / 513 / 767 / 1000: both sides of the switch from 128- to
# 256-row sweep blocks, full and ragged last blocks; nrhs 1 takes the
# one-launch sweep, 3 and 9 the column-group launches (9: a group of 8, then
# its last column through the one-launch sweep)
@pytest.mark.parametrize("n", [1, 5, 128, 129, 300, 511, 512, 513, 767, 1000])
@pytest.mark.parametrize("nrhs", [1, 3, 9])
def test_trsm_parity(H, n, nrhs):
    rng = np.random.default_rng(700 + n + nrhs)
    _, L0 = W.spd_from_factor(rng, n)
    B = rng.standard_normal((n, nrhs))
    say(f"trsm n={n} nrhs={nrhs}")
    Lt = dev(with_upper_garbage(L0, 3))
    for trans in (False, True):
        Bt = dev(B)
        H.trsm(Lt, Bt, trans=trans)
        assert relf(host(Bt), oracle.trsm(L0, B, trans=trans)) <= TOL


# one-launch sweep: a column of a wider matrix (leading dimension 5) at sizes
# with several blocks and a ragged last block; repeated calls agree bit for bit
@pytest.mark.parametrize("n", [2000, 4100])
def test_trsm_one_column_strided_repeatable(H, n):
    rng = np.random.default_rng(900 + n)
    _, L0 = W.spd_from_factor(rng, n)
    B = rng.standard_normal((n, 5))
    say(f"trsm one column n={n}")
    Lt = dev(L0)
    for trans in (False, True):
        outs = []
        for _ in range(2):
            Bt = dev(B)
            H.trsm(Lt, Bt[:, 2:3], trans=trans)
            outs.append(host(Bt))
        assert np.array_equal(outs[0], outs[1])
        assert np.array_equal(np.delete(outs[0], 2, axis=1), np.delete(B, 2, axis=1))   # other columns untouched
        assert relf(outs[0][:, 2:3], oracle.trsm(L0, B[:, 2:3], trans=trans)) <= TOL
        assert not np.isnan(outs[0]).any()


def test_one_launch_sweep_failure_path(H):
    """The one-launch sweep's failure path, forced from the host: with its
    error flag raised before it starts, every wait returns at once and the
    one-column solve completes with NaN entries; column-group solves are not
    affected; clearing the flag restores normal results."""
    from paper_1907_01063_amd.gpchol import GPC_ERR_ARG, GpcError
    rng = np.random.default_rng(77)
    n = 1500
    _, L0 = W.spd_from_factor(rng, n)
    B = rng.standard_normal((n, 3))
    Lt = dev(L0)
    with pytest.raises(GpcError) as ei:
        H.set_options(test_flags=2)
    assert ei.value.status == GPC_ERR_ARG
    from paper_1907_01063_amd.gpchol import GPC_ERR_SWEEP
    H.check()   # no failure recorded so far
    H.set_options(test_flags=1)
    try:
        for trans in (False, True):
            z = dev(B[:, :1])
            H.trsm(Lt, z, trans=trans)
            assert np.isnan(host(z)).all()
            with pytest.raises(GpcError) as ei:   # the failure is reported once, then cleared
                H.check()
            assert ei.value.status == GPC_ERR_SWEEP
            H.check()
        Z3 = dev(B)
        H.trsm(Lt, Z3)
        assert relf(host(Z3), oracle.trsm(L0, B)) <= TOL
    finally:
        H.set_options(test_flags=0)
    z = dev(B[:, :1])
    H.trsm(Lt, z)
    assert relf(host(z), oracle.trsm(L0, B[:, :1])) <= TOL
    H.check()


def test_trsm_vector_and_logdet(H):
    case = W.c3(n=777)
    Lo, _ = oracle.potrf(case["A"])
    Lt = dev(Lo)
    z = dev(case["y"])
    H.trsm(Lt, z)
    zo = oracle.trsm(Lo, case["y"])
    assert relf(host(z), zo) <= TOL
    a = z.clone()
    H.trsm(Lt, a, trans=True)
    assert relf(host(a), oracle.trsm(Lo, zo, trans=True)) <= TOL
    ld = float(host(H.logdet(Lt)))
    assert abs(ld - oracle.logdet(Lo)) <= TOL * abs(oracle.logdet(Lo))


@pytest.mark.parametrize("block,look", [(128, 0), (128, 1), (256, 0), (256, 1), (512, 0), (512, 1)])
@pytest.mark.parametrize("n", [300, 400, 1100, 1700])
def test_blocking_and_lookahead_variants(H, block, look, n):
    # n = 300 / 400: ragged last 256-block with <= 128 / > 128 rows;
    # 1100 / 1700: several outer steps, so the lookahead schedule is exercised
    case = W.c3(n=n)
    say(f"variant block={block} lookahead={look} n={n}")
    H.set_options(block=block, lookahead=look)
    try:
        At = dev(with_upper_garbage(case["A"]))
        info = H.factor(At)
        Lbt = dev(with_upper_garbage(case["Lbar"], 5))
        H.adjoint(At, Lbt)
        Lg, Ag = host(At), host(Lbt)
    finally:
        H.set_options(block=0, lookahead=1)
    Lo, _ = oracle.potrf(case["A"])
    Ao = oracle.potrf_adjoint(Lo, case["Lbar"])
    assert int(host(info)) == 0
    assert np.all(np.triu(Lg, 1) == 0.0) and np.all(np.triu(Ag, 1) == 0.0)
    assert relf(Lg, Lo) <= TOL
    assert relf(Ag, Ao) <= TOL


@pytest.mark.parametrize("group,look", [(1, 1), (2, 1), (3, 0), (3, 1), (4, 0), (4, 1), (8, 1)])
@pytest.mark.parametrize("n", [1000, 1100, 1537, 2048, 2600])
def test_adjoint_step_groups(H, group, look, n):
    """Bbar updates of `group` reverse-sweep steps applied together (products
    of inner dimension up to group x 256 with a staircase of k limits; 1 = one
    product per step), with and without lookahead.  n spans 4 to 11
    256-blocks, whole and partial groups, a ragged last block of one row and
    none."""
    rng = np.random.default_rng(900 + n)
    _, L0 = W.spd_from_factor(rng, n)
    Lb = W.lower_normal(rng, n)
    say(f"adjoint group={group} lookahead={look} n={n}")
    H.set_options(adjoint_group=group, lookahead=look)
    try:
        Lbt = dev(with_upper_garbage(Lb, 3))
        H.adjoint(dev(L0), Lbt)
        Ag = host(Lbt)
    finally:
        H.set_options(adjoint_group=0, lookahead=1)
    assert np.all(np.triu(Ag, 1) == 0.0)
    assert relf(Ag, oracle.potrf_adjoint(L0, Lb)) <= TOL


def test_info_with_lookahead(H):
    # failure in a late outer step while the big updates run on the side stream
    A = W.c3(n=1300)["A"].copy()
    A[1100, 1100] = -1.0
    say("info lookahead")
    _, info = gpu_factor(H, A)
    assert info == oracle.potrf(A)[1] == 1101
