"""Batched path, both schedules (persistent: one workgroup per matrix in one
launch; grouped: every block step one launch over all members), graph
replayed: against the oracle per matrix, with results that must not depend
on queue order or on replay."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpu_util import TOL, host, relf, say

pytestmark = pytest.mark.gpu

SIZES = [1, 5, 31, 32, 33, 63, 64, 65, 100, 128, 129, 200, 257, 300, 0, 17]


@pytest.fixture(scope="module", params=[1, 2], ids=["persistent", "grouped"])
def H(request):
    from paper_1907_01063_amd import Handle
    h = Handle()
    h.set_options(batched_schedule=request.param)
    return h


def pack(mats, align=32):
    offs, pos = [], 0
    for M in mats:
        offs.append(pos)
        pos += M.size
        pos = (pos + align - 1) // align * align
    base = np.zeros(max(pos, 1))
    for M, o in zip(mats, offs):
        base[o:o + M.size] = M.reshape(-1)
    return base, np.array(offs, dtype=np.int64)


def unpack(base, n, off):
    return [base[o:o + k * k].reshape(k, k) for k, o in zip(n, off)]


def make_batch(seed, sizes):
    rng = np.random.default_rng(seed)
    As, Lbs = [], []
    for k in sizes:
        x = rng.standard_normal((k, 3))
        As.append(W.se_cov(x, 1.0, float(rng.uniform(0.5, 2.0)), 0.1) if k else np.zeros((0, 0)))
        Lbs.append(W.lower_normal(rng, k) if k else np.zeros((0, 0)))
    return As, Lbs


def run(H, As, Lbs, sizes):
    a, off = pack(As)
    lb, _ = pack(Lbs)
    at = torch.from_numpy(a).cuda()
    lbt = torch.from_numpy(lb).cuda()
    info = H.factor_adjoint_batched(sizes, off, at, lbt)
    return unpack(host(at), sizes, off), unpack(host(lbt), sizes, off), host(info)


def test_batched_parity(H):
    As, Lbs = make_batch(1, SIZES)
    say("batched parity")
    Ls, Abs, info = run(H, As, Lbs, SIZES)
    assert np.all(info == 0)
    for k, A, Lb, Lg, Ag in zip(SIZES, As, Lbs, Ls, Abs):
        if k == 0:
            continue
        Lo, _ = oracle.potrf(A)
        Ao = oracle.potrf_adjoint(Lo, Lb)
        assert np.all(np.triu(Lg, 1) == 0) and np.all(np.triu(Ag, 1) == 0)
        assert relf(Lg, Lo) <= TOL, k
        assert relf(Ag, Ao) <= TOL, k


def test_batched_parity_long_members(H):
    """Members of 10 to 16 block steps of 64: the grouped factor's step pairs
    (odd and even step counts, ragged last blocks) and the zero fills forked
    part-way through the factor, against the oracle per matrix."""
    sizes = [1000, 700, 129, 1024, 641, 64]
    As, Lbs = make_batch(7, sizes)
    say("batched parity, long members")
    Ls, Abs, info = run(H, As, Lbs, sizes)
    assert np.all(info == 0)
    for k, A, Lb, Lg, Ag in zip(sizes, As, Lbs, Ls, Abs):
        Lo, _ = oracle.potrf(A)
        Ao = oracle.potrf_adjoint(Lo, Lb)
        assert np.all(np.triu(Lg, 1) == 0) and np.all(np.triu(Ag, 1) == 0)
        assert relf(Lg, Lo) <= TOL, k
        assert relf(Ag, Ao) <= TOL, k


def test_batched_separate_calls_and_replay(H):
    As, Lbs = make_batch(2, SIZES[:8])
    a, off = pack(As)
    lb, _ = pack(Lbs)
    outs = []
    for rep in range(3):   # first call builds the plan and graph, later ones replay it
        at = torch.from_numpy(a).cuda()
        lbt = torch.from_numpy(lb).cuda()
        info = H.factor_batched(SIZES[:8], off, at)
        H.adjoint_batched(SIZES[:8], off, at, lbt)
        outs.append((host(at), host(lbt), host(info)))
    for o in outs[1:]:
        assert all(np.array_equal(x, y) for x, y in zip(outs[0], o))
    Ls = unpack(outs[0][0], SIZES[:8], off)
    for k, A, Lg in zip(SIZES[:8], As, Ls):
        assert relf(Lg, oracle.potrf(A)[0]) <= TOL


def test_batched_result_independent_of_queue_order(H):
    As, Lbs = make_batch(3, SIZES)
    Ls1, Ab1, _ = run(H, As, Lbs, SIZES)
    perm = np.random.default_rng(0).permutation(len(SIZES))
    Ls2, Ab2, _ = run(H, [As[i] for i in perm], [Lbs[i] for i in perm], [SIZES[i] for i in perm])
    for pos, i in enumerate(perm):
        assert np.array_equal(Ls2[pos], Ls1[i]) and np.array_equal(Ab2[pos], Ab1[i])


def test_batched_info_per_matrix(H):
    sizes = [40, 90, 150]
    As, Lbs = make_batch(4, sizes)
    As[1] = As[1].copy()
    As[1][70, 70] = -5.0
    a, off = pack(As)
    at = torch.from_numpy(a).cuda()
    info = host(H.factor_batched(sizes, off, at))
    assert list(info) == [0, oracle.potrf(As[1])[1], 0]


def test_autotune_then_parity(H, tmp_path):
    say("autotune")
    path = str(tmp_path / "tune.txt")
    H.autotune_batched(path)
    blocks, tuned = H.tuning()
    say(f"tuned blocks {blocks}")
    assert tuned and all(b in (32, 64) for b in blocks)
    assert len(open(path).read().strip().splitlines()) == 5
    As, Lbs = make_batch(5, SIZES)
    Ls, Abs, info = run(H, As, Lbs, SIZES)
    for k, A, Lb, Lg, Ag in zip(SIZES, As, Lbs, Ls, Abs):
        if k:
            Lo, _ = oracle.potrf(A)
            assert relf(Lg, Lo) <= TOL and relf(Ag, oracle.potrf_adjoint(Lo, Lb)) <= TOL


def test_full_size_batch_sampled(H):
    case = W.c4()
    say("c4 full batch")
    at = torch.from_numpy(case["base"]).cuda()
    lbt = torch.from_numpy(case["Lbar"]).cuda()
    info = host(H.factor_adjoint_batched(case["n"], case["off"], at, lbt))
    assert np.all(info == 0)
    a, lb = host(at), host(lbt)
    rng = np.random.default_rng(1)
    for b in rng.choice(len(case["n"]), size=12, replace=False):
        k, o = int(case["n"][b]), int(case["off"][b])
        A = case["base"][o:o + k * k].reshape(k, k)
        Lb = case["Lbar"][o:o + k * k].reshape(k, k)
        Lo, _ = oracle.potrf(A)
        assert relf(a[o:o + k * k].reshape(k, k), Lo) <= TOL
        assert relf(lb[o:o + k * k].reshape(k, k), oracle.potrf_adjoint(Lo, Lb)) <= TOL


@pytest.mark.parametrize("schedule", [1, 2], ids=["persistent", "grouped"])
def test_batched_mixed_form(schedule):
    """GPC_MIXED batch: FP32 trailing / B-bar / R-bar products.  No oracle of
    its own (parity unpinned): error against the FP64 oracle within the mixed
    budget of the single-matrix tests (L 1e-3, Abar 1e-2), nonzero (the FP32
    products really ran) for matrices beyond one inner block, queue-order
    independent, and bitwise stable across graph replays."""
    from paper_1907_01063_amd import GPC_MIXED, Handle
    Hm = Handle()
    Hm.set_options(precision=GPC_MIXED, batched_schedule=schedule)
    As, Lbs = make_batch(6, SIZES)
    say("batched mixed")
    Ls, Abs, info = run(Hm, As, Lbs, SIZES)
    assert np.all(info == 0)
    for k, A, Lb, Lg, Ag in zip(SIZES, As, Lbs, Ls, Abs):
        if k == 0:
            continue
        Lo, _ = oracle.potrf(A)
        Ao = oracle.potrf_adjoint(Lo, Lb)
        eL, eA = relf(Lg, Lo), relf(Ag, Ao)
        assert np.all(np.triu(Lg, 1) == 0) and np.all(np.triu(Ag, 1) == 0)
        assert eL <= 1e-3 and eA <= 1e-2, (k, eL, eA)
        if k > 64:
            assert eL > 1e-12, k
    Ls2, Ab2, _ = run(Hm, As, Lbs, SIZES)
    assert all(np.array_equal(x, y) for x, y in zip(Ls, Ls2))
    assert all(np.array_equal(x, y) for x, y in zip(Abs, Ab2))
    perm = np.random.default_rng(2).permutation(len(SIZES))
    Ls3, Ab3, _ = run(Hm, [As[i] for i in perm], [Lbs[i] for i in perm], [SIZES[i] for i in perm])
    for pos, i in enumerate(perm):
        assert np.array_equal(Ls3[pos], Ls[i]) and np.array_equal(Ab3[pos], Abs[i])


@pytest.mark.parametrize("schedule", [1, 2], ids=["persistent", "grouped"])
def test_batched_recorded_into_caller_graph(schedule):
    """A batched call inside the caller's graph capture: refused (nothing
    enqueued, the capture stays usable) when its plan was not prepared by the
    same call outside the capture; recorded when it was.  The caller's graph
    is replayed three times, with eager work and synchronisations between the
    replays, each replay bitwise equal to the eager call."""
    from paper_1907_01063_amd import GpcError, Handle
    from paper_1907_01063_amd.gpchol import GPC_ERR_CAPTURE
    Hc = Handle()
    Hc.set_options(batched_schedule=schedule)
    sizes = SIZES[:8]
    As, Lbs = make_batch(7, sizes)
    a, off = pack(As)
    lb, _ = pack(Lbs)
    a0, lb0 = torch.from_numpy(a).cuda(), torch.from_numpy(lb).cuda()
    at, lbt = a0.clone(), lb0.clone()
    info = torch.zeros(len(sizes), dtype=torch.int32, device="cuda")
    Hc.factor_adjoint_batched(sizes, off, at, lbt, info)   # prepares the plan
    ref_l, ref_a = host(at).copy(), host(lbt).copy()
    at.copy_(a0)
    lbt.copy_(lb0)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    refused = None
    with torch.cuda.graph(g, stream=cap):
        try:
            Hc.factor_adjoint_batched(sizes[:5], off[:5], at, lbt, info)   # no plan for these sizes
        except GpcError as e:
            refused = e.status
        Hc.factor_adjoint_batched(sizes, off, at, lbt, info)
    assert refused == GPC_ERR_CAPTURE
    for rep in range(3):
        at.copy_(a0)
        lbt.copy_(lb0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(at), ref_l) and np.array_equal(host(lbt), ref_a), rep
        assert int(info.max().item()) == 0
    del g
