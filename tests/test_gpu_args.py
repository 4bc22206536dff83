"""Argument checks that need a live handle (no kernel runs in these cases):
leading dimensions above 2^20 and outputs that overlap inputs are rejected
with GPC_ERR_ARG before anything is enqueued.  Every buffer is sized for the
leading dimension it is passed with, so even a missed check would stay in
bounds."""
import ctypes

import pytest
import torch

from gpu_util import say

pytestmark = pytest.mark.gpu

BIG = (1 << 20) + 1


@pytest.fixture(scope="module")
def H():
    from paper_1907_01063_amd import Handle
    return Handle()


def test_leading_dimension_above_limit_rejected(H):
    from paper_1907_01063_amd.gpchol import GPC_ERR_ARG, GPC_OK
    lib, h = H.lib, H.h
    A = torch.zeros(4 * BIG, dtype=torch.float64, device="cuda")   # 4 rows of BIG doubles
    Lb = torch.zeros(4 * BIG, dtype=torch.float64, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    y = torch.zeros(4 * BIG, dtype=torch.float64, device="cuda")
    H._sync_stream()
    assert lib.gpc_factor(h, 4, A.data_ptr(), BIG, info.data_ptr()) == GPC_ERR_ARG
    assert lib.gpc_adjoint(h, 4, A.data_ptr(), BIG, Lb.data_ptr(), 4) == GPC_ERR_ARG
    assert lib.gpc_adjoint(h, 4, A.data_ptr(), 4, Lb.data_ptr(), BIG) == GPC_ERR_ARG
    assert lib.gpc_trsm(h, 0, 4, 1, A.data_ptr(), BIG, y.data_ptr(), 1) == GPC_ERR_ARG
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    assert lib.gpc_logdet(h, 4, A.data_ptr(), BIG, out.data_ptr()) == GPC_ERR_ARG
    torch.cuda.synchronize()
    assert torch.count_nonzero(A).item() == 0 and int(info.item()) == 0   # nothing ran
    assert lib.gpc_check(h) == GPC_OK


def test_overlapping_outputs_rejected(H):
    from paper_1907_01063_amd.gpchol import GPC_ERR_ARG
    lib, h = H.lib, H.h
    n = 64
    L = torch.eye(n, dtype=torch.float64, device="cuda")
    big = torch.zeros(2 * n * n, dtype=torch.float64, device="cuda")
    H._sync_stream()
    # Lbar == L, and Lbar starting inside L
    assert lib.gpc_adjoint(h, n, L.data_ptr(), n, L.data_ptr(), n) == GPC_ERR_ARG
    assert lib.gpc_adjoint(h, n, big.data_ptr(), n, big.data_ptr() + 8 * (n * n - 1), n) == GPC_ERR_ARG
    # B overlapping L in a solve
    assert lib.gpc_trsm(h, 0, n, 1, L.data_ptr(), n, L.data_ptr() + 8 * n, 1) == GPC_ERR_ARG
    # refined solution overlapping y
    it = torch.zeros(1, dtype=torch.int32, device="cuda")
    eta = torch.zeros(1, dtype=torch.float64, device="cuda")
    v = torch.zeros(n, dtype=torch.float64, device="cuda")
    assert lib.gpc_solve_refined(h, n, L.data_ptr(), n, L.data_ptr(), n, v.data_ptr(), v.data_ptr(),
                                 it.data_ptr(), eta.data_ptr()) == GPC_ERR_ARG
    torch.cuda.synchronize()
    say("overlap checks ok")


def test_options_out_of_range_rejected(H):
    """gpc_set_options rejects every field outside its documented range with
    GPC_ERR_ARG and keeps the previous options; the ends of each range are
    accepted."""
    from paper_1907_01063_amd.gpchol import GPC_ERR_ARG, GpcError
    before = H.options()
    bad = [("precision", 2), ("block", 100), ("block", 1024), ("refine_maxit", -1), ("refine_tol", 0.0),
           ("mixed_fallback", 2), ("test_flags", 3), ("gemm_max_splits", -1), ("gemm_max_splits", 33),
           ("batched_schedule", 3), ("adjoint_group", -1), ("adjoint_group", 9)]
    for field, value in bad:
        with pytest.raises(GpcError) as ei:
            H.set_options(**{field: value})
        assert ei.value.status == GPC_ERR_ARG, field
        after = H.options()
        assert all(getattr(after, f) == getattr(before, f) for f, _ in after._fields_), field
    for field, value in [("adjoint_group", 8), ("adjoint_group", 1), ("adjoint_group", 0), ("block", 512),
                         ("gemm_max_splits", 32), ("batched_schedule", 2)]:
        H.set_options(**{field: value})
        assert getattr(H.options(), field) == value
    H.set_options(**{f: getattr(before, f) for f, _ in before._fields_})
    say("option range checks ok")
