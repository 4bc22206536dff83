"""gpc_factor_noalloc (the factor for callers that cannot allocate) against
gpc_factor on the same inputs, through the C ABI: two calls in a row, the
second on a smaller matrix, each within the FP64 parity bound of gpc_factor's
result (the same blocked arithmetic, so in practice bit for bit), with the
same info.  A matrix that is not SPD reports the same failing column."""
import numpy as np
import pytest
import torch

import workloads as W
from gpu_util import TOL, dev, host, relf, say, with_upper_garbage

pytestmark = pytest.mark.gpu


def _pair(H, A):
    """(L, info) from gpc_factor and from gpc_factor_noalloc on copies of A."""
    Ar = dev(A)
    ir = H.factor(Ar)
    An = dev(A)
    inn = torch.full((), -7, dtype=torch.int32, device="cuda")
    H.factor_noalloc(An, inn)
    return host(Ar), int(host(ir)), host(An), int(host(inn))


def test_noalloc_factor_two_calls_second_smaller():
    from paper_1907_01063_amd import Handle
    H = Handle()
    H.set_options(block=0, lookahead=1)
    for n in (1500, 333):
        case = W.c3(n=n)
        A = with_upper_garbage(case["A"], seed=n)
        Lr, ir, Ln, inn = _pair(H, A)
        e = relf(Ln, Lr)
        say(f"noalloc factor n={n}: info {inn} (ref {ir}), rel err vs gpc_factor {e:.2e}, "
            f"bitwise {np.array_equal(Ln, Lr)}")
        assert inn == ir == 0
        assert e <= TOL
        assert np.all(np.triu(Ln, 1) == 0.0)


def test_noalloc_factor_block_512_and_not_spd():
    from paper_1907_01063_amd import Handle
    H = Handle()
    H.set_options(block=512, lookahead=1)
    case = W.c3(n=1100)
    Lr, ir, Ln, inn = _pair(H, case["A"])
    assert inn == ir == 0 and relf(Ln, Lr) <= TOL
    A = case["A"].copy()
    A[700, 700] = -1.0
    _, ir, _, inn = _pair(H, A)
    say(f"noalloc factor, pivot 700 negative: info {inn} (ref {ir})")
    assert inn == ir == 701


def test_noalloc_factor_rejects_mixed_and_empty_is_ok():
    from paper_1907_01063_amd import Handle, GPC_MIXED
    from paper_1907_01063_amd.gpchol import GpcError
    H = Handle()
    info = torch.full((), -7, dtype=torch.int32, device="cuda")
    H.factor_noalloc(torch.empty((0, 0), dtype=torch.float64, device="cuda"), info)
    assert int(host(info)) == 0
    H.set_options(precision=GPC_MIXED)
    with pytest.raises(GpcError):
        H.factor_noalloc(dev(W.c3(n=64)["A"]), info)
