"""dht_apply_noalloc (fixed per-GPU scratch, no device allocation at call
time) against dht_apply, through the C ABI: two calls in a row, the second
with fewer right-hand sides, in FP64 and BF16; an input whose chunk exceeds
the scratch is rejected without enqueueing work.  Both entry points run the
same kernels on the same internal layout, so the results must agree exactly.
"""
import numpy as np
import pytest

from paper_1603_05988_amd.workloads import WORKLOADS, gauge_links, random_spinors

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _lib():
    from paper_1603_05988_amd import _lib as L
    return L


@pytest.mark.parametrize("wl,prec,sizes", [("c1", 0, (16, 3)), ("c2", 2, (32, 5)), ("c2", 0, (8, 1))])
def test_noalloc_apply_matches_apply(wl, prec, sizes):
    L = _lib()
    w = WORKLOADS[wl]
    U = gauge_links(w.L, w.eps, w.seed)
    ctx = L.Context(w.L, w.mass)
    ctx.set_gauge(torch.from_numpy(U).cuda())
    for i, n in enumerate(sizes):
        X = torch.from_numpy(random_spinors(w.L, n, 40 + i)).cuda()
        for op in (L.OP_D, L.OP_Q):
            ref = ctx.apply(X, op, prec)
            Y = torch.full_like(X, float("nan"))
            ctx.apply_noalloc(X, Y, op, prec)
            torch.cuda.synchronize()
            diff = (Y - ref).abs().max().item()
            assert diff == 0.0, (wl, prec, n, op, diff)
    ctx.close()


def test_noalloc_rejects_oversize():
    L = _lib()
    w = WORKLOADS["c2"]
    U = gauge_links(w.L, w.eps, w.seed)
    ctx = L.Context(w.L, w.mass)
    ctx.set_gauge(torch.from_numpy(U).cuda())
    n = 16   # 2 x 12 x 8192 x 16 x 16 bytes = 48 MiB > 32 MiB in FP64
    X = torch.from_numpy(random_spinors(w.L, n, 3)).cuda()
    Y = torch.zeros_like(X)
    with pytest.raises(L.DhtError):
        ctx.apply_noalloc(X, Y, L.OP_D, L.FP64)
    torch.cuda.synchronize()
    assert torch.count_nonzero(Y).item() == 0
    ctx.close()
