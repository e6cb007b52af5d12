"""Host read-backs (tree header, walk state, list totals) go through a pinned
mailbox that a kernel writes after the work queued before it; the host polls
it for a bounded time and then blocks on the stream.  A read-back queued
behind tens of milliseconds of other work on the same stream takes that
blocking path, and the results stay the same bit for bit.
"""

import math
import time

import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SPIN_LIMIT_S = 0.020  # the library's polling limit before it blocks


def test_readback_behind_long_work_is_bitwise_equal():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2107_07166_amd import api
    from paper_2107_07166_amd.generators import WORKLOADS

    pos, m = WORKLOADS["plummer1m"].make(n=30000)
    pd = torch.from_numpy(pos).cuda()
    md = torch.from_numpy(m).cuda()
    kw = dict(p=4, theta=0.5, eps=1e-3, variant="conserving", precision="mixed32")
    ctx = api.Context(0)
    tree = api.Tree(ctx, pd, md, n_leaf=64)
    try:
        ref = tree.evaluate(**kw).clone()
        # unrelated work for at least three polling limits, on the same stream
        a = torch.rand(2048, 2048, device="cuda")
        b = torch.empty_like(a)
        torch.mm(a, a, out=b)  # library set-up outside the calibration
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(8):
            torch.mm(a, a, out=b)
        torch.cuda.synchronize()
        per = max((time.perf_counter() - t0) / 8, 1e-6)
        count = min(20000, math.ceil(3 * SPIN_LIMIT_S / per))
        t0 = time.perf_counter()
        for _ in range(count):
            torch.mm(a, a, out=b)
        tree.rebuild(pd, md)  # its header read-back waits behind the products
        f = tree.evaluate(**kw)
        torch.cuda.synchronize()
        waited = time.perf_counter() - t0
        assert waited > SPIN_LIMIT_S
        assert torch.equal(f, ref)
        # and the polling path again right after
        tree.rebuild(pd, md)
        assert torch.equal(tree.evaluate(**kw), ref)
    finally:
        tree.close()
        ctx.close()
