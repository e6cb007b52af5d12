"""The allocation-free diagnostics entry point (tfmm_momentum_diagnostics_noalloc)
against the allocating one, through the C ABI: two calls in a row, the second
with a smaller input; the context holds no more device memory after them;
sizes beyond the limit are refused before any device work."""

import ctypes

import numpy as np
import pytest

from paper_2107_07166_amd.generators import plummer

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def test_noalloc_diagnostics_match_the_allocating_entry_point():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2107_07166_amd import _lib, api
    ctx = api.Context(0)
    lib = ctx.lib
    stream = torch.cuda.current_stream().cuda_stream
    rng = np.random.default_rng(7)
    for n, seed, with_vel in ((300000, 11, True), (20011, 12, False)):
        pos, m, v = plummer(n, seed, velocities=True)
        f = rng.normal(size=(n, 3)) * 1e-3
        pd, md, vd, fd = _dev(pos), _dev(m), _dev(v), _dev(f)
        out = torch.full((20,), float("nan"), dtype=torch.float64, device="cuda")
        held = ctx.bytes_held()
        rc = lib.tfmm_momentum_diagnostics_noalloc(ctx.handle, n, pd.data_ptr(),
                                                   vd.data_ptr() if with_vel else None, md.data_ptr(),
                                                   fd.data_ptr(), out.data_ptr(), stream)
        assert rc == _lib.OK, lib.tfmm_last_error(ctx.handle)
        torch.cuda.synchronize()
        assert ctx.bytes_held() == held
        got = out.cpu().numpy()
        ref = ctx.diagnostics(pd, md, fd, vel=vd if with_vel else None)
        print(f"  n={n}: net force {got[18]:.3e} net torque {got[19]:.3e}", flush=True)
        assert np.array_equal(got, ref), (n, got, ref)
        if not with_vel:
            assert np.all(got[8:14] == 0.0)
    # beyond the limit: refused, nothing enqueued, the context stays usable
    out = torch.zeros(20, dtype=torch.float64, device="cuda")
    small = torch.zeros(3, dtype=torch.float64, device="cuda")
    for bad_n in (0, (1 << 30) + 1):
        rc = lib.tfmm_momentum_diagnostics_noalloc(ctx.handle, bad_n, small.data_ptr(), None, small.data_ptr(),
                                                   small.data_ptr(), out.data_ptr(), stream)
        assert rc == _lib.EINVAL
        assert b"2^30" in lib.tfmm_last_error(ctx.handle)
    rc = lib.tfmm_momentum_diagnostics_noalloc(ctx.handle, 10, small.data_ptr(), None, small.data_ptr(),
                                               small.data_ptr(), None, stream)
    assert rc == _lib.EINVAL
    torch.cuda.synchronize()
    assert np.all(out.cpu().numpy() == 0.0)
    ctx.close()
