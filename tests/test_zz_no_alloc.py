"""hgv_dstebz_noalloc (the allocation-free entry point: its scratch is a device array the
library holds) against hgv_dstebz (the same kernels with the scratch in the caller's
workspace), through the C ABI: equal bit for bit on two calls in a row, the second with a
smaller input, and the size limit rejected on the host."""
import numpy as np
import pytest

from tests.gpu_util import require_gpu, to_dev, to_np

pytestmark = pytest.mark.gpu


def tridiag(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n), rng.standard_normal(max(n - 1, 0))


def test_noalloc_matches_workspace_entry_point():
    import torch
    hgv = require_gpu()
    ctx = hgv.Context.get("cuda:0")
    ctx._sync_stream()
    for n, il, iu, seed in [(3000, 1, 3000, 1), (700, 50, 400, 2)]:
        print("noalloc n=%d il=%d iu=%d" % (n, il, iu), flush=True)
        d, e = tridiag(n, seed)
        dd, ee = to_dev(d), to_dev(e)
        m = iu - il + 1
        W1 = torch.full((m,), 7.0, dtype=torch.float64, device="cuda:0")
        hgv.hgv_dstebz_noalloc(ctx.handle, n, dd.data_ptr(), ee.data_ptr(), il, iu, W1.data_ptr())
        wsb = hgv.hgv_dstebz_bufsize(ctx.handle, n)
        w = torch.empty(wsb, dtype=torch.uint8, device="cuda:0")
        W2 = torch.full((m,), -7.0, dtype=torch.float64, device="cuda:0")
        hgv.hgv_dstebz(ctx.handle, n, dd.data_ptr(), ee.data_ptr(), il, iu, W2.data_ptr(), w.data_ptr(), wsb)
        torch.cuda.synchronize()
        assert np.array_equal(to_np(W1), to_np(W2))
        # and against LAPACK's tridiagonal eigenvalues
        from scipy.linalg import eigvalsh_tridiagonal
        wl = eigvalsh_tridiagonal(d, e)[il - 1:iu]
        nT = np.abs(d).max() + 2 * np.abs(e).max()
        np.testing.assert_allclose(to_np(W1), wl, rtol=0, atol=1e-13 * nT * max(1, n / 100))


def test_noalloc_rejects_oversize():
    hgv = require_gpu()
    ctx = hgv.Context.get("cuda:0")
    with pytest.raises(hgv.HgvError) as ex:
        hgv.hgv_dstebz_noalloc(ctx.handle, hgv.HGV_DSTEBZ_NOALLOC_MAX + 1, 1, 1, 1, 1, 1)
    assert ex.value.status == -2
