"""Eigenvalues only and selection by value (the eigenvalue-only and RANGE = 'V' forms of
Alg. 1 / Alg. 2; Sec. 1: only part of the spectrum is wanted), through the C ABI.

* hgv_dstebz (Sturm-count multisection on the tridiagonal) against the oracle's implicit
  QL on the same (d, e): |lambda - lambda_oracle| <= 1e-13 ||T||_1 max(1, n/100).
* hgv_zhegvx with values_only against the oracle's generalized eigenvalues (1e-12
  max|lambda|) and against the constructed spectrum.
* hgv_zhegvx_range: the count m of eigenvalues in (vl, vu] equals the oracle's, W and X
  are the oracle's pairs il..iu with il = 1 + #{lambda <= vl} (vectors up to phase, the
  residual and B-orthogonality bars of the full solve), truncation at mmax, an empty
  interval, the single-leaf case, values only, and a HIP-graph capture replayed with the
  count read on the device.
The interval ends are put halfway between consecutive oracle eigenvalues, so that no
eigenvalue sits within rounding of an end.
"""
import numpy as np
import pytest

import oracle
from inputs import constructed, gue_pair
from tests.gpu_util import rand_herm, rand_hpd, require_gpu, to_dev, to_np
from tests.metrics import orthogonality, pair_alignment, residual
from tests.test_gpu_stedc import tridiag_cases

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hgv():
    return require_gpu()


@pytest.fixture(scope="module")
def ctx(hgv):
    return hgv.Context.get("cuda:0")


@pytest.mark.parametrize("n", [1, 2, 5, 64, 65, 257, 600])
@pytest.mark.parametrize("kind", ["rand", "toeplitz", "clustered", "glued", "split"])
def test_stebz_vs_oracle(ctx, n, kind):
    d, e = tridiag_cases(n, kind, n + 3)
    wo, _, info = oracle.steql(d, e)
    assert info == 0
    nT = np.abs(np.diag(d) + np.diag(e, -1) + np.diag(e, 1)).sum(axis=0).max()
    W = to_np(ctx.stebz(to_dev(d), to_dev(e), 1, n))
    np.testing.assert_allclose(W, wo, rtol=0, atol=1e-13 * max(nT, 1e-300) * max(1, n / 100))
    if n >= 5:   # a subset is the same slice
        il, iu = 2, n - 2
        Ws = to_np(ctx.stebz(to_dev(d), to_dev(e), il, iu))
        np.testing.assert_allclose(Ws, wo[il - 1:iu], rtol=0, atol=1e-13 * nT * max(1, n / 100))


def test_stebz_n2049_vs_lapack(ctx):
    """n = 2049 against LAPACK's tridiagonal eigenvalue routine (the oracle's QL with
    vectors takes about 10 s at this size)."""
    from scipy.linalg import eigvalsh_tridiagonal
    n = 2049
    d, e = tridiag_cases(n, "glued", n)
    nT = np.abs(np.diag(d) + np.diag(e, -1) + np.diag(e, 1)).sum(axis=0).max()
    W = to_np(ctx.stebz(to_dev(d), to_dev(e)))
    np.testing.assert_allclose(W, eigvalsh_tridiagonal(d, e), rtol=0, atol=1e-13 * nT * n / 100)


@pytest.mark.parametrize("n,il,iu,nb", [(300, 1, 300, 32), (700, 1, 70, 64), (129, 40, 90, 32), (50, 1, 50, 64)])
def test_values_only_vs_oracle(ctx, n, il, iu, nb):
    A, B, parts = constructed(n, 20 + n, "loguniform", return_parts=True)
    A, B = A.numpy(), B.numpy()
    W, X, info, _ = ctx.zhegvx(to_dev(A), to_dev(B), il, iu, nb=nb, values_only=True)
    assert info == 0 and X is None
    W = to_np(W)
    Wo, _, _ = oracle.zhegv(A, B, il, iu)
    np.testing.assert_allclose(W, Wo, rtol=0, atol=1e-12 * np.abs(Wo).max())
    np.testing.assert_allclose(W, np.sort(parts["D"])[il - 1:iu], rtol=0, atol=1e-12 * np.abs(parts["D"]).max())


def test_values_only_random_pencil(ctx):
    n = 333
    A, B = rand_herm(n, 90), rand_hpd(n, 91)
    W, _, info, _ = ctx.zhegvx(to_dev(A), to_dev(B), values_only=True, nb=32)
    assert info == 0
    Wo, _, _ = oracle.zhegv(A, B)
    np.testing.assert_allclose(to_np(W), Wo, rtol=0, atol=1e-12 * np.abs(Wo).max())


def _ends(w, i0, i1):
    """vl, vu halfway between oracle eigenvalues: (vl, vu] holds w[i0 .. i1-1] (0-based)."""
    vl = 0.5 * (w[i0 - 1] + w[i0]) if i0 > 0 else w[0] - 1.0
    vu = 0.5 * (w[i1 - 1] + w[i1]) if i1 < len(w) else w[-1] + 1.0
    return vl, vu


def _check_pairs(A, B, W, X, Wo_all, Xo, i0, k):
    np.testing.assert_allclose(W[:k], Wo_all[i0:i0 + k], rtol=0, atol=1e-12 * np.abs(Wo_all).max())
    n = A.shape[0]
    assert residual(A, B, W[:k], X[:, :k]) <= 1e-14
    assert orthogonality(B, X[:, :k]) <= 1e-13 * n
    gaps = np.minimum(np.abs(np.diff(Wo_all, prepend=-np.inf)), np.abs(np.diff(Wo_all, append=np.inf)))[i0:i0 + k]
    sep = gaps > 1e-6 * np.abs(Wo_all).max()
    if sep.any():
        assert pair_alignment(B, X[:, :k], Xo[:, i0:i0 + k])[sep].min() > 1 - 1e-8


@pytest.mark.parametrize("n,i0,i1,mmax,nb", [(300, 10, 50, 100, 32), (300, 0, 300, 300, 32), (500, 200, 260, 60, 64),
                                             (48, 5, 30, 48, 32), (200, 150, 200, 51, 16)])
def test_range_vs_oracle(ctx, n, i0, i1, mmax, nb):
    A, B = gue_pair(n, 30 + n, cond_b=1e2)
    A, B = A.numpy(), B.numpy()
    Wo, Xo, info_o = oracle.zhegv(A, B)
    assert info_o == 0
    vl, vu = _ends(Wo, i0, i1)
    W, X, m, info, _ = ctx.zhegvx_range(to_dev(A), to_dev(B), vl, vu, mmax, nb=nb)
    assert info == 0
    assert m == i1 - i0
    W, X = to_np(W), to_np(X)
    _check_pairs(A, B, W, X, Wo, Xo, i0, m)
    assert not W[m:].any() and not X[:, m:].any()


def test_range_truncated(ctx):
    n = 256
    A, B = gue_pair(n, 41, cond_b=1e2)
    A, B = A.numpy(), B.numpy()
    Wo, Xo, _ = oracle.zhegv(A, B)
    vl, vu = _ends(Wo, 20, 120)
    W, X, m, info, _ = ctx.zhegvx_range(to_dev(A), to_dev(B), vl, vu, 30, nb=32)
    assert info == 0 and m == 100
    _check_pairs(A, B, to_np(W), to_np(X), Wo, Xo, 20, 30)


def test_range_empty(ctx):
    n = 120
    A, B = rand_herm(n, 50), rand_hpd(n, 51)
    Wo, _, _ = oracle.zhegv(A, B)
    k = int(np.argmax(np.diff(Wo)))   # the widest gap
    vl, vu = Wo[k] + 0.25 * (Wo[k + 1] - Wo[k]), Wo[k] + 0.75 * (Wo[k + 1] - Wo[k])
    W, X, m, info, _ = ctx.zhegvx_range(to_dev(A), to_dev(B), vl, vu, 10, nb=32)
    assert info == 0 and m == 0
    assert not to_np(W).any() and not to_np(X).any()


def test_range_values_only(ctx):
    n = 400
    A, B, parts = constructed(n, 44, "uniform", return_parts=True)
    A, B = A.numpy(), B.numpy()
    D = np.sort(parts["D"])
    vl, vu = _ends(D, 100, 180)
    W, X, m, info, _ = ctx.zhegvx_range(to_dev(A), to_dev(B), vl, vu, 100, nb=32, values_only=True)
    assert info == 0 and X is None and m == 80
    W = to_np(W)
    np.testing.assert_allclose(W[:m], D[100:180], rtol=0, atol=1e-12)
    assert not W[m:].any()


def test_range_graph_capture(hgv, ctx):
    """The count stays on the device: a captured call replays correctly."""
    import torch
    from paper_1207_1773_amd.tensors import _opts, _ptr, colmajor, from_colmajor
    n, mmax = 260, 80
    A, B = gue_pair(n, 45, cond_b=1e2)
    Wo, Xo, _ = oracle.zhegv(A.numpy(), B.numpy())
    vl, vu = _ends(Wo, 30, 90)
    A0, B0 = colmajor(A.to("cuda:0")), colmajor(B.to("cuda:0"))
    Aw, Bw = A0.clone(), B0.clone()
    W = torch.zeros(mmax, dtype=torch.float64, device="cuda:0")
    Xc = torch.zeros((mmax, n), dtype=torch.complex128, device="cuda:0")
    info = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    dm = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    opts = _opts("fp64", 32)
    w = ctx._work(hgv.hgv_zhegvx_range_bufsize(ctx.handle, n, mmax, opts))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            Aw.copy_(A0)
            Bw.copy_(B0)
            hgv.hgv_set_stream(ctx.handle, torch.cuda.current_stream().cuda_stream)
            hgv.hgv_zhegvx_range(ctx.handle, n, _ptr(Aw), n, _ptr(Bw), n, vl, vu, mmax, _ptr(W), _ptr(Xc), n,
                                 _ptr(dm), _ptr(w), w.numel(), opts, _ptr(info), None)
    torch.cuda.current_stream().wait_stream(side)
    ctx._sync_stream()
    for rep in range(3):
        W.fill_(7.0)
        Xc.fill_(7.0)
        dm.fill_(-1)
        info.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        junk = torch.randn(256, 256, device="cuda:0") @ torch.randn(256, 256, device="cuda:0")
        torch.cuda.synchronize()
        del junk
        assert int(info.item()) == 0 and int(dm.item()) == 60, rep
        Wr, Xr = to_np(W), to_np(from_colmajor(Xc))
        _check_pairs(A.numpy(), B.numpy(), Wr, Xr, Wo, Xo, 30, 60)
        assert not Wr[60:].any() and not Xr[:, 60:].any()


def test_range_argument_checks(hgv, ctx):
    import torch
    from paper_1207_1773_amd.tensors import _opts
    n = 10
    buf = torch.zeros((n, n), dtype=torch.complex128, device="cuda:0")
    W = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    dm = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    p = lambda t: t.data_ptr()
    with pytest.raises(hgv.HgvError) as ex:   # vu <= vl
        hgv.hgv_zhegvx_range(ctx.handle, n, p(buf), n, p(buf), n, 1.0, 1.0, n, p(W), p(buf), n, p(dm), None, 0)
    assert ex.value.status == -8
    with pytest.raises(hgv.HgvError) as ex:   # mmax out of range
        hgv.hgv_zhegvx_range(ctx.handle, n, p(buf), n, p(buf), n, 0.0, 1.0, n + 1, p(W), p(buf), n, p(dm), None, 0)
    assert ex.value.status == -9
    with pytest.raises(hgv.HgvError) as ex:   # mixed precision is not supported here
        hgv.hgv_zhegvx_range(ctx.handle, n, p(buf), n, p(buf), n, 0.0, 1.0, n, p(W), p(buf), n, p(dm), None, 0,
                             _opts("mixed"))
    assert ex.value.status == hgv.HGV_E_NOTSUP
