"""Failure reporting and degenerate pencils through the C ABI.

* Bounded waits: with the HGV_TEST_WAIT_FAIL hook the give-up flags of the band
  reduction's panel kernel and of the bulge-chasing kernel start set, so every wait
  returns at once (each kernel still runs to its end, on data that is not final) and
  the call must report d_info = 2n+2.  Without the hook the same context solves
  correctly again.
* Refinement check: with HGV_TEST_NAN_RESIDUAL the mixed-precision refinement sees a
  NaN residual; the check must not take it for convergence (FP64 fallback when the host
  checks, d_info = 2n+1 under graph capture).
* Degenerate pencils end to end: A = c B (every eigenvalue c, every coupling zero, all
  entries deflate), diagonal pencils (lambda_i = a_ii / b_ii), B = I.
"""
import numpy as np
import pytest

import oracle
from inputs import constructed
from tests.gpu_util import rand_herm, rand_hpd, require_gpu, to_dev, to_np
from tests.metrics import orthogonality, pair_alignment, residual

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hgv():
    return require_gpu()


@pytest.fixture
def ctx(hgv):
    c = hgv.Context.get("cuda:0")
    yield c
    hgv.hgv_test_hooks(c.handle, 0)


def test_wait_fail_reported_by_full_solve(hgv, ctx):
    n = 300
    A, B = rand_herm(n, 31), rand_hpd(n, 32)
    print("wait-fail hook, full solve n=%d nb=32" % n, flush=True)
    hgv.hgv_test_hooks(ctx.handle, hgv.HGV_TEST_WAIT_FAIL)
    _, _, info, _ = ctx.zhegvx(to_dev(A), to_dev(B), nb=32)
    assert info == 2 * n + 2
    hgv.hgv_test_hooks(ctx.handle, 0)
    W, X, info, _ = ctx.zhegvx(to_dev(A), to_dev(B), nb=32)
    assert info == 0
    W, X = to_np(W), to_np(X)
    Wo, _, _ = oracle.zhegv(A, B)
    np.testing.assert_allclose(W, Wo, rtol=0, atol=1e-12 * np.abs(Wo).max())
    assert residual(A, B, W, X) <= 1e-14


@pytest.mark.parametrize("nb", [32, 64])
def test_wait_fail_reported_by_bulge_chasing(hgv, ctx, nb):
    n = 257
    band = np.tril(rand_herm(n, 40 + nb))
    band[np.tril_indices(n, -nb - 1)] = 0.0
    print("wait-fail hook, bulge chasing n=%d nb=%d" % (n, nb), flush=True)
    hgv.hgv_test_hooks(ctx.handle, hgv.HGV_TEST_WAIT_FAIL)
    ctx.hb2st(to_dev(band), nb)
    assert int(ctx.last_info.item()) == 2 * n + 2
    hgv.hgv_test_hooks(ctx.handle, 0)
    d, e, _, _ = ctx.hb2st(to_dev(band), nb)
    assert int(ctx.last_info.item()) == 0
    from scipy.linalg import eigvalsh_tridiagonal
    full = band + np.tril(band, -1).conj().T
    np.testing.assert_allclose(eigvalsh_tridiagonal(to_np(d), to_np(e)), np.linalg.eigvalsh(full), rtol=0,
                               atol=1e-12 * np.abs(full).sum(0).max())


def test_wait_fail_reported_by_band_reduction(hgv, ctx):
    n = 400
    A = rand_herm(n, 50)
    print("wait-fail hook, band reduction n=%d nb=64" % n, flush=True)
    hgv.hgv_test_hooks(ctx.handle, hgv.HGV_TEST_WAIT_FAIL)
    ctx.he2hb(to_dev(np.tril(A)), 64)
    assert int(ctx.last_info.item()) == 2 * n + 2
    hgv.hgv_test_hooks(ctx.handle, 0)
    ctx.he2hb(to_dev(np.tril(A)), 64)
    assert int(ctx.last_info.item()) == 0


def test_nan_residual_is_not_convergence(hgv, ctx):
    n, il, iu = 300, 1, 40
    A, B = constructed(n, 9, "uniform")
    print("nan-residual hook, mixed n=%d" % n, flush=True)
    hgv.hgv_test_hooks(ctx.handle, hgv.HGV_TEST_NAN_RESIDUAL)
    W1, X1, info1, st = ctx.zhegvx(A.to("cuda:0"), B.to("cuda:0"), il, iu, precision="mixed", stats=True)
    hgv.hgv_test_hooks(ctx.handle, 0)
    assert info1 == 0
    assert st["fallback"] == 1
    assert np.isnan(st["refine_resid"])
    W0, X0, info0, _ = ctx.zhegvx(A.to("cuda:0"), B.to("cuda:0"), il, iu, precision="fp64")
    assert info0 == 0
    assert np.array_equal(to_np(W1), to_np(W0))
    assert np.array_equal(to_np(X1), to_np(X0))


def test_nan_residual_under_capture_sets_info(hgv, ctx):
    import torch
    from paper_1207_1773_amd.tensors import _opts, _ptr, colmajor
    n, il, iu = 200, 1, 30
    A, B = constructed(n, 10, "uniform")
    A0, B0 = colmajor(A.to("cuda:0")), colmajor(B.to("cuda:0"))
    Aw, Bw = A0.clone(), B0.clone()
    m = iu - il + 1
    W = torch.zeros(m, dtype=torch.float64, device="cuda:0")
    Xc = torch.zeros((m, n), dtype=torch.complex128, device="cuda:0")
    info = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    opts = _opts("mixed", 0, 2, 0.0)
    w = ctx._work(hgv.hgv_zhegvx_bufsize(ctx.handle, n, il, iu, opts))
    print("nan-residual hook, mixed under capture n=%d" % n, flush=True)
    hgv.hgv_test_hooks(ctx.handle, hgv.HGV_TEST_NAN_RESIDUAL)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            Aw.copy_(A0)
            Bw.copy_(B0)
            hgv.hgv_set_stream(ctx.handle, torch.cuda.current_stream().cuda_stream)
            hgv.hgv_zhegvx(ctx.handle, n, _ptr(Aw), n, _ptr(Bw), n, il, iu, _ptr(W), _ptr(Xc), n, _ptr(w),
                           w.numel(), opts, _ptr(info), None)
    torch.cuda.current_stream().wait_stream(side)
    hgv.hgv_test_hooks(ctx.handle, 0)
    ctx._sync_stream()
    for rep in range(2):
        info.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert int(info.item()) == 2 * n + 1, rep


def test_pencil_a_equals_c_b(ctx):
    """A = c B: every eigenvalue is c; any B-orthonormal basis is an answer."""
    n, c = 260, -1.75
    B = rand_hpd(n, 61)
    A = c * B
    W, X, info, _ = ctx.zhegvx(to_dev(A), to_dev(B), nb=32)
    assert info == 0
    W, X = to_np(W), to_np(X)
    np.testing.assert_allclose(W, np.full(n, c), rtol=0, atol=1e-12 * abs(c))
    assert residual(A, B, W, X) <= 1e-14
    assert orthogonality(B, X) <= 1e-13 * n
    Wo, _, info_o = oracle.zhegv(A, B)
    assert info_o == 0
    np.testing.assert_allclose(W, Wo, rtol=0, atol=1e-12 * abs(c))


def test_pencil_a_equals_c_b_subset(ctx):
    n, c = 150, 3.0
    B = rand_hpd(n, 62)
    A = c * B
    W, X, info, _ = ctx.zhegvx(to_dev(A), to_dev(B), 20, 60, nb=32)
    assert info == 0
    W, X = to_np(W), to_np(X)
    np.testing.assert_allclose(W, np.full(41, c), rtol=0, atol=1e-12 * c)
    assert residual(A, B, W, X) <= 1e-14
    assert orthogonality(B, X) <= 1e-13 * n


@pytest.mark.parametrize("n", [1, 7, 64, 200])
def test_diagonal_pencil(ctx, n):
    """Diagonal A, B: lambda_i = a_ii / b_ii, eigenvectors e_i / sqrt(b_ii) up to phase."""
    rng = np.random.default_rng(70 + n)
    a = rng.standard_normal(n)
    b = rng.uniform(0.5, 2.0, n)
    A, B = np.diag(a).astype(complex), np.diag(b).astype(complex)
    W, X, info, _ = ctx.zhegvx(to_dev(A), to_dev(B), nb=32)
    assert info == 0
    W, X = to_np(W), to_np(X)
    lam = a / b
    order = np.argsort(lam, kind="stable")
    np.testing.assert_allclose(W, lam[order], rtol=0, atol=1e-14 * np.abs(lam).max())
    assert residual(A, B, W, X) <= 1e-14
    assert orthogonality(B, X) <= 1e-13 * n
    E = np.zeros((n, n), dtype=complex)
    E[order, np.arange(n)] = 1.0 / np.sqrt(b[order])
    assert pair_alignment(B, X, E).min() >= 1 - 1e-10


def test_identity_b_is_the_standard_problem(ctx):
    n = 230
    A = rand_herm(n, 80)
    B = np.eye(n, dtype=complex)
    W, X, info, _ = ctx.zhegvx(to_dev(A), to_dev(B), nb=32)
    assert info == 0
    W = to_np(W)
    np.testing.assert_allclose(W, np.linalg.eigvalsh(A), rtol=0, atol=1e-12 * np.abs(W).max())
    assert residual(A, B, W, to_np(X)) <= 1e-14
