"""Mixed precision (complex64 band reduction, bulge chasing and back-transforms, FP64
tridiagonal solve and FP64 refinement) against the oracle, at the FP64 bars.

* Eigenvalues within 1e-12 max|lambda| of the oracle's, residual <= 1e-14 and
  ||X^H B X - I||_1 <= 1e-13 n (the same bars as the FP64 path), with the refinement
  converged (no fallback) after at least one correction.
* max_refine_iters < 0 forces the FP64 fallback, whose result is the FP64 path's bit
  for bit.
* Under HIP-graph capture the iteration count is fixed; replays match the eager run.
* Batched mixed solves meet the same bars.
"""
import math

import numpy as np
import pytest

import oracle
from inputs import batch_problem, constructed, gue_pair
from tests.gpu_util import require_gpu, to_dev, to_np
from tests.metrics import orthogonality, residual

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hgv():
    return require_gpu()


def check(A, B, il, iu, W, X, info, tol_w=1e-12):
    assert info == 0
    Wo, _, _ = oracle.zhegv(A, B, il, iu)
    np.testing.assert_allclose(W, Wo, rtol=0, atol=tol_w * np.abs(Wo).max())
    n = A.shape[0]
    assert residual(A, B, W, X) <= 1e-14
    assert orthogonality(B, X) <= 1e-13 * n


@pytest.mark.parametrize("n,il,iu,spec,seed", [
    (512, 1, 52, "uniform", 1),        # lowest 10 %
    (700, 1, 175, "loguniform", 2),    # lowest 25 %
    (300, 100, 150, "uniform", 3),     # interior range: guards on both sides
    (256, 1, 256, "uniform", 4),       # all pairs
    (130, 130, 130, "loguniform", 5),  # the largest one
    (40, 1, 3, "uniform", 6),          # smaller than the guard band
])
def test_mixed_constructed(hgv, n, il, iu, spec, seed):
    A, B = constructed(n, seed, spec)
    A, B = A.numpy(), B.numpy()
    ctx = hgv.Context.get("cuda:0")
    W, X, info, st = ctx.zhegvx(to_dev(A), to_dev(B), il, iu, precision="mixed", stats=True)
    print("n=%d il=%d iu=%d iters=%d rho=%.3e fallback=%d" % (n, il, iu, st["refine_iters"], st["refine_resid"],
                                                               st["fallback"]), flush=True)
    assert st["fallback"] == 0
    # a working subspace that is the whole space is exact after one Rayleigh-Ritz step
    working = min(n, iu + 32) - max(1, il - 32) + 1
    assert st["refine_iters"] >= (1 if working < n else 0)
    assert st["refine_resid"] <= 32 * np.finfo(float).eps * math.sqrt(n)
    check(A, B, il, iu, to_np(W), to_np(X), info)


def test_mixed_random_pencil(hgv):
    n = 400
    A, B = gue_pair(n, 11, cond_b=1e3)
    A, B = A.numpy(), B.numpy()
    ctx = hgv.Context.get("cuda:0")
    W, X, info, st = ctx.zhegvx(to_dev(A), to_dev(B), 1, 80, precision="mixed", stats=True)
    assert st["fallback"] == 0
    check(A, B, 1, 80, to_np(W), to_np(X), info)


def test_mixed_forced_fallback_equals_fp64(hgv):
    n = 300
    A, B = constructed(n, 7, "uniform")
    ctx = hgv.Context.get("cuda:0")
    W1, X1, info1, st = ctx.zhegvx(A.to("cuda:0"), B.to("cuda:0"), 1, 40, precision="mixed", stats=True,
                                   max_refine_iters=-1)
    W0, X0, info0, _ = ctx.zhegvx(A.to("cuda:0"), B.to("cuda:0"), 1, 40, precision="fp64")
    assert info1 == 0 and info0 == 0
    assert st["fallback"] == 1
    assert np.array_equal(to_np(W1), to_np(W0))
    assert np.array_equal(to_np(X1), to_np(X0))


def test_mixed_graph_capture_fixed_iterations(hgv):
    import torch
    import paper_1207_1773_amd as h
    from paper_1207_1773_amd.tensors import _opts, _ptr, colmajor, from_colmajor
    n, il, iu = 200, 1, 30
    A, B = constructed(n, 8, "uniform")
    ctx = h.Context.get("cuda:0")
    We, Xe, infoe, _ = ctx.zhegvx(A.to("cuda:0"), B.to("cuda:0"), il, iu, precision="mixed")
    assert infoe == 0
    A0, B0 = colmajor(A.to("cuda:0")), colmajor(B.to("cuda:0"))
    Aw, Bw = A0.clone(), B0.clone()
    m = iu - il + 1
    W = torch.zeros(m, dtype=torch.float64, device="cuda:0")
    Xc = torch.zeros((m, n), dtype=torch.complex128, device="cuda:0")
    info = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    opts = _opts("mixed", 0, 2, 0.0)
    w = ctx._work(h.hgv_zhegvx_bufsize(ctx.handle, n, il, iu, opts))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            Aw.copy_(A0)
            Bw.copy_(B0)
            h.hgv_set_stream(ctx.handle, torch.cuda.current_stream().cuda_stream)
            h.hgv_zhegvx(ctx.handle, n, _ptr(Aw), n, _ptr(Bw), n, il, iu, _ptr(W), _ptr(Xc), n, _ptr(w), w.numel(),
                         opts, _ptr(info), None)
    torch.cuda.current_stream().wait_stream(side)
    ctx._sync_stream()
    for rep in range(3):
        W.zero_()
        Xc.zero_()
        info.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        junk = torch.randn(256, 256, device="cuda:0") @ torch.randn(256, 256, device="cuda:0")
        torch.cuda.synchronize()
        assert int(info.item()) == 0, rep
        Wr, Xr = to_np(W), to_np(from_colmajor(Xc))
        check(A.numpy(), B.numpy(), il, iu, Wr, Xr, 0)
        np.testing.assert_allclose(Wr, to_np(We), rtol=0, atol=1e-13)
    del junk


def test_batched_mixed(hgv):
    import torch
    sizes = [200, 77, 150, 33]
    As, Bs, il, iu = [], [], [], []
    for i, n in enumerate(sizes):
        A, B = batch_problem(i, n, seed=17)
        As.append(A)
        Bs.append(B)
        il.append(1)
        iu.append(max(1, int(math.ceil(0.2 * n))))
    ctx = hgv.Context.get("cuda:0")
    bs = hgv.tensors.BatchedSolve(ctx, As, Bs, il, iu, precision="mixed", max_refine_iters=2)
    bs.run()
    torch.cuda.synchronize()
    Ws, Xs, infos = bs.results()
    assert infos == [0] * len(sizes)
    for i in range(len(sizes)):
        check(As[i].numpy(), Bs[i].numpy(), il[i], iu[i], to_np(Ws[i]), to_np(Xs[i]), 0)
