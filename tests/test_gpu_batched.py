"""Batched solves of uneven-size pencils (hgv_zhegvx_batched): concurrent streams, one
HIP-graph capture of the whole batch, and the band-width autotuner.

* Every problem of the batch equals its own single solve bit for bit (all kernels are
  deterministic and each problem has its own workspace) and meets the fp64 bars
  against the oracle.
* The batch captured in a HIP graph (torch.cuda.CUDAGraph) replays three times, with
  eager work in between, to the eager result bit for bit.
"""
import math

import numpy as np
import pytest

import oracle
from inputs import batch_problem
from tests.gpu_util import require_gpu, to_np
from tests.metrics import orthogonality, residual

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hgv():
    return require_gpu()


def make_batch(sizes, frac=0.2):
    As, Bs, il, iu = [], [], [], []
    for i, n in enumerate(sizes):
        A, B = batch_problem(i, n, seed=13)
        As.append(A)
        Bs.append(B)
        il.append(1)
        iu.append(max(1, int(math.ceil(frac * n))))
    return As, Bs, il, iu


def test_batched_equals_single_solves(hgv):
    import torch
    sizes = [37, 260, 64, 129, 300, 1, 95]
    As, Bs, il, iu = make_batch(sizes)
    ctx = hgv.Context.get("cuda:0")
    nb = [32 if n <= 128 else 64 for n in sizes]
    bs = hgv.tensors.BatchedSolve(ctx, As, Bs, il, iu, nb)
    bs.run()
    torch.cuda.synchronize()
    Ws, Xs, infos = bs.results()
    assert infos == [0] * len(sizes)
    for i, n in enumerate(sizes):
        # the batch chases the bulges of all its problems with the sweep-per-workgroup
        # schedule; single solves on that schedule do the same arithmetic in the same order
        hgv.hgv_test_hooks(ctx.handle, hgv.HGV_TEST_HB2ST_SWEEPS)
        try:
            W1, X1, info1, _ = ctx.zhegvx(As[i].to("cuda:0"), Bs[i].to("cuda:0"), il[i], iu[i], nb=nb[i])
        finally:
            hgv.hgv_test_hooks(ctx.handle, 0)
        assert info1 == 0
        assert np.array_equal(to_np(Ws[i]), to_np(W1))
        assert np.array_equal(to_np(Xs[i]), to_np(X1))
        A, B = As[i].numpy(), Bs[i].numpy()
        W, X = to_np(Ws[i]), to_np(Xs[i])
        Wo, _, _ = oracle.zhegv(A, B, il[i], iu[i])
        np.testing.assert_allclose(W, Wo, rtol=0, atol=1e-12 * np.abs(Wo).max())
        assert residual(A, B, W, X) <= 1e-14
        assert orthogonality(B, X) <= 1e-13 * n


def test_batched_graph_replay(hgv):
    import torch
    sizes = [200, 77, 150, 33]
    As, Bs, il, iu = make_batch(sizes)
    ctx = hgv.Context.get("cuda:0")
    bs = hgv.tensors.BatchedSolve(ctx, As, Bs, il, iu)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        bs.run()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    W0, X0, info0 = bs.results()
    W0 = [to_np(w).copy() for w in W0]
    X0 = [to_np(x).copy() for x in X0]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        bs.run()
    for rep in range(3):
        for w in bs.W:
            w.zero_()
        for x in bs.X:
            x.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        # eager work between replays
        junk = torch.randn(512, 512, device="cuda:0") @ torch.randn(512, 512, device="cuda:0")
        torch.cuda.synchronize()
        W1, X1, info1 = bs.results()
        assert info1 == [0] * len(sizes)
        for i in range(len(sizes)):
            assert np.array_equal(to_np(W1[i]), W0[i]), (rep, i)
            assert np.array_equal(to_np(X1[i]), X0[i]), (rep, i)
    del junk


def test_autotuner_picks_a_candidate(hgv, tmp_path):
    from paper_1207_1773_amd import autotune
    table = autotune.tune("cuda:0", classes=((100, 200),), candidates=(16, 32), path=str(tmp_path / "tune.json"))
    assert table[(100, 200)] in (16, 32)
    again = autotune.tune("cuda:0", classes=((100, 200),), candidates=(16, 32), path=str(tmp_path / "tune.json"))
    assert again == table
    assert autotune.nb_for(table, 150) == table[(100, 200)]
