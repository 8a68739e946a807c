"""The two workloads of the benchmark suite that the other parity tests do not reach:

* the n = 4096 GUE-like pencil (A = (G + G^H)/2, B = U diag(logspace(0, 3, n)) U^H, seed 1),
  all eigenpairs, band width 64: eigenvalues entry by entry against the oracle's
  (stored by tests/golden/make_oracle_values.py; the oracle needs minutes at this size)
  within 1e-12 max|lambda|, the residual and B-orthogonality over every column, and the
  stored oracle vectors of five columns up to phase;
* the batched workload: 64 pencils with n uniform in [500, 3000] (the GUE recipe with
  cond(B) = 1e2, problem i seeded [3, i]), the lowest 20 % of each, the whole batch
  captured in one HIP graph and replayed, in FP64 and in mixed precision: residual and
  B-orthogonality of all 64 problems on the device, and the eigenvalues and sampled
  vectors of the two smallest and the two largest problems against the stored oracle
  values.
The pencils are built on the device (the same seeded draws; the products run in torch), so
they differ from the ones the stored values were computed on by rounding only, far below
the tolerances.
"""
import math
import os

import numpy as np
import pytest

from inputs import batch_problem, batch_sizes, gue_pair
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def hgv():
    return require_gpu()


def load_golden(prefix):
    W = np.loadtxt(os.path.join(GOLDEN, prefix + "_W.txt"))
    X = np.load(os.path.join(GOLDEN, prefix + "_X_cols.npy"), allow_pickle=False)
    return np.atleast_1d(W), X


def device_metrics(A, B, W, X):
    """(residual, B-orthogonality) in the 1-norm convention of tests.metrics, on the device."""
    import torch
    n1 = lambda M: float(M.abs().sum(0).max())
    n = A.shape[0]
    BX = B @ X
    R = A @ X - BX * W.to(X.dtype)[None, :]
    G = X.conj().T @ BX
    res = n1(R) / (n * n1(A) * n1(X))
    orth = n1(G - torch.eye(G.shape[0], dtype=G.dtype, device=G.device))
    return res, orth


def alignment(B, X, Xo):
    """|x_i^H B xo_i| per column (1 when equal up to phase), on the device."""
    import torch
    Xo = torch.as_tensor(Xo).to(X.device)
    return (X.conj() * (B @ Xo)).sum(0).abs().cpu().numpy()


def test_config1_gue_n4096_all_pairs(hgv):
    import torch
    n = 4096
    dev = torch.device("cuda:0")
    print("config 1: n=%d nb=64 all pairs" % n, flush=True)
    A, B = gue_pair(n, 1, cond_b=1e3, device=dev)
    ctx = hgv.Context.get(dev)
    W, X, info, st = ctx.zhegvx(A, B, nb=64, stats=True)
    assert info == 0
    Wo, Xcols = load_golden("config1_n4096")
    Wn = W.cpu().numpy()
    np.testing.assert_allclose(Wn, Wo, rtol=0, atol=1e-12 * np.abs(Wo).max())
    # residual per quarter of the columns and B-orthogonality over all of them
    for q in range(4):
        sl = slice(q * n // 4, (q + 1) * n // 4)
        res, _ = device_metrics(A, B, W[sl], X[:, sl])
        assert res <= 1e-14, (q, res)
    _, orth = device_metrics(A, B, W, X)
    assert orth <= 1e-13 * n
    cols = [0, 1, 2047, 4094, 4095]
    gaps = np.minimum(np.abs(np.diff(Wo, prepend=-np.inf)), np.abs(np.diff(Wo, append=np.inf)))[cols]
    al = alignment(B, X[:, cols], Xcols)
    sep = gaps > 1e-6 * np.abs(Wo).max()
    assert sep.any()
    assert (1 - al[sep]).max() < 1e-8, al


def batch_ends():
    s = np.asarray(batch_sizes())
    order = np.argsort(s, kind="stable")
    return [int(i) for i in list(order[:2]) + list(order[-2:])]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_config3_batched_64_pencils(hgv, precision):
    import torch
    dev = torch.device("cuda:0")
    sizes = batch_sizes()
    il = [1] * len(sizes)
    iu = [int(math.ceil(0.2 * n)) for n in sizes]
    print("config 3: %d pencils, n in [%d, %d], %s" % (len(sizes), min(sizes), max(sizes), precision), flush=True)
    As, Bs = [], []
    for i, n in enumerate(sizes):
        A, B = batch_problem(i, n, device=dev)
        As.append(A)
        Bs.append(B)
    ctx = hgv.Context.get(dev)
    nb = [hgv.hgv_default_nb(n) for n in sizes]
    bs = hgv.tensors.BatchedSolve(ctx, As, Bs, il, iu, nb, precision=precision,
                                  max_refine_iters=2 if precision == "mixed" else 0)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            bs.run()
    torch.cuda.current_stream().wait_stream(side)
    ctx._sync_stream()
    for rep in range(2):
        for w in bs.W:
            w.fill_(7.0)
        bs.info.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        Ws, Xs, infos = bs.results()
        assert infos == [0] * len(sizes), rep
        for i, n in enumerate(sizes):
            res, orth = device_metrics(As[i], Bs[i], Ws[i], Xs[i])
            assert res <= 1e-14 and orth <= 1e-13 * n, (rep, i, n, res, orth)
        for i in batch_ends():
            n = sizes[i]
            Wo, Xcols = load_golden("batch_%d_n%d" % (i, n))
            np.testing.assert_allclose(Ws[i].cpu().numpy(), Wo, rtol=0, atol=1e-12 * np.abs(Wo).max())
            m = iu[i]
            cols = [0, 1, m - 2, m - 1]
            gaps = np.minimum(np.abs(np.diff(Wo, prepend=-np.inf)), np.abs(np.diff(Wo, append=np.inf)))[cols]
            gaps[-1] = np.abs(Wo[-1] - Wo[-2])   # the next eigenvalue above the selection is not stored
            sep = gaps > 1e-6 * np.abs(Wo).max()
            al = alignment(Bs[i], Xs[i][:, cols], Xcols)
            if sep.any():
                assert (1 - al[sep]).max() < 1e-8, (i, al)
