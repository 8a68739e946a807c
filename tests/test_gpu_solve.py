"""End-to-end GPU parity of the generalized solve (Algorithm 1 with the two-stage
Algorithm 2) against the CPU oracle, through the C ABI (hgv_zhegvx).

Bars (fp64): res = ||AX - BX L||_1/(n ||A||_1 ||X||_1) <= 1e-14 and ||X^H B X - I||_1 <=
1e-13 n; eigenvalues |W - W_oracle| <= 1e-12 max|W|; eigenvectors of eigenvalues with
relative gap > 1e-6 agree with the oracle's up to a phase (|x^H B x~| >= 1 - 1e-8).
Sizes span several 32-wide bands / panels, ragged tails, subsets, n < nb and nb = 1.
"""
import numpy as np
import pytest

import oracle
from inputs import constructed, gue_pair
from tests.gpu_util import rand_herm, rand_hpd, require_gpu, to_dev, to_np
from tests.metrics import orthogonality, pair_alignment, residual

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    hgv = require_gpu()
    return hgv.Context.get("cuda:0")


def compare(A, B, W, X, il, iu):
    n = A.shape[0]
    Wo, Xo, info = oracle.zhegv(A, B, il, iu)
    assert info == 0
    np.testing.assert_allclose(W, Wo, rtol=0, atol=1e-12 * max(np.abs(Wo).max(), 1e-300))
    assert residual(A, B, W, X) <= 1e-14
    assert orthogonality(B, X) <= 1e-13 * n
    Wall = oracle.zhegv(A, B)[0] if (il, iu) != (1, n) else Wo
    gaps = np.minimum(np.abs(np.diff(Wall, prepend=-np.inf)), np.abs(np.diff(Wall, append=np.inf)))[il - 1:iu]
    sep = gaps > 1e-6 * np.abs(Wall).max()
    if sep.any():
        assert pair_alignment(B, X, Xo)[sep].min() > 1 - 1e-8


@pytest.mark.parametrize("n,nb", [(1, 32), (2, 32), (3, 1), (17, 4), (64, 32), (65, 32), (130, 8), (333, 32),
                                  (200, 16), (40, 64)])
def test_solve_random_pencils(ctx, n, nb):
    A = rand_herm(n, 500 + n)
    B = rand_hpd(n, 600 + n)
    W, X, info, _ = ctx.zhegvx(to_dev(A), to_dev(B), nb=nb)
    assert info == 0
    compare(A, B, to_np(W), to_np(X), 1, n)


@pytest.mark.parametrize("il,iu", [(1, 51), (200, 256), (77, 77), (1, 256)])
def test_solve_subsets(ctx, il, iu):
    A, B = gue_pair(256, 11, cond_b=1e2)
    A, B = A.numpy(), B.numpy()
    W, X, info, _ = ctx.zhegvx(to_dev(A), to_dev(B), il, iu, nb=32)
    assert info == 0
    compare(A, B, to_np(W), to_np(X), il, iu)


def test_config0_constructed_spectrum(ctx):
    """n = 512, all pairs, nb = 32 on the constructed pencil: lambda = sort(D)."""
    A, B, parts = constructed(512, 0, "uniform", return_parts=True)
    A, B = A.numpy(), B.numpy()
    W, X, info, st = ctx.zhegvx(to_dev(A), to_dev(B), nb=32, stats=True)
    assert info == 0
    W, X = to_np(W), to_np(X)
    np.testing.assert_allclose(W, np.sort(parts["D"]), rtol=0, atol=1e-13)
    compare(A, B, W, X, 1, 512)


def test_not_positive_definite(ctx):
    n = 50
    A = rand_herm(n, 1)
    Lb = np.linalg.cholesky(rand_hpd(n, 2))
    Dg = np.ones(n)
    Dg[19] = -1.0
    B = (Lb * Dg) @ Lb.conj().T
    _, _, info, _ = ctx.zhegvx(to_dev(A), to_dev(B))
    _, _, info_o = oracle.zhegv(A, B)
    assert info == info_o == n + 20


def test_all_columns_constructed_n4096(ctx):
    """n = 4096, all pairs: lambda = sort(D), and the residual (per half of the columns)
    and B-orthogonality over every column, beyond the leading columns the benchmark's
    accuracy check samples."""
    import torch

    n = 4096
    A, B, parts = constructed(n, 7, "uniform", return_parts=True)
    A, B = A.numpy(), B.numpy()
    W, X, info, _ = ctx.zhegvx(to_dev(A), to_dev(B))
    assert info == 0
    D = np.sort(parts["D"])
    np.testing.assert_allclose(to_np(W), D, rtol=0, atol=1e-12 * np.abs(D).max())
    # the same metrics as tests.metrics, with the n^3 products on the device
    Ad, Bd = to_dev(A), to_dev(B)
    norm1 = lambda M: float(M.abs().sum(0).max())
    BX = Bd @ X
    R = Ad @ X - BX * W.to(X.dtype)[None, :]
    for h in (slice(0, n // 2), slice(n // 2, n)):
        assert norm1(R[:, h]) / (n * norm1(Ad) * norm1(X[:, h])) <= 1e-14
    G = X.conj().T @ BX
    assert norm1(G - torch.eye(n, dtype=G.dtype, device=G.device)) <= 1e-13 * n


@pytest.mark.parametrize("k", [19, 249])
def test_not_positive_definite_split(ctx, k):
    """n = 300: the first failing pivot in the leading block of the top split (k = 19) or
    in the trailing one (k = 249), where the factorisation continues after the reduction of
    the leading block has been started; info = n + k + 1 either way."""
    n = 300
    A = rand_herm(n, 3)
    Lb = np.linalg.cholesky(rand_hpd(n, 4))
    Dg = np.ones(n)
    Dg[k] = -1.0
    B = (Lb * Dg) @ Lb.conj().T
    _, _, info, _ = ctx.zhegvx(to_dev(A), to_dev(B))
    _, _, info_o = oracle.zhegv(A, B)
    assert info == info_o == n + k + 1


def test_reads_lower_triangles_only(ctx):
    n = 90
    A = rand_herm(n, 3)
    B = rand_hpd(n, 4)
    junk = np.triu(np.full((n, n), 7.0 + 7.0j), 1)
    W1, X1, _, _ = ctx.zhegvx(to_dev(A), to_dev(B))
    W2, X2, _, _ = ctx.zhegvx(to_dev(np.tril(A) + junk), to_dev(np.tril(B) + junk))
    assert np.array_equal(to_np(W1), to_np(W2))
    assert np.array_equal(to_np(X1), to_np(X2))


def test_repeatable(ctx):
    n = 300
    A = rand_herm(n, 5)
    B = rand_hpd(n, 6)
    r1 = ctx.zhegvx(to_dev(A), to_dev(B))
    r2 = ctx.zhegvx(to_dev(A), to_dev(B))
    assert np.array_equal(to_np(r1[0]), to_np(r2[0]))
    assert np.array_equal(to_np(r1[1]), to_np(r2[1]))
