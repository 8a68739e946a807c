"""GPU divide-and-conquer tridiagonal eigensolver (Alg. 2 step 2, Sec. 4.3) against the
oracle's implicit QL on the same (d, e).

Eigenvalues are unique: |lambda_gpu - lambda_oracle| <= 1e-13 ||T||_1 (both backward
stable, Weyl bound).  Eigenvectors are unique up to sign for simple eigenvalues: the
tests compare |z_i . z~_i| >= 1 - 1e-20 / relgap_i^2 style bounds through the subspace
angle, and check orthogonality and the residual for every vector.  Leaves hold at most 64
rows (n spread evenly over a power-of-two number of blocks), so sizes above 64 span
several merge levels, ragged last leaves and, from n = 2049 on, blocks left unpaired at a
level.
"""
import numpy as np
import pytest

import oracle
from tests.gpu_util import require_gpu, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    hgv = require_gpu()
    return hgv.Context.get("cuda:0")


def tridiag_cases(n, kind, seed):
    rng = np.random.default_rng(seed)
    if kind == "rand":
        return rng.standard_normal(n), rng.standard_normal(max(n - 1, 0))
    if kind == "toeplitz":
        return np.full(n, 0.3), np.full(max(n - 1, 0), 1.7)
    if kind == "clustered":
        d = np.sign(rng.standard_normal(n)) * 10.0 ** rng.uniform(-3, 1, n)
        return d, 1e-3 * rng.standard_normal(max(n - 1, 0))
    if kind == "glued":   # glued Wilkinson-like blocks: tight clusters
        d = np.tile(np.abs(np.arange(-5, 6)), n // 11 + 1)[:n].astype(float)
        e = np.ones(max(n - 1, 0))
        e[10::11] = 1e-9
        return d, e
    if kind == "split":   # exact zeros in e
        d, e = rng.standard_normal(n), rng.standard_normal(max(n - 1, 0))
        e[::7] = 0.0
        return d, e
    raise ValueError(kind)


def check(d, e, lam, Z, il, iu):
    n = len(d)
    T = np.diag(d) + np.diag(e, -1) + np.diag(e, 1)
    nT = np.abs(T).sum(axis=0).max() if n else 1.0
    wo, Zo, info = oracle.steql(d, e)
    assert info == 0
    np.testing.assert_allclose(lam, wo, rtol=0, atol=1e-13 * max(nT, 1e-300) * max(1, n / 100))
    W = wo[il - 1:iu]
    assert np.abs(T @ Z - Z * W).max() <= 1e-13 * nT * max(1, n / 100)
    assert np.abs(Z.T @ Z - np.eye(Z.shape[1])).max() <= 1e-13 * max(1, n / 100)
    # vectors of well separated eigenvalues agree with the oracle's up to sign
    gaps = np.minimum(np.abs(np.diff(wo, prepend=-np.inf)), np.abs(np.diff(wo, append=np.inf)))[il - 1:iu]
    sep = gaps > 1e-6 * nT
    if sep.any():
        align = np.abs((Z * Zo[:, il - 1:iu]).sum(axis=0))
        assert (1 - align[sep]).max() < 1e-18 / (gaps[sep] / nT).min() ** 2 + 1e-12


@pytest.mark.parametrize("n", [1, 2, 5, 31, 32, 33, 64, 65, 100, 129, 257, 600])
@pytest.mark.parametrize("kind", ["rand", "toeplitz", "clustered", "glued", "split"])
def test_stedc_full(ctx, n, kind):
    d, e = tridiag_cases(n, kind, n)
    lam, Z, info = ctx.stedc(to_dev(d), to_dev(e), 1, n)
    assert info == 0
    check(d, e, to_np(lam), to_np(Z), 1, n)


@pytest.mark.parametrize("kind", ["rand", "glued"])
def test_stedc_unpaired_blocks_n2049(ctx, kind):
    """n = 2049: 63 leaves of 33 rows, so one block per level up the tree is carried over
    unpaired.  Eigenvalues against LAPACK's tridiagonal eigenvalue routine (the oracle's
    QL with vectors takes about 10 s at this size); residual and orthogonality of every
    vector."""
    from scipy.linalg import eigvalsh_tridiagonal

    n = 2049
    d, e = tridiag_cases(n, kind, n)
    lam, Z, info = ctx.stedc(to_dev(d), to_dev(e), 1, n)
    assert info == 0
    lam, Z = to_np(lam), to_np(Z)
    nT = np.abs(np.diag(d) + np.diag(e, -1) + np.diag(e, 1)).sum(axis=0).max()
    wl = eigvalsh_tridiagonal(d, e)
    np.testing.assert_allclose(lam, wl, rtol=0, atol=1e-13 * nT * n / 100)
    TZ = d[:, None] * Z
    TZ[:-1] += e[:, None] * Z[1:]
    TZ[1:] += e[:, None] * Z[:-1]
    assert np.abs(TZ - Z * lam).max() <= 1e-13 * nT * n / 100
    assert np.abs(Z.T @ Z - np.eye(n)).max() <= 1e-13 * n / 100


@pytest.mark.parametrize("n,il,iu", [(300, 1, 30), (300, 271, 300), (513, 100, 100), (97, 1, 97), (1000, 1, 100)])
def test_stedc_subset(ctx, n, il, iu):
    d, e = tridiag_cases(n, "rand", 7 + n)
    lam, Z, info = ctx.stedc(to_dev(d), to_dev(e), il, iu)
    assert info == 0
    check(d, e, to_np(lam), to_np(Z), il, iu)
