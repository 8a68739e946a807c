"""GPU parity of the level-3 building blocks and of Alg. 1 steps 1, 2 and 4.

* zgemm (the MFMA tiles every stage uses) against numpy's fp64 product, over all
  operand modes, ragged sizes that span several 64 x 64 tiles, small products on
  32 x 32 tiles (fewer than 128 tiles of 64 x 64 and K <= 512), and split-K shapes.
  The in-place tiles (32 x 64 and 64 x 32) run inside the Cholesky, reduction and
  triangular-solve parity tests below.
* Cholesky (Alg. 1 step 1) and the reduction to standard form (Alg. 1 step 2) have
  unique results, so they are compared entry by entry with the oracle.
* The back-substitution X = L^-H Y (Alg. 1 step 4) against a triangular solve.
Tolerances: fp64 rounding of an order-k product is bounded by about k eps |A||B|;
the tests use 1e-13 relative Frobenius error (about 50 eps) for products, and
1e-12 for the factorisations (condition numbers of the test matrices < 1e2).
"""
import numpy as np
import pytest
import scipy.linalg as sl

import oracle
from tests.gpu_util import rand_herm, rand_hpd, rel_fro, require_gpu, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    hgv = require_gpu()
    return hgv.Context.get("cuda:0")


def _op(M, op):
    return M if op == "N" else (M.T if op == "T" else M.conj().T)


@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (64, 64, 64), (65, 33, 17), (200, 130, 300), (16, 16, 5000),
                                   (300, 64, 4096), (129, 257, 0), (500, 301, 128), (100, 700, 512)])
@pytest.mark.parametrize("opa,opb", [("N", "N"), ("N", "C"), ("C", "N"), ("T", "T"), ("C", "C"), ("N", "T")])
def test_zgemm_parity(ctx, m, n, k, opa, opb):
    rng = np.random.default_rng(m * 7 + n * 3 + k)
    ra, ca = (m, k) if opa == "N" else (k, m)
    rb, cb = (k, n) if opb == "N" else (n, k)
    A = rng.standard_normal((ra, ca)) + 1j * rng.standard_normal((ra, ca))
    B = rng.standard_normal((rb, cb)) + 1j * rng.standard_normal((rb, cb))
    C = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
    alpha, beta = 0.7 - 0.2j, -1.3 + 0.5j
    ref = alpha * (_op(A, opa) @ _op(B, opb)) + beta * C
    out = to_np(ctx.gemm(opa, opb, to_dev(A), to_dev(B), alpha, beta, to_dev(C)))
    assert rel_fro(out, ref) < 1e-13


def test_zgemm_beta_zero_ignores_nan(ctx):
    rng = np.random.default_rng(3)
    A = rng.standard_normal((70, 40)) + 0j
    B = rng.standard_normal((40, 90)) + 0j
    C = np.full((70, 90), np.nan + 0j)
    out = to_np(ctx.gemm("N", "N", to_dev(A), to_dev(B), 1.0, 0.0, to_dev(C)))
    assert np.isfinite(out).all()
    assert rel_fro(out, A @ B) < 1e-13


@pytest.mark.parametrize("n", [1, 2, 17, 64, 65, 128, 200, 513])
def test_potrf_parity(ctx, n):
    B = rand_hpd(n, n)
    Lo, info_o = oracle.potrf(np.tril(B))
    assert info_o == 0
    L, info = ctx.potrf(to_dev(np.tril(B)))
    L = to_np(L)
    assert info == 0
    assert rel_fro(L, Lo) < 1e-12
    assert np.abs(np.diag(L).imag).max() == 0.0
    assert rel_fro(L @ L.conj().T, B) < 1e-14


@pytest.mark.parametrize("n,k", [(8, 3), (100, 71), (300, 1), (300, 300)])
def test_potrf_not_pd(ctx, n, k):
    B = rand_hpd(n, 5)
    Lb = np.linalg.cholesky(B)
    # make the leading minor of order k indefinite: B = L D L^H with D_kk < 0
    D = np.ones(n)
    D[k - 1] = -1.0
    Bbad = (Lb * D) @ Lb.conj().T
    _, info_o = oracle.potrf(np.tril(Bbad))
    _, info = ctx.potrf(to_dev(np.tril(Bbad)))
    assert info_o == k
    assert info == k


@pytest.mark.parametrize("n", [1, 3, 64, 65, 130, 333, 600])
def test_hegst_parity(ctx, n):
    A = rand_herm(n, 10 + n)
    B = rand_hpd(n, 20 + n)
    Lo, _ = oracle.potrf(np.tril(B))
    Co = oracle.hegst(np.tril(A), Lo)
    # garbage in the strict upper triangles must not matter
    junk = np.triu(np.full((n, n), 1e30 + 1e30j), 1)
    C = to_np(ctx.hegst(to_dev(np.tril(A) + junk), to_dev(Lo)))
    assert rel_fro(C, np.tril(Co)) < 1e-12
    assert np.abs(np.diag(C).imag).max() == 0.0


@pytest.mark.parametrize("n,m", [(1, 1), (64, 10), (65, 65), (257, 100), (500, 1)])
def test_trsm_lh_parity(ctx, n, m):
    B = rand_hpd(n, 30 + n)
    L = np.linalg.cholesky(B)
    rng = np.random.default_rng(n + m)
    Y = rng.standard_normal((n, m)) + 1j * rng.standard_normal((n, m))
    ref = sl.solve_triangular(L.conj().T, Y, lower=False)
    X = to_np(ctx.trsm_lh(to_dev(L), to_dev(Y)))
    assert rel_fro(X, ref) < 1e-12
