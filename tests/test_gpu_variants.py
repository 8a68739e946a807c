"""The other storage types of the generalized solve, through the C ABI: complex64 pencils
(hgv_chegvx) and real symmetric-definite pencils (hgv_dsygvx), against the FP64 oracle.

complex64 bars (a backward-stable solver in FP32 arithmetic, eps32 = 2^-23):
  |W - W_oracle| <= 4 eps32 (||A||_2 + |lambda| ||B||_2) ||B^-1||_2   (first-order
  perturbation of a simple eigenvalue by backward errors of size eps32 ||A||, eps32 ||B||),
  residual ||AX - BXW||_1 / (n ||A||_1 ||X||_1) <= eps32 / 4, ||X^H B X - I||_1 <= eps32 n cond(B)
  (measured on the first runs: at most 0.15, 0.13 and 0.12 of these bars);
the oracle runs on the complex128 copy of the same complex64 input.
real bars: those of the complex-double solve (the real pencil runs through it), and the
complex solve of the zero-imaginary copy has eigenvectors with imaginary parts exactly 0.
"""
import numpy as np
import pytest

import oracle
from inputs import gue_pair
from tests.gpu_util import rand_herm, rand_hpd, require_gpu, to_dev, to_np
from tests.metrics import orthogonality, pair_alignment, residual

pytestmark = pytest.mark.gpu
EPS32 = float(np.finfo(np.float32).eps)


@pytest.fixture(scope="module")
def ctx():
    hgv = require_gpu()
    return hgv.Context.get("cuda:0")


def c64_bars(A, B, Wo):
    n = A.shape[0]
    sb = np.linalg.eigvalsh(B)
    na = np.abs(np.linalg.eigvalsh(A)).max()
    tol_w = 4 * EPS32 * (na + np.abs(Wo) * sb.max()) / sb.min()
    return tol_w, EPS32 * n * sb.max() / sb.min()


@pytest.mark.parametrize("n,il,iu,nb,kind", [(300, 1, 300, 32, "hpd"), (257, 1, 52, 32, "gue"), (520, 100, 300, 64, "gue"),
                                           (64, 1, 64, 32, "hpd"), (33, 5, 9, 64, "gue")])
def test_chegvx_vs_oracle(ctx, n, il, iu, nb, kind):
    if kind == "hpd":
        A, B = rand_herm(n, 100 + n), rand_hpd(n, 101 + n)
    else:
        A, B = gue_pair(n, 102 + n, cond_b=1e2)
        A, B = A.numpy(), B.numpy()
    A32, B32 = A.astype(np.complex64), B.astype(np.complex64)
    A64, B64 = A32.astype(np.complex128), B32.astype(np.complex128)
    W, X, info, _ = ctx.chegvx(to_dev(A32), to_dev(B32), il, iu, nb=nb)
    assert info == 0
    assert W.dtype.is_floating_point and X.dtype == __import__("torch").complex64
    W, X = to_np(W).astype(np.float64), to_np(X).astype(np.complex128)
    Wo, Xo, info_o = oracle.zhegv(A64, B64, il, iu)
    assert info_o == 0
    tol_w, tol_o = c64_bars(A64, B64, Wo)
    err = np.abs(W - Wo)
    res, orth = residual(A64, B64, W, X), orthogonality(B64, X)
    print("n=%d max|dW|/tol=%.3f res=%.2e orth=%.2e (bar %.2e)" % (n, (err / tol_w).max(), res, orth, tol_o),
          flush=True)
    assert (err <= tol_w).all()
    assert res <= EPS32 / 4
    assert orth <= tol_o


def test_chegvx_values_only(ctx):
    n = 400
    A, B = gue_pair(n, 110, cond_b=1e2)
    A32, B32 = A.numpy().astype(np.complex64), B.numpy().astype(np.complex64)
    W, X, info, _ = ctx.chegvx(to_dev(A32), to_dev(B32), 1, 80, values_only=True)
    assert info == 0 and X is None
    Wo, _, _ = oracle.zhegv(A32.astype(np.complex128), B32.astype(np.complex128), 1, 80)
    tol_w, _ = c64_bars(A32.astype(np.complex128), B32.astype(np.complex128), Wo)
    assert (np.abs(to_np(W) - Wo) <= tol_w).all()


def test_chegvx_not_positive_definite(ctx):
    n = 80
    A = rand_herm(n, 111)
    Lb = np.linalg.cholesky(rand_hpd(n, 112))
    Dg = np.ones(n)
    Dg[30] = -1.0
    B = (Lb * Dg) @ Lb.conj().T
    _, _, info, _ = ctx.chegvx(to_dev(A.astype(np.complex64)), to_dev(B.astype(np.complex64)))
    assert info == n + 31


def real_pencil(n, seed):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n))
    A = 0.5 * (G + G.T)
    H = rng.standard_normal((n, n))
    B = H @ H.T + n * np.eye(n)
    return A, B


@pytest.mark.parametrize("n,il,iu,nb,precision", [(300, 1, 300, 32, "fp64"), (211, 20, 70, 32, "fp64"),
                                                  (65, 1, 65, 64, "fp64"), (256, 1, 40, 32, "mixed")])
def test_dsygvx_vs_oracle(ctx, n, il, iu, nb, precision):
    from scipy.linalg import cholesky, eigh
    A, B = real_pencil(n, 120 + n)
    W, X, info, _, L = ctx.dsygvx(to_dev(A), to_dev(B), il, iu, precision, nb=nb)
    assert info == 0
    W, X, L = to_np(W), to_np(X), to_np(L)
    assert X.dtype == np.float64
    Wo, Xo, info_o = oracle.zhegv(A.astype(complex), B.astype(complex), il, iu)
    assert info_o == 0
    np.testing.assert_allclose(W, Wo, rtol=0, atol=1e-12 * np.abs(Wo).max())
    np.testing.assert_allclose(W, eigh(A, B, eigvals_only=True, subset_by_index=[il - 1, iu - 1]), rtol=0,
                               atol=1e-12 * np.abs(Wo).max())
    assert residual(A, B, W, X) <= 1e-14
    assert orthogonality(B, X) <= 1e-13 * n
    assert pair_alignment(B.astype(complex), X.astype(complex), Xo).min() > 1 - 1e-8
    np.testing.assert_allclose(L, cholesky(B, lower=True), rtol=0, atol=1e-12 * np.abs(B).max())


def test_dsygvx_values_only(ctx):
    from scipy.linalg import eigh
    n = 350
    A, B = real_pencil(n, 130)
    W, X, info, _, _ = ctx.dsygvx(to_dev(A), to_dev(B), 1, n, values_only=True)
    assert info == 0 and X is None
    Wl = eigh(A, B, eigvals_only=True)
    np.testing.assert_allclose(to_np(W), Wl, rtol=0, atol=1e-12 * np.abs(Wl).max())


def test_real_data_stays_real(ctx):
    """The claim the real front end rests on: the complex solve of a pencil with zero
    imaginary parts returns eigenvectors with imaginary parts exactly zero."""
    n = 300
    A, B = real_pencil(n, 140)
    W, X, info, _ = ctx.zhegvx(to_dev(A.astype(complex)), to_dev(B.astype(complex)), nb=32)
    assert info == 0
    assert not np.any(to_np(X).imag)
