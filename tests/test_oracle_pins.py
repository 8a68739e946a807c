"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test names the passage of the paper (Algorithm 1 / Algorithm 2) or the
mathematical fact it relies on.  Together they are chosen so that a dropped term,
a wrong sign or index, or a transposed operand anywhere in the oracle fails one
of them:
  * closed forms (n = 1, n = 2, diagonal pencils, B = I, A = cB, Toeplitz
    tridiagonals, block-diagonal tridiagonals);
  * brute force at n <= 5: exact characteristic polynomial det(A - lambda B) in
    rational arithmetic, roots and null vectors at 40 digits;
  * constructed spectra A = L Q D Q^H L^H, B = L L^H (eigenvalues exactly D);
  * an independent library (LAPACK zhegvd/zhegvx through scipy);
  * stage identities: L L^H = B, L A' L^H = A, Q T Q^H = A'.
No test here needs a GPU.
"""
import math

import mpmath
import numpy as np
import pytest
import scipy.linalg as sl
import sympy

import oracle
from inputs import constructed, gue_pair
from tests.metrics import full_hermitian, orthogonality, pair_alignment, residual


def rand_pencil(n, seed, shift=None):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    A = 0.5 * (G + G.conj().T)
    H = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    B = H @ H.conj().T + (n if shift is None else shift) * np.eye(n)
    return A, B


# --------------------------------------------------------------------------- closed forms
def test_n1_closed_form():
    """n = 1: lambda = a/b, x = phase/sqrt(b)."""
    A = np.array([[3.5 + 0j]])
    B = np.array([[2.0 + 0j]])
    W, X, info = oracle.zhegv(A, B)
    assert info == 0
    assert W[0] == pytest.approx(1.75, rel=1e-15)
    assert abs(X[0, 0]) == pytest.approx(1 / math.sqrt(2.0), rel=1e-15)


def test_n2_closed_form():
    """n = 2: roots of (b11 b22 - |b21|^2) l^2 - (a11 b22 + a22 b11 - 2 Re(a21 conj b21)) l
    + (a11 a22 - |a21|^2) = 0."""
    a11, a22, a21 = 1.25, -0.5, 0.3 - 0.7j
    b11, b22, b21 = 2.0, 1.5, 0.2 + 0.4j
    A = np.array([[a11, np.conj(a21)], [a21, a22]])
    B = np.array([[b11, np.conj(b21)], [b21, b22]])
    qa = b11 * b22 - abs(b21) ** 2
    qb = -(a11 * b22 + a22 * b11 - 2 * (a21 * np.conj(b21)).real)
    qc = a11 * a22 - abs(a21) ** 2
    disc = math.sqrt(qb * qb - 4 * qa * qc)
    ref = sorted([(-qb - disc) / (2 * qa), (-qb + disc) / (2 * qa)])
    W, X, info = oracle.zhegv(A, B)
    assert info == 0
    np.testing.assert_allclose(W, ref, rtol=1e-14, atol=0)
    assert orthogonality(B, X) < 1e-14


def test_diagonal_pencil():
    """Diagonal A and B: lambda_i = a_ii / b_ii, eigenvectors are scaled unit vectors."""
    rng = np.random.default_rng(11)
    n = 40
    a = rng.uniform(-3, 3, n)
    b = rng.uniform(0.5, 4, n)
    W, X, info = oracle.zhegv(np.diag(a).astype(complex), np.diag(b).astype(complex))
    assert info == 0
    ref = np.sort(a / b)
    np.testing.assert_allclose(W, ref, rtol=1e-13, atol=1e-15)
    # each column has exactly one entry of modulus 1/sqrt(b_k)
    order = np.argsort(a / b)
    for j, k in enumerate(order):
        col = np.abs(X[:, j])
        assert col[k] == pytest.approx(1 / math.sqrt(b[k]), rel=1e-12)
        assert np.delete(col, k).max() < 1e-12


def test_identity_b_is_standard_problem():
    """B = I reduces to the standard problem: eigenvalues of LAPACK's zheevd (numpy)."""
    A, _ = rand_pencil(60, 5)
    W, X, info = oracle.zhegv(A, np.eye(60, dtype=complex))
    assert info == 0
    np.testing.assert_allclose(W, np.linalg.eigvalsh(A), rtol=0, atol=1e-13 * np.abs(W).max())
    assert orthogonality(np.eye(60), X) < 1e-13 * 60


def test_a_multiple_of_b():
    """A = c B: every eigenvalue equals c and any B-orthonormal basis is correct."""
    _, B = rand_pencil(30, 6)
    c = -0.75
    W, X, info = oracle.zhegv(c * B, B)
    assert info == 0
    np.testing.assert_allclose(W, c, rtol=1e-12)
    assert orthogonality(B, X) < 1e-12


@pytest.mark.parametrize("n", [1, 2, 7, 64, 129])
def test_toeplitz_tridiagonal_closed_form(n):
    """QL stage: tridiag(b, a, b) has lambda_k = a + 2 b cos(k pi/(n+1)) and eigenvectors
    proportional to sin(j k pi/(n+1))."""
    a, b = 0.3, 1.7
    d = np.full(n, a)
    e = np.full(max(n - 1, 0), b)
    w, Z, info = oracle.steql(d, e)
    assert info == 0
    k = np.arange(1, n + 1)
    ref = np.sort(a + 2 * b * np.cos(k * np.pi / (n + 1)))
    np.testing.assert_allclose(w, ref, rtol=0, atol=1e-14 * 4 * abs(b) * n)
    kk = np.argsort(a + 2 * b * np.cos(k * np.pi / (n + 1)))
    j = np.arange(1, n + 1)[:, None]
    S = np.sin(j * (kk[None, :] + 1) * np.pi / (n + 1))
    S /= np.linalg.norm(S, axis=0)
    align = np.abs((S * Z).sum(axis=0))
    assert align.min() > 1 - 1e-12


def test_block_tridiagonal_union_of_spectra():
    """A zero off-diagonal splits T: the spectrum is the union of the blocks' closed forms."""
    n1, n2 = 9, 14
    d = np.concatenate([np.full(n1, 1.0), np.full(n2, -2.0)])
    e = np.concatenate([np.full(n1 - 1, 0.5), [0.0], np.full(n2 - 1, 0.25)])
    w, Z, info = oracle.steql(d, e)
    assert info == 0
    ref = np.sort(np.concatenate([
        1.0 + 1.0 * np.cos(np.arange(1, n1 + 1) * np.pi / (n1 + 1)),
        -2.0 + 0.5 * np.cos(np.arange(1, n2 + 1) * np.pi / (n2 + 1))]))
    np.testing.assert_allclose(w, ref, atol=1e-14 * 4)
    np.testing.assert_allclose(Z.T @ Z, np.eye(n1 + n2), atol=1e-13)


# --------------------------------------------------------------------------- brute force
def _exact_pencil(n, seed):
    rng = np.random.default_rng(seed)
    Ar = rng.integers(-4, 5, (n, n))
    Ai = rng.integers(-4, 5, (n, n))
    A = np.tril(Ar + 1j * Ai, -1)
    A = A + A.conj().T + np.diag(rng.integers(-4, 5, n))
    Lr = rng.integers(-2, 3, (n, n))
    Li = rng.integers(-2, 3, (n, n))
    L = np.tril(Lr + 1j * Li, -1) + np.diag(rng.integers(1, 4, n))
    B = L @ L.conj().T                     # exact: small Gaussian integers
    return A.astype(complex), B.astype(complex)


@pytest.mark.parametrize("n,seed", [(2, 1), (3, 2), (4, 3), (5, 4)])
def test_brute_force_small(n, seed):
    """n <= 5 Gaussian-integer pencil: eigenvalues are the roots of the exact polynomial
    det(A - lambda B); eigenvectors span the 40-digit null space of A - lambda B."""
    A, B = _exact_pencil(n, seed)
    lam = sympy.symbols("lam")
    As = sympy.Matrix(n, n, lambda i, j: sympy.Integer(int(A[i, j].real)) + sympy.I * int(A[i, j].imag))
    Bs = sympy.Matrix(n, n, lambda i, j: sympy.Integer(int(B[i, j].real)) + sympy.I * int(B[i, j].imag))
    p = sympy.Poly(sympy.expand((As - lam * Bs).det(method="berkowitz")), lam)
    coeffs = [sympy.nsimplify(c) for c in p.all_coeffs()]
    assert all(sympy.im(c) == 0 for c in coeffs)
    roots40 = sorted((sympy.re(r) for r in sympy.Poly([sympy.re(c) for c in coeffs], lam).nroots(n=40)),
                     key=float)
    roots = [float(r) for r in roots40]
    W, X, info = oracle.zhegv(A, B)
    assert info == 0
    np.testing.assert_allclose(W, roots, rtol=1e-12, atol=1e-12 * max(abs(r) for r in roots))
    mpmath.mp.dps = 40
    Bm = mpmath.matrix(B.tolist())
    Am = mpmath.matrix(A.tolist())
    for j, r in enumerate(roots40):
        M = Am - mpmath.mpf(str(r)) * Bm
        # null vector of A - lambda B at the 40-digit root: the right singular vector of
        # the smallest singular value
        _, S, Vh = mpmath.svd_c(M)
        v = Vh.H[:, n - 1]
        nb = mpmath.sqrt(abs((v.H * Bm * v)[0]))
        v = np.array([complex(v[i] / nb) for i in range(n)])
        align = abs(np.vdot(X[:, j], B @ v))
        assert align > 1 - 1e-10


# --------------------------------------------------------------------------- constructed spectra
@pytest.mark.parametrize("n,spectrum,seed", [(64, "uniform", 0), (200, "loguniform", 2), (512, "uniform", 0)])
def test_constructed_spectrum(n, spectrum, seed):
    """A = L Q D Q^H L^H, B = L L^H: lambda = sort(D); Q_pi^H L^H X is a diagonal unitary."""
    A, B, parts = constructed(n, seed, spectrum, return_parts=True)
    A, B = A.numpy(), B.numpy()
    D = parts["D"]
    Q = parts["Q"].numpy()
    L = parts["L"].numpy()
    W, X, info = oracle.zhegv(A, B)
    assert info == 0
    order = np.argsort(D)
    np.testing.assert_allclose(W, D[order], rtol=0, atol=1e-13 * np.abs(D).max())
    M = Q[:, order].conj().T @ (L.conj().T @ X)
    diag = np.abs(np.diag(M))
    gaps = np.minimum(np.abs(np.diff(D[order], prepend=-np.inf)), np.abs(np.diff(D[order], append=np.inf)))
    assert diag.min() > 1 - 1e-9
    off = np.abs(M - np.diag(np.diag(M)))
    assert (off.max(axis=0) * np.minimum(gaps, 1.0)).max() < 1e-11


def test_config0_invariants():
    """Plain FP64 bars: res <= 1e-14 and ||X^H B X - I||_1 <= 1e-13 n on the n = 512 pencil."""
    A, B = constructed(512, 0, "uniform")
    A, B = A.numpy(), B.numpy()
    W, X, info = oracle.zhegv(A, B)
    assert info == 0
    assert residual(A, B, W, X) <= 1e-14
    assert orthogonality(B, X) <= 1e-13 * 512


# --------------------------------------------------------------------------- library cross-check
@pytest.mark.parametrize("il,iu", [(1, 150), (11, 40), (150, 150)])
def test_scipy_cross_check(il, iu):
    """LAPACK zhegvd / zhegvx (scipy) as an independent implementation."""
    A, B = gue_pair(150, 9, cond_b=1e3)
    A, B = A.numpy(), B.numpy()
    W, X, info = oracle.zhegv(A, B, il, iu)
    assert info == 0
    Wr, Xr = sl.eigh(A, B, subset_by_index=[il - 1, iu - 1])
    np.testing.assert_allclose(W, Wr, rtol=0, atol=1e-13 * np.abs(Wr).max())
    gaps = np.abs(np.diff(sl.eigh(A, B, eigvals_only=True)))
    if gaps.min() > 1e-6:
        assert pair_alignment(B, X, Xr).min() > 1 - 1e-9


def test_subset_equals_columns_of_full():
    """Selecting il..iu gives the same pairs (up to phase) as the columns of the full solve."""
    A, B = rand_pencil(80, 12)
    W, X, _ = oracle.zhegv(A, B)
    Ws, Xs, info = oracle.zhegv(A, B, 17, 33)
    assert info == 0
    np.testing.assert_array_equal(Ws, W[16:33])
    assert pair_alignment(B, Xs, X[:, 16:33]).min() > 1 - 1e-12


# --------------------------------------------------------------------------- stage identities
def test_potrf_matches_numpy_cholesky():
    """The Cholesky factor with positive real diagonal is unique: LAPACK's (numpy) must agree."""
    _, B = rand_pencil(90, 13)
    L, info = oracle.potrf(np.tril(B))
    assert info == 0
    np.testing.assert_allclose(L, np.linalg.cholesky(B), rtol=0, atol=1e-13 * np.abs(B).max())
    assert np.all(np.triu(L, 1) == 0)


def test_potrf_not_pd_minor():
    """Non-PD leading minor of order k gives info = k."""
    B = np.diag([1.0, 2.0, -1.0, 3.0]).astype(complex)
    _, info = oracle.potrf(B)
    assert info == 3


def test_hegst_identity():
    """L A' L^H = A with A' Hermitian (Algorithm 1 step 2)."""
    A, B = rand_pencil(70, 14)
    L, _ = oracle.potrf(B)
    C = oracle.hegst(np.tril(A), L)
    np.testing.assert_array_equal(C, C.conj().T)
    np.testing.assert_allclose(L @ C @ L.conj().T, A, rtol=0, atol=1e-12 * np.abs(A).max())


def test_hegst_reads_lower_triangle_only():
    """Garbage in the strict upper triangle of A must not change A'."""
    A, B = rand_pencil(33, 15)
    L, _ = oracle.potrf(B)
    junk = np.triu(np.random.default_rng(1).standard_normal((33, 33)) * 1e3, 1)
    np.testing.assert_array_equal(oracle.hegst(np.tril(A), L), oracle.hegst(np.tril(A) + junk, L))


@pytest.mark.parametrize("n", [3, 4, 50])
def test_hetrd_reconstruction(n):
    """Algorithm 2 step 1: C = Q Psi T Psi^H Q^H with Q = H_0 ... H_{n-3} unitary."""
    A, _ = rand_pencil(n, 16)
    d, e, U, beta, psi = oracle.hetrd(A)
    Q = np.eye(n, dtype=complex)
    for k in range(n - 2):
        u = U[:, k]
        Q = Q @ (np.eye(n) - beta[k] * np.outer(u, u.conj()))
    T = np.diag(d) + np.diag(e, -1) + np.diag(e, 1)
    P = np.diag(psi)
    np.testing.assert_allclose(Q @ P @ T @ P.conj().T @ Q.conj().T, A, atol=1e-13 * np.abs(A).max() * n)
    np.testing.assert_allclose(Q.conj().T @ Q, np.eye(n), atol=1e-14 * n)
    assert np.all(e >= 0)
    np.testing.assert_allclose(np.linalg.eigvalsh(T), np.linalg.eigvalsh(A), atol=1e-13 * n)


def test_full_pipeline_identities_random():
    """Random pencil: residual / orthogonality bars and LAPACK eigenvalues."""
    A, B = rand_pencil(257, 17)
    W, X, info = oracle.zhegv(A, B)
    assert info == 0
    assert residual(A, B, W, X) <= 1e-15
    assert orthogonality(B, X) <= 1e-13 * 257
    np.testing.assert_allclose(W, sl.eigh(A, B, eigvals_only=True), atol=1e-13 * np.abs(W).max())


def test_reads_lower_triangles_only():
    """The solver reads only the lower triangles of A and B."""
    A, B = rand_pencil(25, 18)
    junk = np.triu(np.random.default_rng(2).standard_normal((25, 25)), 1) * 7
    W1, X1, _ = oracle.zhegv(A, B)
    W2, X2, _ = oracle.zhegv(np.tril(A) + junk, np.tril(B) - junk)
    np.testing.assert_array_equal(W1, W2)
    np.testing.assert_array_equal(X1, X2)


# --------------------------------------------------------------------------- failure reporting
def test_not_pd_b_reports_n_plus_k():
    n = 6
    A, _ = rand_pencil(n, 19)
    B = np.diag([1.0, 1.0, -1.0, 1.0, 1.0, 1.0]).astype(complex)
    _, _, info = oracle.zhegv(A, B)
    assert info == n + 3


def test_nan_in_b_reports_not_pd():
    n = 5
    A, B = rand_pencil(n, 20)
    B[0, 0] = np.nan
    _, _, info = oracle.zhegv(A, B)
    assert info == n + 1


def test_ql_failure_reported():
    A, B = rand_pencil(12, 21)
    oracle.set_ql_maxit(0)
    try:
        _, _, info = oracle.zhegv(A, B)
    finally:
        oracle.set_ql_maxit(30)
    assert 1 <= info <= 12


@pytest.mark.parametrize("il,iu,code", [(0, 3, -6), (3, 2, -7), (1, 9, -7)])
def test_bad_range_arguments(il, iu, code):
    A, B = rand_pencil(8, 22)
    _, _, info = oracle.zhegv(A, B, il, iu)
    assert info == code


def test_literal_l_recipe_loses_definiteness():
    """Negative result: with strict-lower std 0.1 at every n, cond(B) explodes (B = L L^H)."""
    _, B_lit = constructed(1024, 0, literal_l=True)
    _, B_fix = constructed(1024, 0)
    c_lit = np.linalg.cond(B_lit.numpy())
    c_fix = np.linalg.cond(B_fix.numpy())
    assert c_lit > 1e7 and c_fix < 1e6 and c_lit > 100 * c_fix
