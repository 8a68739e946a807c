"""GPU checks of the two-stage tridiagonalisation (Alg. 2 step 1, Sec. 4.2) and of the
two back-transformation steps (Alg. 2 step 3).

The band matrix, the tridiagonal and the reflectors are not unique (they depend on the
reflector convention and blocking), so these stages are checked through properties that
hold for any correct implementation:
  * he2hb: exact zeros outside the band, A' = Q1 Band Q1^H, Q1 unitary;
  * hb2st: eig(T) = eig(Band), Band = Q2 T Q2^H, Q2 unitary, T real;
  * the bulge-chasing schedule is pipelined across workgroups, yet every task's
    arithmetic is fixed, so repeated runs are bitwise identical.
Tolerance: a product of O(n) reflectors perturbs by O(n eps) relative; the tests use
1e-13 * max(1, n/100) relative Frobenius error.
"""
import numpy as np
import pytest

import oracle
from tests.gpu_util import rand_herm, rand_hpd, rel_fro, require_gpu, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    hgv = require_gpu()
    return hgv.Context.get("cuda:0")


def _tol(n):
    return 1e-13 * max(1.0, n / 100.0)


def band_part(M, b):
    n = M.shape[0]
    i, j = np.indices((n, n))
    L = np.where((i - j >= 0) & (i - j <= b), M, 0)
    return L + np.tril(L, -1).conj().T


def random_band(n, b, seed):
    A = rand_herm(n, seed)
    B = band_part(np.tril(A), b)
    return B


@pytest.fixture(params=["fixed", "householder"])
def panels(request, ctx):
    """The two forms of the band reduction's panel QR: Cholesky QR twice with
    Householder reconstruction where the panel allows it (the default), or the
    Householder column steps for every panel."""
    import paper_1207_1773_amd as hgv
    hgv.hgv_test_hooks(ctx.handle, hgv.HGV_TEST_HOUSEHOLDER_PANELS if request.param == "householder" else 0)
    yield request.param
    hgv.hgv_test_hooks(ctx.handle, 0)


def check_he2hb(ctx, A, nb):
    """A' = Q1 Band Q1^H, Q1 unitary, eig(Band) = eig(A'); returns the band."""
    n = A.shape[0]
    Ab, T1 = ctx.he2hb(to_dev(np.tril(A)), nb)
    band = band_part(to_np(Ab), nb)
    Q1 = to_np(ctx.q1(Ab, T1, to_dev(np.eye(n, dtype=complex)), nb))
    scale = max(np.abs(A).max(), 1e-300)
    assert np.linalg.norm(Q1 @ band @ Q1.conj().T - A) <= _tol(n) * max(np.linalg.norm(A), scale)
    assert np.linalg.norm(Q1.conj().T @ Q1 - np.eye(n)) < _tol(n) * np.sqrt(n)
    np.testing.assert_allclose(np.linalg.eigvalsh(band), np.linalg.eigvalsh(A), atol=_tol(n) * scale * n)
    return band


def panel_diagonals(band, n, nb):
    """Entry (k + nb + i, k + i) of the band for every panel k and i < nb: the diagonal
    of the panel's triangular factor (real for the Householder column steps)."""
    out = []
    for k in range(0, n - nb - 1, nb):
        r = min(nb, n - k - nb)
        out.append(np.array([band[k + nb + i, k + i] for i in range(r)]))
    return out


@pytest.mark.parametrize("n,nb", [(1, 4), (2, 1), (5, 3), (40, 8), (100, 32), (129, 16), (300, 32), (513, 32),
                                  (200, 64), (97, 1), (130, 64), (256, 48), (128, 64), (96, 32)])
def test_he2hb_reconstruction(ctx, panels, n, nb):
    A = rand_herm(n, 100 + n)
    band = check_he2hb(ctx, A, nb)
    diags = panel_diagonals(band, n, nb)
    if panels == "householder":
        assert all(np.all(d.imag == 0) for d in diags)
    elif diags and n - nb >= nb:
        # the first panel (at least nb rows below the band) takes the fixed-launch form,
        # whose triangular factor has complex diagonal entries
        assert np.any(diags[0].imag != 0)


def _fallback_inputs(n, nb):
    rng = np.random.default_rng(7)
    A = rand_herm(n, 41)
    rankdef = A.copy()   # panel 0: two equal columns below the band
    rankdef[nb:, 1] = rankdef[nb:, 0]
    rankdef = np.tril(rankdef) + np.tril(rankdef, -1).conj().T
    graded = A.copy()    # panel 0: columns scaled from 1 to 1e-9 (condition number ~1e9)
    graded[nb:, :nb] *= np.logspace(0, -9, nb)[None, :]
    graded = np.tril(graded) + np.tril(graded, -1).conj().T
    nearpar = A.copy()   # panel 0: two nearly parallel columns (condition number ~2e4): its
    nearpar[nb:, 1] = nearpar[nb:, 0] + 1e-4 * nearpar[nb:, 1]   # Gram matrix factors, but
    nearpar = np.tril(nearpar) + np.tril(nearpar, -1).conj().T   # one pass leaves |G2 - I| ~ 1e-8
    blockdiag = A.copy()  # panel 0 identically zero below the band
    blockdiag[nb:, :nb] = 0
    blockdiag = np.tril(blockdiag) + np.tril(blockdiag, -1).conj().T
    diag = np.diag(rng.standard_normal(n)).astype(complex)   # every panel zero
    return {"rank_deficient": rankdef, "graded": graded, "near_parallel": nearpar, "zero_panel": blockdiag,
            "diagonal": diag}


@pytest.mark.parametrize("kind", ["rank_deficient", "near_parallel", "zero_panel"])
def test_solve_with_mixed_panel_forms(ctx, kind):
    """A whole solve (B = 2I, so A' = A/2 keeps the panel structure) whose band reduction
    takes the column steps for its first panel and the fixed-launch form for the rest:
    eigenvalues against the oracle at the FP64 bars, residual and B-orthogonality."""
    from tests.metrics import orthogonality, residual
    n, nb = 300, 32
    A = _fallback_inputs(n, nb)[kind]
    B = 2.0 * np.eye(n, dtype=complex)
    W, X, info, _ = ctx.zhegvx(to_dev(A), to_dev(B), 1, n, nb=nb)
    assert info == 0
    W, X = to_np(W), to_np(X)
    Wo, _, _ = oracle.zhegv(A, B, 1, n)
    np.testing.assert_allclose(W, Wo, rtol=0, atol=1e-12 * np.abs(Wo).max())
    assert residual(A, B, W, X) <= 1e-14
    assert orthogonality(B, X) <= 1e-13 * n


@pytest.mark.parametrize("kind", ["rank_deficient", "graded", "near_parallel", "zero_panel", "diagonal"])
def test_he2hb_panel_fallback(ctx, kind):
    """Panels that Cholesky QR cannot factor accurately (rank deficient; condition number
    beyond 1e5, caught when G1 is factored; nearly parallel columns, caught by the second
    Gram matrix; zero) are factored by the column steps, chosen on the device; the later
    panels of the same reduction still take the fixed-launch form."""
    n, nb = 300, 32
    A = _fallback_inputs(n, nb)[kind]
    band = check_he2hb(ctx, A, nb)
    diags = panel_diagonals(band, n, nb)
    assert np.all(diags[0].imag == 0)   # the first panel: column steps
    if kind != "diagonal":
        assert np.any(diags[1].imag != 0)   # the next one: fixed-launch form


@pytest.fixture(params=["owners", "sweeps"])
def schedule(request, ctx):
    """The two bulge-chasing schedules: one workgroup per window for all sweeps (the
    default), or one workgroup per sweep (used when the windows do not all fit)."""
    import paper_1207_1773_amd as hgv
    hgv.hgv_test_hooks(ctx.handle, hgv.HGV_TEST_HB2ST_SWEEPS if request.param == "sweeps" else 0)
    yield request.param
    hgv.hgv_test_hooks(ctx.handle, 0)


@pytest.mark.parametrize("n,b", [(1, 3), (2, 1), (3, 2), (10, 3), (64, 8), (100, 32), (101, 7), (257, 16),
                                 (300, 32), (150, 64), (130, 64), (129, 64), (200, 48), (66, 33), (7, 64)])
def test_hb2st_properties(ctx, schedule, n, b):
    band = random_band(n, b, 200 + n)
    d, e, V2, tau2 = ctx.hb2st(to_dev(band), b)
    d, e = to_np(d), to_np(e)
    T = np.diag(d) + np.diag(e, -1) + np.diag(e, 1)
    np.testing.assert_allclose(np.linalg.eigvalsh(T), np.linalg.eigvalsh(band),
                               atol=_tol(n) * np.abs(band).max() * max(n, 1))
    Q2 = to_np(ctx.q2(V2, tau2, to_dev(np.eye(n, dtype=complex)), b))
    assert rel_fro(Q2 @ T @ Q2.conj().T, band) < _tol(n)
    assert np.linalg.norm(Q2.conj().T @ Q2 - np.eye(n)) < _tol(n) * np.sqrt(n)


@pytest.mark.parametrize("n,b", [(700, 32), (1500, 64)])
def test_hb2st_bitwise_repeatable(ctx, schedule, n, b):
    band = random_band(n, b, 7)
    runs = [ctx.hb2st(to_dev(band), b) for _ in range(3)]
    for r in runs[1:]:
        for x, y in zip(runs[0], r):
            assert torch_equal(x, y)


@pytest.mark.parametrize("n,b", [(1000, 64), (777, 32), (500, 48)])
def test_hb2st_schedules_agree(ctx, n, b):
    """Both schedules apply the same reflectors in the same order (only the summation
    order inside a task differs), so T and Q2 agree to rounding."""
    import paper_1207_1773_amd as hgv
    band = random_band(n, b, 11 + n)
    out = {}
    for mode in (0, hgv.HGV_TEST_HB2ST_SWEEPS):
        hgv.hgv_test_hooks(ctx.handle, mode)
        try:
            d, e, V2, tau2 = ctx.hb2st(to_dev(band), b)
        finally:
            hgv.hgv_test_hooks(ctx.handle, 0)
        out[mode] = (to_np(d), to_np(e), to_np(V2), to_np(tau2))
    (d0, e0, V0, t0), (d1, e1, V1, t1) = out[0], out[hgv.HGV_TEST_HB2ST_SWEEPS]
    scale = np.abs(band).max() * n
    assert np.abs(d0 - d1).max() < 1e-13 * scale
    assert np.abs(e0 - e1).max() < 1e-13 * scale
    assert np.abs(V0 - V1).max() < 1e-10 and np.abs(t0 - t1).max() < 1e-10


def torch_equal(x, y):
    import torch
    return bool(torch.equal(x.view(torch.float64) if x.is_complex() else x,
                            y.view(torch.float64) if y.is_complex() else y))


@pytest.mark.parametrize("n,nb,m", [(300, 32, 7), (257, 16, 257), (64, 8, 1), (300, 64, 40), (200, 48, 33)])
def test_q2_q1_on_rectangular_blocks(ctx, n, nb, m):
    """Back-transformations applied to an n x m block equal the same columns of Q applied to I."""
    band = random_band(n, nb, 300 + n)
    d, e, V2, tau2 = ctx.hb2st(to_dev(band), nb)
    rng = np.random.default_rng(n)
    Y = rng.standard_normal((n, m)) + 1j * rng.standard_normal((n, m))
    Q2 = to_np(ctx.q2(V2, tau2, to_dev(np.eye(n, dtype=complex)), nb))
    QY = to_np(ctx.q2(V2, tau2, to_dev(Y), nb))
    assert rel_fro(QY, Q2 @ Y) < _tol(n)


@pytest.mark.parametrize("n,nb", [(200, 64), (150, 32)])
def test_q2_many_columns_and_adjoint(ctx, n, nb):
    """Q2 on 8300 columns (the per-group kernel; fewer columns take the LDS super-block
    kernel) equals the explicit Q2 formed on the identity, and Q2^H undoes Q2 on both."""
    band = random_band(n, nb, 700 + n)
    d, e, V2, tau2 = ctx.hb2st(to_dev(band), nb)
    Q2 = to_np(ctx.q2(V2, tau2, to_dev(np.eye(n, dtype=complex)), nb))
    rng = np.random.default_rng(n + 1)
    for m in (8300, 37):
        Y = rng.standard_normal((n, m)) + 1j * rng.standard_normal((n, m))
        QY = to_np(ctx.q2(V2, tau2, to_dev(Y), nb))
        assert rel_fro(QY, Q2 @ Y) < _tol(n)
        QhY = to_np(ctx.q2(V2, tau2, to_dev(Y), nb, adj=True))
        assert rel_fro(QhY, Q2.conj().T @ Y) < _tol(n)
        back = to_np(ctx.q2(V2, tau2, to_dev(QY), nb, adj=True))
        assert rel_fro(back, Y) < _tol(n)


@pytest.mark.parametrize("n,nb,m", [(300, 32, 20), (700, 64, 9), (260, 16, 300)])
def test_q1_adjoint(ctx, n, nb, m):
    """Q1^H Q1 Y = Y and Q1^H Y equals the explicit Q1^H (merged-panel application)."""
    A = rand_herm(n, 900 + n)
    Ab, T1 = ctx.he2hb(to_dev(np.tril(A)), nb)
    Q1 = to_np(ctx.q1(Ab, T1, to_dev(np.eye(n, dtype=complex)), nb))
    rng = np.random.default_rng(m)
    Y = rng.standard_normal((n, m)) + 1j * rng.standard_normal((n, m))
    QY = to_np(ctx.q1(Ab, T1, to_dev(Y), nb))
    assert rel_fro(QY, Q1 @ Y) < _tol(n)
    QhY = to_np(ctx.q1(Ab, T1, to_dev(Y), nb, adj=True))
    assert rel_fro(QhY, Q1.conj().T @ Y) < _tol(n)
    assert rel_fro(to_np(ctx.q1(Ab, T1, to_dev(QY), nb, adj=True)), Y) < _tol(n)
    # Q1 is unitary
    assert rel_fro(Q1.conj().T @ Q1, np.eye(n)) < _tol(n)


def test_two_stage_eigenvalues_match_oracle(ctx):
    """he2hb + hb2st on A' = L^-1 A L^-H keeps the oracle's eigenvalues of the pencil."""
    n, nb = 400, 32
    A = rand_herm(n, 1)
    B = rand_hpd(n, 2)
    W, X, info = oracle.zhegv(A, B)
    assert info == 0
    L, _ = ctx.potrf(to_dev(np.tril(B)))
    Ap = ctx.hegst(to_dev(np.tril(A)), L)
    Ab, T1 = ctx.he2hb(Ap, nb)
    d, e, V2, tau2 = ctx.hb2st(Ab, nb)
    d, e = to_np(d), to_np(e)
    T = np.diag(d) + np.diag(e, -1) + np.diag(e, 1)
    np.testing.assert_allclose(np.linalg.eigvalsh(T), W, atol=1e-12 * np.abs(W).max())
