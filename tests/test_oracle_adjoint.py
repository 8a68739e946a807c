"""Pins of the oracle's dense reference gradient (oracle/adjoint.py).

* Central finite differences of the loss, evaluated with independent oracle forward
  solves, along random Hermitian directions of A and of B.
* Closed form for a diagonal pencil: lambda_i = a_i / b_i, so dL/da_i = w_i / b_i and
  dL/db_i = -w_i a_i / b_i^2 for the eigenvalue part.
* Hellmann-Feynman: with no eigenvector cotangent, Abar = X diag(w) X^H.
"""
import numpy as np
import pytest

from oracle import adjoint


def rand_pencil(n, seed):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    A = 0.5 * (G + G.conj().T)
    H = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    B = H @ H.conj().T + n * np.eye(n)
    return A, B


def rand_herm_dir(n, seed):
    rng = np.random.default_rng(seed)
    E = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    E = 0.5 * (E + E.conj().T)
    return E / np.linalg.norm(E)


@pytest.mark.parametrize("n,il,iu,seed", [(8, 1, 8, 1), (10, 2, 5, 2), (12, 7, 7, 3)])
def test_gradient_matches_central_differences(n, il, iu, seed):
    A, B = rand_pencil(n, seed)
    m = iu - il + 1
    rng = np.random.default_rng(seed + 100)
    w = rng.standard_normal(m)
    G = rng.standard_normal((n, m)) + 1j * rng.standard_normal((n, m))
    Abar, Bbar = adjoint.gradient(A, B, il, iu, w, G)
    np.testing.assert_allclose(Abar, Abar.conj().T, atol=1e-14)
    np.testing.assert_allclose(Bbar, Bbar.conj().T, atol=1e-14)
    h = 1e-5
    for t in range(3):
        E = rand_herm_dir(n, 1000 * seed + t)
        fd = (adjoint.loss(A + h * E, B, il, iu, w, G) - adjoint.loss(A - h * E, B, il, iu, w, G)) / (2 * h)
        an = np.real(np.sum(Abar.conj() * E))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)
        F = rand_herm_dir(n, 2000 * seed + t)
        fd = (adjoint.loss(A, B + h * F, il, iu, w, G) - adjoint.loss(A, B - h * F, il, iu, w, G)) / (2 * h)
        an = np.real(np.sum(Bbar.conj() * F))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)


def test_diagonal_pencil_closed_form():
    rng = np.random.default_rng(4)
    n = 6
    a = np.array([3.0, -1.0, 0.5, 2.0, -2.5, 1.2])
    b = rng.uniform(0.5, 2.0, n)
    A, B = np.diag(a).astype(complex), np.diag(b).astype(complex)
    order = np.argsort(a / b)
    w = rng.standard_normal(n)
    Abar, Bbar = adjoint.gradient(A, B, 1, n, w, np.zeros((n, n), complex))
    for j, k in enumerate(order):
        assert Abar[k, k].real == pytest.approx(w[j] / b[k], rel=1e-13)
        assert Bbar[k, k].real == pytest.approx(-w[j] * a[k] / b[k] ** 2, rel=1e-13)
    off = Abar - np.diag(np.diag(Abar))
    assert np.abs(off).max() < 1e-14


def test_hellmann_feynman():
    A, B = rand_pencil(15, 9)
    w = np.random.default_rng(1).standard_normal(4)
    Abar, Bbar = adjoint.gradient(A, B, 3, 6, w, np.zeros((15, 4), complex))
    lam, Xall = adjoint.solve(A, B, 3, 6)
    X = Xall[:, 2:6]
    np.testing.assert_allclose(Abar, (X * w) @ X.conj().T, atol=1e-14)
    np.testing.assert_allclose(Bbar, -(X * (w * lam[2:6])) @ X.conj().T, atol=1e-13)
