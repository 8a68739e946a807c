"""Accuracy measures shared by the tests (plain numpy, fp64).

res  = ||A X - B X diag(W)||_1 / (n ||A||_1 ||X||_1)      (backward-error style residual)
orth = ||X^H B X - I||_1                                    (B-orthonormality)
Norms are matrix 1-norms (largest absolute column sum), A is the full Hermitian
matrix, X the n x m selected eigenvectors, n the full order.
"""
import numpy as np


def norm1(M):
    M = np.asarray(M)
    if M.size == 0:
        return 0.0
    return float(np.abs(M).sum(axis=0).max())


def full_hermitian(M):
    """Full Hermitian matrix from the lower triangle of M (diagonal made real)."""
    M = np.asarray(M)
    L = np.tril(M, -1)
    return L + L.conj().T + np.diag(np.diag(M).real)


def residual(A, B, W, X):
    n = A.shape[0]
    R = A @ X - (B @ X) * W[None, :]
    den = n * norm1(A) * norm1(X)
    return norm1(R) / den if den > 0 else norm1(R)


def orthogonality(B, X):
    m = X.shape[1]
    return norm1(X.conj().T @ B @ X - np.eye(m))


def pair_alignment(B, X, Y):
    """|x_i^H B y_i| per column: 1 when the two B-normalised vectors agree up to phase."""
    return np.abs(np.einsum("ij,ij->j", X.conj(), B @ Y))


def subspace_distance(B, X, Y):
    """sin of the largest principal angle between span(X) and span(Y) in the B inner product
    (both B-orthonormal): ||(I - X X^H B) Y||_2 measured as ||Y - X (X^H B Y)||_B."""
    P = Y - X @ (X.conj().T @ (B @ Y))
    G = P.conj().T @ (B @ P)
    return float(np.sqrt(max(np.linalg.eigvalsh(0.5 * (G + G.conj().T)).max(), 0.0)))
