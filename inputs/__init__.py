"""Seeded synthetic Hermitian-definite pencils (A, B) shared by the tests, the
smoke check and the benchmark.

This module holds no eigensolver arithmetic: it only draws random numbers
(numpy PCG64, fixed seeds and draw order) and multiplies matrices to build
pencils with known structure.  The matrix products run in torch, on the CPU for
small sizes or on a GPU device when one is passed (building an n = 10000 pencil
on the host would take minutes).

Recipes (the paper's workloads are electronic-structure pencils that are not
available; these synthetic pencils stand in for them):

* ``constructed(n, seed, spectrum)``: A = L Q diag(D) Q^H L^H, B = L L^H, so the
  pencil's eigenvalues are exactly D and X = L^-H Q (up to order and phase).
  Q is the product of n Householder reflectors with complex Gaussian vectors;
  L is lower triangular with diagonal U[1, 2] and strict-lower entries
  N(0, s^2) + i N(0, s^2) with s = 0.1 * sqrt(512 / n).  At n = 512 this is the
  literal recipe (s = 0.1); keeping s at 0.1 for larger n makes cond(B) grow
  exponentially (about 1e12 at n = 2048), so B stops being numerically
  definite.  ``literal_l=True`` keeps s = 0.1 for recording that failure.
  spectrum "uniform": D ~ U[-1, 1]; "loguniform": |D| = 10^U(-3, 1), random sign.
* ``gue_pair(n, seed, cond_b)``: A = (G + G^H)/2, G complex Gaussian; B = U diag(s) U^H
  with U Haar-unitary and s log-spaced over [1, cond_b].
* ``batch_sizes(count, seed)``: problem orders drawn uniformly from [500, 3000].
"""
import math

import numpy as np
import torch


def _to(x, device):
    return torch.as_tensor(x).to(device)


def householder_product(V, block=64):
    """Q = H_1 H_2 ... H_k for H_j = I - 2 v_j v_j^H / (v_j^H v_j), v_j = V[:, j].

    Blocks of reflectors are multiplied in the accumulated form P = I + W Y^H
    (Bischof & Van Loan), w_j = -beta_j (v_j + W (Y^H v_j)), then Q <- Q + (Q W) Y^H."""
    n, k = V.shape
    Q = torch.eye(n, dtype=V.dtype, device=V.device)
    for j0 in range(0, k, block):
        Y = V[:, j0:j0 + block]
        b = Y.shape[1]
        W = torch.zeros_like(Y)
        for j in range(b):
            v = Y[:, j]
            beta = 2.0 / torch.vdot(v, v).real
            if j == 0:
                W[:, 0] = -beta * v
            else:
                W[:, j] = -beta * (v + W[:, :j] @ (Y[:, :j].conj().T @ v))
        Q = Q + (Q @ W) @ Y.conj().T
    return Q


def _l_factor(rng, n, literal_l):
    diag = rng.uniform(1.0, 2.0, n)
    s = 0.1 if literal_l else 0.1 * math.sqrt(512.0 / n)
    lr = rng.normal(0.0, s, (n, n))
    li = rng.normal(0.0, s, (n, n))
    L = np.tril(lr + 1j * li, -1)
    L[np.diag_indices(n)] = diag
    return L


def constructed(n, seed, spectrum="uniform", device="cpu", literal_l=False, return_parts=False):
    """Pencil with known spectrum D (draw order: D, V real, V imag, L diag, L strict-lower)."""
    rng = np.random.default_rng(seed)
    if spectrum == "uniform":
        D = rng.uniform(-1.0, 1.0, n)
    elif spectrum == "loguniform":
        mag = 10.0 ** rng.uniform(-3.0, 1.0, n)
        sign = np.where(rng.random(n) < 0.5, -1.0, 1.0)
        D = sign * mag
    else:
        raise ValueError(spectrum)
    V = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    L = _l_factor(rng, n, literal_l)
    Vt = _to(V, device)
    del V
    Q = householder_product(Vt)
    del Vt
    Lt = _to(L, device)
    Dt = _to(D, device).to(torch.complex128)
    LQ = Lt @ Q
    A = (LQ * Dt) @ LQ.conj().T
    A = 0.5 * (A + A.conj().T)
    B = Lt @ Lt.conj().T
    B = 0.5 * (B + B.conj().T)
    if return_parts:
        return A, B, {"D": D, "Q": Q, "L": Lt}
    return A, B


def haar_unitary(rng, n, device="cpu"):
    """Haar unitary from the QR of a complex Gaussian, R's diagonal phases moved into Q."""
    Z = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    Zt = _to(Z, device)
    Qz, Rz = torch.linalg.qr(Zt)
    ph = torch.diagonal(Rz)
    ph = ph / ph.abs()
    return Qz * ph


def gue_pair(n, seed, cond_b=1e3, device="cpu"):
    """A = (G + G^H)/2; B = U diag(logspace(0, log10 cond_b, n)) U^H (draw order: G re, G im, U)."""
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    Gt = _to(G, device)
    A = 0.5 * (Gt + Gt.conj().T)
    U = haar_unitary(rng, n, device)
    s = torch.as_tensor(np.logspace(0.0, math.log10(cond_b), n), device=device).to(torch.complex128)
    B = (U * s) @ U.conj().T
    B = 0.5 * (B + B.conj().T)
    return A, B


def batch_sizes(count=64, seed=3, lo=500, hi=3000):
    """Orders of the batched workload: uniform integers in [lo, hi]."""
    return [int(x) for x in np.random.default_rng(seed).integers(lo, hi + 1, count)]


def batch_problem(i, n, seed=3, cond_b=1e2, device="cpu"):
    """Problem i of the batched workload: the GUE recipe seeded with [seed, i]."""
    return gue_pair(n, [seed, i], cond_b=cond_b, device=device)


def adjoint_cotangents(n, m, seed=4):
    """Loss weights for the differentiable solve: w ~ N(0,1)^m, G = N(0,1) + i N(0,1) (n x m)."""
    rng = np.random.default_rng([seed, 1])
    w = rng.standard_normal(m)
    G = rng.standard_normal((n, m)) + 1j * rng.standard_normal((n, m))
    return w, G


def hermitian_lower_noise(n, seed):
    """Small complex Gaussian n x n matrix (used to fill the unread upper triangle in tests)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
