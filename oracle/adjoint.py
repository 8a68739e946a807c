"""Dense fp64 reference gradient of the generalized eigensolve (test infrastructure).

For the loss  L = sum_i wbar_i lambda_i + Re sum_i gbar_i^H x_i  over the selected pairs
il..iu (x_i B-normalised, gauge fixed so that the entry of largest modulus of x_i,
k_i = argmax_r |x_ri| with the smallest r on ties, is real and positive), the gradient with
respect to Hermitian A and B (dL = Re tr(Abar^H dA) + Re tr(Bbar^H dB)) follows from
first-order perturbation theory of A x = lambda B x, x^H B x = 1:

  d lambda_i = x_i^H (dA - lambda_i dB) x_i,
  dx_i = sum_{j != i} x_j x_j^H (dA - lambda_i dB) x_i / (lambda_i - lambda_j)
         - 1/2 x_i (x_i^H dB x_i) + i phi_i x_i,

where phi_i keeps the gauge.  Folding the gauge into the cotangent,
g_i = gbar_i + i c_i e_{k_i} with c_i = Im(gbar_i^H x_i) / x_{k_i, i}, gives

  Abar = herm( X diag(wbar) X^H + Z X^H ),
  Bbar = -herm( X diag(wbar lambda) X^H + Z diag(lambda) X^H + 1/2 X diag(Re g_i^H x_i) X^H ),
  z_i  = sum_{j != i} x_j (x_j^H g_i) / (lambda_i - lambda_j)   (all n eigenvectors x_j),

herm(M) = (M + M^H)/2.  Only the tests and the benchmark's CPU leg use this module.
"""
import numpy as np

from . import zhegv


def gauge_fix(X):
    """Scale each column so its entry of largest modulus (first on ties) is real positive."""
    X = np.array(X, dtype=np.complex128, copy=True)
    k = np.argmax(np.abs(X), axis=0)
    piv = X[k, np.arange(X.shape[1])]
    X *= (np.abs(piv) / piv)[None, :]
    return X, k


def solve(A, B, il, iu):
    """Selected pairs (gauge fixed) plus every eigenpair, from the oracle."""
    lam, Xall, info = zhegv(A, B)
    if info != 0:
        raise RuntimeError("oracle zhegv info %d" % info)
    Xall, _ = gauge_fix(Xall)
    return lam, Xall


def loss(A, B, il, iu, wbar, gbar):
    lam, Xall = solve(A, B, il, iu)
    X = Xall[:, il - 1:iu]
    return float(np.dot(wbar, lam[il - 1:iu]) + np.real(np.sum(gbar.conj() * X)))


def herm(M):
    return 0.5 * (M + M.conj().T)


def gradient(A, B, il, iu, wbar, gbar):
    """(Abar, Bbar) of the loss above, dense fp64."""
    lam, Xall = solve(A, B, il, iu)
    m = iu - il + 1
    sel = np.arange(il - 1, iu)
    X = Xall[:, sel]
    lam_s = lam[sel]
    k = np.argmax(np.abs(X), axis=0)
    xk = X[k, np.arange(m)].real
    ghx = np.sum(gbar.conj() * X, axis=0)
    c = ghx.imag / xk
    G = np.array(gbar, dtype=np.complex128, copy=True)
    G[k, np.arange(m)] += 1j * c
    C = Xall.conj().T @ G                                  # n x m: x_j^H g_i
    with np.errstate(divide="ignore"):
        F = 1.0 / (lam_s[None, :] - lam[:, None])
    F[sel, np.arange(m)] = 0.0
    Z = Xall @ (F * C)
    s = np.real(np.sum(G.conj() * X, axis=0))
    Abar = herm((X * wbar[None, :] + Z) @ X.conj().T)
    Bbar = -herm((X * (wbar * lam_s)[None, :] + Z * lam_s[None, :] + 0.5 * X * s[None, :]) @ X.conj().T)
    return Abar, Bbar
