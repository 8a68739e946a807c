"""Host simulation of the bulge-chasing schedule (Alg. 2 step 1, second stage; Sec. 4.2).

The GPU kernel runs the tasks (s, j) of the column-wise bulge chasing on many workgroups at
once: task (s, j) of sweep s may start once sweep s-1 has completed min(j + 2, all) of its
tasks (the rule derived from the rows each task touches).  Each task's arithmetic is fixed,
so every order that respects the rule must give the sequential result bit for bit.  Here
the tasks are modelled on the host (numpy, on a dense Hermitian matrix: task j of sweep s
right-applies the previous reflector to the block A[I_j, I_{j-1}], makes the reflector of
its first column, applies it from the left there and on both sides of A[I_j, I_j], with
I_j = rows s+1+j*b .. s+(j+1)*b), and run
  * in the sequential order, checked against the mathematics: T is tridiagonal (exact zeros
    outside it), real, and eig(T) = eig(band);
  * in random legal orders (a pool of "workgroups" picking random ready tasks), which must
    reproduce the sequential matrix bit for bit;
  * with the rule weakened to min(j + 1, all), where some order must differ (the rule is
    not slack: one task less of lag lets a task read a block its predecessor sweep has not
    finished).
"""
import numpy as np
import pytest


def tasks(n, b, s):
    return (n - 2 - s) // b + 1


def refl(x):
    """H = I - tau v v^H with H^H x = beta e_1, beta real (v_0 = 1)."""
    alpha = x[0]
    t2 = float(np.vdot(x[1:], x[1:]).real)
    v = np.zeros_like(x)
    v[0] = 1.0
    if t2 == 0.0 and alpha.imag == 0.0:
        return v, 0.0 + 0.0j, alpha.real
    beta = -np.copysign(np.sqrt(abs(alpha) ** 2 + t2), alpha.real)
    tau = (beta - alpha.real) / beta - 1j * alpha.imag / beta
    v[1:] = x[1:] / (alpha - beta)
    return v, tau, beta


def run_task(A, n, b, s, j, prev):
    """One task on the dense Hermitian matrix A (both triangles kept); prev[s] holds the
    reflector of the sweep's previous task."""
    r0 = s + 1 + j * b
    L = min(b, n - r0)
    I = slice(r0, r0 + L)
    if j == 0:
        x = A[I, s].copy()
        v, tau, beta = refl(x)
        A[I, s] = 0.0
        A[r0, s] = beta
        A[s, I] = np.conj(A[I, s])
    else:
        p0 = r0 - b
        P = slice(p0, p0 + b)
        vp, taup = prev[s]
        E = A[I, P]
        E -= taup * np.outer(E @ vp, np.conj(vp))          # E H_prev
        v, tau, beta = refl(E[:, 0].copy())
        E -= np.conj(tau) * np.outer(v, np.conj(v) @ E)    # H^H E
        E[:, 0] = 0.0
        E[0, 0] = beta
        A[P, I] = np.conj(E.T)
    D = A[I, I]
    D = D - np.conj(tau) * np.outer(v, np.conj(v) @ D)     # H^H D
    D = D - tau * np.outer(D @ v, np.conj(v))              # (H^H D) H
    D[np.diag_indices(L)] = D.diagonal().real              # Hermitian: real diagonal
    A[I, I] = D
    prev[s] = (v, tau)


def band_matrix(n, b, seed):
    rng = np.random.default_rng(seed)
    A = np.zeros((n, n), dtype=complex)
    for t in range(b + 1):
        vals = rng.standard_normal(n - t) + 1j * rng.standard_normal(n - t)
        if t == 0:
            vals = vals.real + 0j
        idx = np.arange(n - t)
        A[idx + t, idx] = vals
        A[idx, idx + t] = np.conj(vals)
    return A


def simulate(A0, b, order_rng=None, lag=2, workers=4):
    n = A0.shape[0]
    A = A0.copy()
    prev = {}
    done = [0] * max(n - 1, 1)
    if order_rng is None:
        for s in range(n - 1):
            for j in range(tasks(n, b, s)):
                run_task(A, n, b, s, j, prev)
        return A
    # a pool of workers, each owning the sweeps s = w, w + workers, ... in order (as the
    # persistent kernel deals sweeps to workgroups); at every step a random worker whose
    # next task is ready runs it
    nxt = {w: (w, 0) for w in range(workers) if w < n - 1}
    while nxt:
        ready = []
        for w, (s, j) in nxt.items():
            need = min(j + lag, tasks(n, b, s - 1)) if s > 0 else 0
            if s == 0 or done[s - 1] >= need:
                ready.append(w)
        assert ready, "schedule deadlocked"
        w = ready[order_rng.integers(len(ready))]
        s, j = nxt[w]
        run_task(A, n, b, s, j, prev)
        done[s] = j + 1
        if j + 1 < tasks(n, b, s):
            nxt[w] = (s, j + 1)
        elif s + workers < n - 1:
            nxt[w] = (s + workers, 0)
        else:
            del nxt[w]
    return A


@pytest.mark.parametrize("n,b", [(12, 2), (20, 3), (33, 4), (40, 8)])
def test_sequential_order_reduces_to_tridiagonal(n, b):
    A0 = band_matrix(n, b, n * b)
    T = simulate(A0, b)
    off = np.abs(np.tril(T, -2)).max()
    assert off == 0.0
    assert np.abs(np.diag(T).imag).max() == 0.0 and np.abs(np.diag(T, -1).imag).max() == 0.0
    np.testing.assert_allclose(np.linalg.eigvalsh(T), np.linalg.eigvalsh(A0), rtol=0,
                               atol=1e-13 * np.abs(A0).sum(0).max())


@pytest.mark.parametrize("n,b,workers", [(20, 3, 3), (33, 4, 5), (40, 8, 4), (29, 2, 7)])
def test_random_legal_orders_are_bitwise_sequential(n, b, workers):
    A0 = band_matrix(n, b, 7 * n + b)
    ref = simulate(A0, b)
    for seed in range(12):
        got = simulate(A0, b, np.random.default_rng(seed), workers=workers)
        assert np.array_equal(got, ref), seed


def test_one_task_less_of_lag_breaks_the_result():
    n, b = 24, 3
    A0 = band_matrix(n, b, 5)
    ref = simulate(A0, b)
    differs = 0
    for seed in range(40):
        got = simulate(A0, b, np.random.default_rng(seed), lag=1, workers=4)
        differs += not np.array_equal(got, ref)
    assert differs > 0
