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

The second part models the window-owner schedule of the same tasks: owner w keeps, for
every sweep s, the diagonal block of the rows I_w(s) and the block below it, index i at
slot i mod b, and talks to its neighbours only through mailboxes: the reflector H_{s,w+1}
to owner w+1, and the band column of the index leaving its window to owner w-1.  Owners
are generators that yield before every mailbox read; a random scheduler runs them.  Checked:
no order deadlocks, no mailbox is written again before its reader has taken the previous
message (so one buffer per mailbox would suffice), every order gives the same d, e and
reflectors bit for bit, d and e agree with the sequential dense model to rounding, and the
reflectors reproduce Q^H A Q = T.
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


# ---- window-owner schedule ----------------------------------------------------------------


class Box:
    def __init__(self):
        self.tag = -1
        self.data = None
        self.consumed = True


def owner(w, n, b, A0, boxH, boxS, out):
    """Owner w of the window pipeline (a generator yielding ('wait', box, tag))."""
    D = np.zeros((b, b), complex)
    E = np.zeros((b, b), complex)
    for s in range(n - 1 - w * b):
        r0 = s + 1 + w * b
        L = min(b, n - r0)
        Le = min(b, n - r0 - b)
        f = r0 % b
        if s == 0:
            for i in range(L):
                for k in range(L):
                    D[(r0 + i) % b, (r0 + k) % b] = A0[r0 + i, r0 + k]
            for i in range(max(Le, 0)):
                for k in range(L):
                    E[(r0 + i) % b, (r0 + k) % b] = A0[r0 + b + i, r0 + k]
            if w == 0:
                x = A0[1:1 + L, 0].copy()
                out["d"][0] = A0[0, 0].real
        else:
            t = (r0 - 1) % b
            c = r0 - 1 + b
            if w == 0:   # column s = r0 - 1, the index leaving the window
                x = np.array([D[(r0 + i) % b, t] if i < b - 1 else E[t, t] for i in range(L)])
                out["d"][r0 - 1] = D[t, t].real
            if c <= n - 1:
                yield ("wait", boxS[w], s)
                msg = boxS[w].data.copy()
                boxS[w].consumed = True
            else:
                msg = np.zeros(b + 1, complex)
            row = E[t, :].copy()
            D[t, :] = row
            D[:, t] = np.conj(row)
            D[t, t] = msg[0].real
            E[t, :] = 0.0
            for i in range(1, b):
                E[(c + i) % b, t] = msg[i]
            E[t, t] = msg[b]
        if w == 0:
            v, tau, beta = refl(x)
            out["e"][r0 - 1] = beta
            out["V"][(r0 - 1, 0)] = (np.pad(v, (0, b - L)), tau)
        else:
            yield ("wait", boxH[w], s)
            vv, tau = boxH[w].data
            boxH[w].consumed = True
            v = vv[:L]
        vs = np.zeros(b, complex)
        for i in range(L):
            vs[(r0 + i) % b] = v[i]
        if Le > 0:
            E -= tau * np.outer(E @ vs, np.conj(vs))
            v2, tau2, beta2 = refl(np.array([E[(r0 + i) % b, f] for i in range(Le)]))
            bx = boxH[w + 1]
            assert bx.consumed, "reflector mailbox written before it was read"
            bx.data, bx.tag, bx.consumed = (np.pad(v2, (0, b - Le)), tau2), s, False
            out["V"][(s, w + 1)] = (np.pad(v2, (0, b - Le)), tau2)
            yield ("posted",)
        p = tau * (D @ vs)
        half = 0.5 * (np.conj(tau) * np.vdot(vs, p)).real
        wv = p - half * vs
        D = D - np.outer(vs, np.conj(wv)) - np.outer(wv, np.conj(vs))
        D[np.diag_indices(b)] = D.diagonal().real
        if w >= 1:
            msg = np.zeros(b + 1, complex)
            for i in range(L):
                msg[i] = D[(r0 + i) % b, f]
            if Le > 0:
                msg[b] = beta2
            bx = boxS[w - 1]
            assert bx.consumed, "column mailbox written before it was read"
            bx.data, bx.tag, bx.consumed = msg, s + 1, False
            yield ("posted",)
        if Le > 0:
            v2s = np.zeros(b, complex)
            for i in range(Le):
                v2s[(r0 + i) % b] = v2[i]
            E -= np.conj(tau2) * np.outer(v2s, np.conj(v2s) @ E)
            E[:, f] = 0.0
            E[f, f] = beta2
    if w == 0:
        out["d"][n - 1] = D[(n - 1) % b, (n - 1) % b].real


def run_owners(A0, b, rng=None):
    n = A0.shape[0]
    J = tasks(n, b, 0)
    boxH = [Box() for _ in range(J + 1)]
    boxS = [Box() for _ in range(J + 1)]
    out = {"d": np.zeros(n), "e": np.zeros(n - 1), "V": {}}
    gens = {w: owner(w, n, b, A0, boxH, boxS, out) for w in range(J)}
    pending = {}
    for w in list(gens):
        try:
            pending[w] = next(gens[w])
        except StopIteration:
            del gens[w]
    while gens:
        ready = [w for w in gens if pending[w][0] != "wait" or pending[w][1].tag == pending[w][2]]
        assert ready, "schedule deadlocked"
        w = ready[0] if rng is None else ready[rng.integers(len(ready))]
        try:
            pending[w] = gens[w].send(None)
        except StopIteration:
            del gens[w]
    return out


def q_from(V, n, b):
    Q = np.eye(n, dtype=complex)
    for s in range(n - 1):
        for j in range(tasks(n, b, s)):
            v, tau = V[(s, j)]
            r0 = s + 1 + j * b
            L = min(b, n - r0)
            vv = np.zeros(n, complex)
            vv[r0:r0 + L] = v[:L]
            Q = Q - tau * np.outer(Q @ vv, np.conj(vv))
    return Q


@pytest.mark.parametrize("n,b", [(12, 2), (20, 3), (33, 4), (40, 8), (29, 2), (70, 16), (9, 1), (5, 8), (17, 16)])
def test_owner_schedule_matches_the_sequential_reduction(n, b):
    A0 = band_matrix(n, min(b, n - 1), 3 * n + b)   # a band at least as wide as the matrix is full
    T = simulate(A0, b)
    o = run_owners(A0, b)
    scale = np.abs(A0).sum(0).max()
    assert np.abs(o["d"] - np.diag(T).real).max() < 1e-13 * scale
    assert np.abs(o["e"] - np.diag(T, -1).real).max() < 1e-13 * scale
    Tt = np.diag(o["d"]) + np.diag(o["e"], 1) + np.diag(o["e"], -1)
    Q = q_from(o["V"], n, b)
    assert np.abs(Q.conj().T @ A0 @ Q - Tt).max() < 1e-13 * scale
    assert np.abs(Q.conj().T @ Q - np.eye(n)).max() < 1e-13 * n


@pytest.mark.parametrize("n,b", [(20, 3), (40, 8), (29, 2), (70, 16)])
def test_owner_schedule_random_orders_are_bitwise_equal(n, b):
    A0 = band_matrix(n, b, 5 * n + b)
    ref = run_owners(A0, b)
    for seed in range(8):
        got = run_owners(A0, b, np.random.default_rng(seed))
        assert np.array_equal(got["d"], ref["d"]) and np.array_equal(got["e"], ref["e"]), seed
        for key, (v, tau) in ref["V"].items():
            assert np.array_equal(got["V"][key][0], v) and got["V"][key][1] == tau, (seed, key)
