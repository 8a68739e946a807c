"""Helpers for the GPU parity tests (host-side numpy/torch conversions only)."""
import numpy as np
import pytest


def require_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1207_1773_amd as hgv
    hgv.load()   # raises when the library is not built: the GPU tests never fall back
    return hgv


def to_dev(M):
    import torch
    return torch.as_tensor(np.ascontiguousarray(M)).to("cuda:0")


def to_np(T):
    return T.detach().cpu().numpy()


def rand_hpd(n, seed, shift=None):
    rng = np.random.default_rng(seed)
    H = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return H @ H.conj().T + (float(n) if shift is None else shift) * np.eye(n)


def rand_herm(n, seed):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return 0.5 * (G + G.conj().T)


def rel_fro(X, Y):
    d = np.linalg.norm(Y)
    return np.linalg.norm(X - Y) / (d if d > 0 else 1.0)
