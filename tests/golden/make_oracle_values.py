"""Writes the stored oracle values used by the GPU parity tests at sizes where the oracle
takes minutes (it calls only oracle/ and the seeded generators in inputs/).

* config1_n4096_W.txt / config1_n4096_X_cols.npy: the GUE-like pencil A = (G + G^H)/2,
  B = U diag(logspace(0, 3, n)) U^H (cond(B) = 1e3), n = 4096, seed 1: all eigenvalues
  (ascending), and the B-orthonormal eigenvectors of the columns listed in
  CONFIG1_COLS (phase as the oracle leaves it).
* batch_{i}_n{n}_W.txt / batch_{i}_n{n}_X_cols.npy: problems of the batched workload
  (64 pencils, n uniform in [500, 3000], seed [3, i], cond(B) = 1e2) at both ends of the
  size range: eigenvalues 1 .. ceil(0.2 n) and the vectors of BATCH_COLS.

Run from the repository root:  python tests/golden/make_oracle_values.py
"""
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from inputs import batch_problem, batch_sizes, gue_pair  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
CONFIG1_COLS = [0, 1, 2047, 4094, 4095]
BATCH_COLS = [0, 1, -2, -1]   # of the selected ceil(0.2 n) pairs


def batch_ends():
    """Indices of the two smallest and the two largest problems of the batched draw."""
    s = np.asarray(batch_sizes())
    order = np.argsort(s, kind="stable")
    return [int(i) for i in list(order[:2]) + list(order[-2:])]


def write(prefix, W, Xcols, note):
    np.savetxt(os.path.join(HERE, prefix + "_W.txt"), W, fmt="%.17g", header=note)
    np.save(os.path.join(HERE, prefix + "_X_cols.npy"), Xcols, allow_pickle=False)


def main():
    t = time.time()
    A, B = gue_pair(4096, 1, cond_b=1e3)
    W, X, info = oracle.zhegv(A.numpy(), B.numpy())
    assert info == 0
    write("config1_n4096", W, X[:, CONFIG1_COLS],
          "oracle.zhegv eigenvalues, gue_pair(4096, seed 1, cond_b 1e3); vector columns %s" % CONFIG1_COLS)
    print("config 1: %.0f s" % (time.time() - t), flush=True)
    sizes = batch_sizes()
    for i in batch_ends():
        t = time.time()
        n = sizes[i]
        m = int(math.ceil(0.2 * n))
        A, B = batch_problem(i, n)
        W, X, info = oracle.zhegv(A.numpy(), B.numpy(), 1, m)
        assert info == 0
        cols = [c % m for c in BATCH_COLS]
        write("batch_%d_n%d" % (i, n), W, X[:, cols],
              "oracle.zhegv eigenvalues 1..%d, batch_problem(%d, n=%d, seed [3, %d], cond_b 1e2); vector columns %s"
              % (m, i, n, i, cols))
        print("batch problem %d (n=%d): %.0f s" % (i, n, time.time() - t), flush=True)


if __name__ == "__main__":
    main()
