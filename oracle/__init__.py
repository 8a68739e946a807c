"""CPU oracle for the Hermitian-definite generalized eigensolve (test infrastructure).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may import this package.  The product library never loads it.  The numerical work
is in ``hgv_oracle.c`` (plain C99, fp64, no BLAS); this module compiles it with gcc
and marshals numpy arrays.  Matrices are passed as ordinary numpy 2-D arrays
(``M[i, j]`` is element (i, j)); they are converted to column-major here.

Functions follow Algorithm 1 of the paper (Cholesky, reduction to standard form,
standard eigensolve, back-substitution) with the one-stage Algorithm 2
(Householder tridiagonalisation, tridiagonal eigensolve, back-transformation).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hgv_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force=True):
    """Compile hgv_oracle.c into liboracle.so with gcc (OpenMP)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                           "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    I = ctypes.c_int
    lib.oracle_potrf.argtypes = [I, P, I]
    lib.oracle_potrf.restype = I
    lib.oracle_hegst.argtypes = [I, P, I, P, I, P, I]
    lib.oracle_hegst.restype = None
    lib.oracle_hetrd.argtypes = [I, P, I, P, P, P, I, P, P]
    lib.oracle_hetrd.restype = None
    lib.oracle_steql.argtypes = [I, P, P, P, I]
    lib.oracle_steql.restype = I
    lib.oracle_zhegv.argtypes = [I, P, I, P, I, I, I, P, P, I]
    lib.oracle_zhegv.restype = I
    lib.oracle_set_ql_maxit.argtypes = [I]
    lib.oracle_set_ql_maxit.restype = None
    _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _fortran_c128(M):
    return np.asfortranarray(np.asarray(M, dtype=np.complex128)).copy(order="F")


def set_ql_maxit(maxit):
    """Test hook: iterations allowed per eigenvalue in the QL solver (default 30)."""
    _load().oracle_set_ql_maxit(int(maxit))


def potrf(B):
    """Unblocked Cholesky B = L L^H of the lower triangle (Alg. 1 step 1).

    Returns (L, info); info = k > 0 when the leading minor of order k is not PD."""
    lib = _load()
    L = _fortran_c128(B)
    n = L.shape[0]
    info = lib.oracle_potrf(n, _ptr(L), max(n, 1))
    return np.ascontiguousarray(L), int(info)


def hegst(A, L):
    """A' = L^-1 A L^-H from the lower triangle of A (Alg. 1 step 2); full Hermitian result."""
    lib = _load()
    Af = _fortran_c128(A)
    Lf = _fortran_c128(L)
    n = Af.shape[0]
    C = np.zeros((n, n), dtype=np.complex128, order="F")
    lib.oracle_hegst(n, _ptr(Af), max(n, 1), _ptr(Lf), max(n, 1), _ptr(C), max(n, 1))
    return np.ascontiguousarray(C)


def hetrd(C):
    """Householder tridiagonalisation of a full Hermitian C (Alg. 2 step 1, Sec. 4.1).

    Returns (d, e, U, beta, psi) with C = Q Psi T Psi^H Q^H, Q = H_0 ... H_{n-3},
    H_k = I - beta_k u_k u_k^H (u_k in U[k+1:, k]), T = tridiag(e, d, e) real."""
    lib = _load()
    Cf = _fortran_c128(C)
    n = Cf.shape[0]
    d = np.zeros(n)
    e = np.zeros(max(n - 1, 1))
    U = np.zeros((n, n), dtype=np.complex128, order="F")
    beta = np.zeros(max(n, 1))
    psi = np.zeros(max(n, 1), dtype=np.complex128)
    lib.oracle_hetrd(n, _ptr(Cf), max(n, 1), _ptr(d), _ptr(e), _ptr(U), max(n, 1),
                     _ptr(beta), _ptr(psi))
    return d, e[:max(n - 1, 0)], np.ascontiguousarray(U), beta[:n], psi[:n]


def steql(d, e, Z=None):
    """Implicit QL on the real symmetric tridiagonal (d, e) (Alg. 2 step 2).

    Returns (w, Z, info): eigenvalues ascending and eigenvectors (columns), Z
    rotated from the identity (or from the given basis)."""
    lib = _load()
    n = len(d)
    dd = np.array(d, dtype=np.float64, copy=True)
    ee = np.zeros(max(n, 1))
    ee[:max(n - 1, 0)] = np.asarray(e, dtype=np.float64)[:max(n - 1, 0)]
    Zf = np.asfortranarray(np.eye(n) if Z is None else np.array(Z, dtype=np.float64))
    Zf = Zf.copy(order="F")
    info = lib.oracle_steql(n, _ptr(dd), _ptr(ee), _ptr(Zf), max(n, 1))
    return dd, np.ascontiguousarray(Zf), int(info)


def zhegv(A, B, il=1, iu=None):
    """Eigenpairs il..iu (1-based, inclusive, ascending) of A x = lambda B x.

    Returns (W, X, info) with X^H B X = I.  info: 0 ok; n+k: B not PD at minor k;
    k in [1, n]: the QL solver failed on eigenvalue k; negative: bad argument."""
    lib = _load()
    Af = _fortran_c128(A)
    Bf = _fortran_c128(B)
    n = Af.shape[0]
    if iu is None:
        iu = n
    m = max(iu - il + 1, 0)
    W = np.zeros(max(m, 1))
    X = np.zeros((n, max(m, 1)), dtype=np.complex128, order="F")
    info = lib.oracle_zhegv(n, _ptr(Af), max(n, 1), _ptr(Bf), max(n, 1), il, iu,
                            _ptr(W), _ptr(X), max(n, 1))
    return W[:m], np.ascontiguousarray(X[:, :m]), int(info)
