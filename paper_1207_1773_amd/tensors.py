"""torch marshalling for libhgv: column-major device buffers, workspace, stream.

Matrices are handed to the library as column-major buffers.  A torch matrix M
(rows x cols) is stored column-major by the contiguous tensor ``M.mT.contiguous()``
(shape cols x rows); the library's column-major output of shape rows x cols comes
back as ``buf.mT``.  All arithmetic happens in the library; these helpers only copy,
allocate and pass pointers.
"""
import atexit
import ctypes

import torch

from . import (hgv_chegvx, hgv_chegvx_bufsize, hgv_dstebz, hgv_dstebz_bufsize, hgv_dsygvx, hgv_dsygvx_bufsize,
               hgv_zhegvx_range, hgv_zhegvx_range_bufsize, hgv_zhetrd, hgv_zhetrd_bufsize, hgv_zunmtr_tr)
from . import (HGV_FP64, HGV_MIXED, HGV_ST_HB2ST, HGV_ST_HE2HB, HGV_ST_HEGST, HGV_ST_POTRF, HGV_ST_Q1,
               HGV_ST_Q2, HGV_ST_STEDC, HGV_ST_TRSM, Opts, Stats, c128, hgv_create, hgv_destroy, hgv_dstedc,
               hgv_set_stream, hgv_stage_bufsize, hgv_v2_elems, hgv_v2_taus, hgv_zgemm, hgv_zhb2st, hgv_zhe2hb,
               hgv_zhegst, hgv_zhegvx, hgv_zhegvx_batched, hgv_zhegvx_batched_bufsize, hgv_zhegvx_bufsize,
               hgv_zpotrf, hgv_ztrsm_lh, hgv_zunmtr_q1, hgv_zunmtr_q2, hgv_device_peaks, load)


def colmajor(M, dtype=torch.complex128):
    """Column-major copy of a matrix: a contiguous (cols x rows) tensor holding M^T."""
    return M.to(dtype).mT.contiguous()


def from_colmajor(buf):
    """The (rows x cols) matrix whose column-major storage is buf (a view)."""
    return buf.mT


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Context:
    """One library context per device; calls run on torch's current stream."""

    _cache = {}

    def __init__(self, device=None):
        load()
        dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        if dev.type != "cuda":
            raise ValueError("libhgv runs on a GPU device, got %s" % dev)
        self.device = dev
        self.handle = hgv_create(dev.index if dev.index is not None else 0)

    @classmethod
    def get(cls, device=None):
        dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        key = dev.index or 0
        if key not in cls._cache:
            cls._cache[key] = Context(dev)
        return cls._cache[key]

    def close(self):
        """Destroy the library context (its streams and events); idempotent."""
        h, self.handle = getattr(self, "handle", None), None
        if h:
            hgv_destroy(h)

    def __del__(self):
        # never at interpreter shutdown: the cached contexts are closed by the
        # atexit hook below while the HIP runtime is still fully up, and a
        # context collected during finalisation would destroy streams after
        # the runtime (or a profiler attached to it) has begun to shut down
        if _closing:
            return
        try:
            self.close()
        except Exception:
            pass

    def _sync_stream(self):
        hgv_set_stream(self.handle, ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream))

    def _work(self, nbytes):
        n = max(int(nbytes), 256)
        return torch.empty(n, dtype=torch.uint8, device=self.device)

    def _info(self):
        return torch.zeros(1, dtype=torch.int32, device=self.device)

    # ---- stages (inputs/outputs as ordinary torch matrices) -----------------------------
    def potrf(self, B):
        """Alg. 1 step 1: returns (L lower, info) for Hermitian PD B (lower triangle read)."""
        self._sync_stream()
        n = B.shape[0]
        Bc = colmajor(B)
        w = self._work(hgv_stage_bufsize(self.handle, HGV_ST_POTRF, n))
        info = self._info()
        hgv_zpotrf(self.handle, n, _ptr(Bc), max(n, 1), _ptr(w), w.numel(), _ptr(info))
        return torch.tril(from_colmajor(Bc)), int(info.item())

    def hegst(self, A, L):
        """Alg. 1 step 2: returns the lower triangle of L^-1 A L^-H."""
        self._sync_stream()
        n = A.shape[0]
        Ac, Lc = colmajor(A), colmajor(L)
        w = self._work(hgv_stage_bufsize(self.handle, HGV_ST_HEGST, n))
        hgv_zhegst(self.handle, n, _ptr(Ac), max(n, 1), _ptr(Lc), max(n, 1), _ptr(w), w.numel())
        return torch.tril(from_colmajor(Ac))

    def he2hb(self, A, nb):
        """Alg. 2 step 1, first stage: returns (A_out column-major buffer view, T1)."""
        self._sync_stream()
        n = A.shape[0]
        Ac = colmajor(A)
        np_ = (n + nb - 1) // nb
        T1 = torch.zeros((max(np_, 1), nb, nb), dtype=torch.complex128, device=self.device)
        w = self._work(hgv_stage_bufsize(self.handle, HGV_ST_HE2HB, n, nb))
        info = self._info()
        hgv_zhe2hb(self.handle, n, nb, _ptr(Ac), max(n, 1), _ptr(T1), _ptr(w), w.numel(), _ptr(info))
        self.last_info = info
        return from_colmajor(Ac), T1

    def hb2st(self, Aband, nb):
        """Alg. 2 step 1, second stage: (d, e, V2, tau2) from the lower band of Aband."""
        self._sync_stream()
        n = Aband.shape[0]
        Ac = colmajor(Aband)
        d = torch.zeros(max(n, 1), dtype=torch.float64, device=self.device)
        e = torch.zeros(max(n - 1, 1), dtype=torch.float64, device=self.device)
        V2 = torch.zeros(max(hgv_v2_elems(n, nb), 1), dtype=torch.complex128, device=self.device)
        tau2 = torch.zeros(max(hgv_v2_taus(n, nb), 1), dtype=torch.complex128, device=self.device)
        w = self._work(hgv_stage_bufsize(self.handle, HGV_ST_HB2ST, n, nb))
        info = self._info()
        hgv_zhb2st(self.handle, n, nb, _ptr(Ac), max(n, 1), _ptr(d), _ptr(e), _ptr(V2), _ptr(tau2), _ptr(w),
                   w.numel(), _ptr(info))
        self.last_info = info
        return d[:n], e[:max(n - 1, 0)], V2, tau2

    def stedc(self, d, e, il=1, iu=None):
        """Alg. 2 step 2: (all eigenvalues, eigenvectors il..iu as n x m real, info)."""
        self._sync_stream()
        n = d.shape[0]
        iu = n if iu is None else iu
        m = iu - il + 1
        dd = d.to(self.device, torch.float64).contiguous()
        ee = torch.zeros(max(n - 1, 1), dtype=torch.float64, device=self.device)
        if n > 1:
            ee[:n - 1] = e[:n - 1]
        lam = torch.zeros(max(n, 1), dtype=torch.float64, device=self.device)
        Zc = torch.zeros((max(m, 1), max(n, 1)), dtype=torch.float64, device=self.device)
        w = self._work(hgv_stage_bufsize(self.handle, HGV_ST_STEDC, n, 0, m))
        info = self._info()
        hgv_dstedc(self.handle, n, _ptr(dd), _ptr(ee), il, iu, _ptr(lam), _ptr(Zc), max(n, 1), _ptr(w), w.numel(),
                   _ptr(info))
        return lam[:n], from_colmajor(Zc)[:n, :m], int(info.item())

    def hetrd(self, A, nb):
        """One-stage tridiagonalisation (Sec. 4.1): (A_out column-major view, d, e, T1)."""
        self._sync_stream()
        n = A.shape[0]
        Ac = colmajor(A)
        d = torch.zeros(max(n, 1), dtype=torch.float64, device=self.device)
        e = torch.zeros(max(n - 1, 1), dtype=torch.float64, device=self.device)
        T1 = torch.zeros((max((n + nb - 1) // nb, 1), nb, nb), dtype=torch.complex128, device=self.device)
        w = self._work(hgv_zhetrd_bufsize(self.handle, n, nb))
        hgv_zhetrd(self.handle, n, nb, _ptr(Ac), max(n, 1), _ptr(d), _ptr(e), _ptr(T1), _ptr(w), w.numel())
        return from_colmajor(Ac), d[:n], e[:max(n - 1, 0)], T1

    def unmtr_tr(self, Ab, T1, Y, nb, adj=False):
        """Q Y (Q^H Y with adj=True) with Q from hetrd (Ab as returned by hetrd)."""
        self._sync_stream()
        n, m = Y.shape
        Ac = colmajor(Ab)
        Yc = colmajor(Y)
        w = self._work(hgv_stage_bufsize(self.handle, HGV_ST_Q1, n, nb, m))
        hgv_zunmtr_tr(self.handle, "C" if adj else "N", n, nb, m, _ptr(Ac), max(n, 1), _ptr(T1), _ptr(Yc), max(n, 1),
                      _ptr(w), w.numel())
        return from_colmajor(Yc)

    def stebz(self, d, e, il=1, iu=None):
        """Eigenvalues il..iu of the tridiagonal (d, e) by Sturm-count multisection."""
        self._sync_stream()
        n = d.shape[0]
        iu = n if iu is None else iu
        dd = d.to(self.device, torch.float64).contiguous()
        ee = torch.zeros(max(n - 1, 1), dtype=torch.float64, device=self.device)
        if n > 1:
            ee[:n - 1] = e[:n - 1]
        W = torch.zeros(max(iu - il + 1, 1), dtype=torch.float64, device=self.device)
        w = self._work(hgv_dstebz_bufsize(self.handle, n))
        hgv_dstebz(self.handle, n, _ptr(dd), _ptr(ee), il, iu, _ptr(W), _ptr(w), w.numel())
        return W[:iu - il + 1]

    def q2(self, V2, tau2, Y, nb, adj=False):
        """Alg. 2 step 3 (first part): Q2 Y (Q2^H Y with adj=True)."""
        self._sync_stream()
        n, m = Y.shape
        Yc = colmajor(Y)
        w = self._work(hgv_stage_bufsize(self.handle, HGV_ST_Q2, n, nb, m))
        hgv_zunmtr_q2(self.handle, "C" if adj else "N", n, nb, m, _ptr(V2), _ptr(tau2), _ptr(Yc), max(n, 1), _ptr(w),
                      w.numel())
        return from_colmajor(Yc)

    def q1(self, Ab, T1, Y, nb, adj=False):
        """Alg. 2 step 3 (second part): Q1 Y (Q1^H Y with adj=True) with reflectors from he2hb
        (Ab as returned by he2hb)."""
        self._sync_stream()
        n, m = Y.shape
        Ac = colmajor(Ab)
        Yc = colmajor(Y)
        w = self._work(hgv_stage_bufsize(self.handle, HGV_ST_Q1, n, nb, m))
        hgv_zunmtr_q1(self.handle, "C" if adj else "N", n, nb, m, _ptr(Ac), max(n, 1), _ptr(T1), _ptr(Yc), max(n, 1),
                      _ptr(w), w.numel())
        return from_colmajor(Yc)

    def device_peaks(self, nbytes=1 << 30):
        """Measured (FP64 MFMA TFLOP/s, copy GB/s read + write) of this device; nbytes of scratch."""
        self._sync_stream()
        w = self._work(nbytes)
        return hgv_device_peaks(self.handle, _ptr(w), w.numel())

    def trsm_lh(self, L, X):
        """Alg. 1 step 4: L^-H X."""
        self._sync_stream()
        n, m = X.shape
        Lc, Xc = colmajor(L), colmajor(X)
        w = self._work(hgv_stage_bufsize(self.handle, HGV_ST_TRSM, n, 0, m))
        hgv_ztrsm_lh(self.handle, n, m, _ptr(Lc), max(n, 1), _ptr(Xc), max(n, 1), _ptr(w), w.numel())
        return from_colmajor(Xc)

    def gemm(self, opa, opb, A, B, alpha=1.0, beta=0.0, C=None):
        """C <- alpha op(A) op(B) + beta C on the library's MFMA tiles."""
        self._sync_stream()
        Ac, Bc = colmajor(A), colmajor(B)
        ra, ca = A.shape
        rb, cb = B.shape
        m = ra if opa == "N" else ca
        k = ca if opa == "N" else ra
        n = cb if opb == "N" else rb
        Cc = colmajor(C) if C is not None else torch.zeros((n, m), dtype=torch.complex128, device=self.device)
        hgv_zgemm(self.handle, opa, opb, m, n, k, complex(alpha), _ptr(Ac), max(ra, 1), _ptr(Bc), max(rb, 1),
                  complex(beta), _ptr(Cc), max(m, 1))
        return from_colmajor(Cc)

    # ---- full solve ------------------------------------------------------------------------------
    def zhegvx(self, A, B, il=1, iu=None, precision="fp64", nb=0, stats=False, inplace=False, max_refine_iters=0,
               refine_tol=0.0, values_only=False, one_stage=False):
        """Eigenpairs il..iu of (A, B).  Returns (W, X, info, stats_dict_or_None).

        precision "mixed" runs the complex64 reduction with FP64 refinement
        (max_refine_iters / refine_tol as in hgv_opts; 0 picks the defaults).
        values_only=True computes the eigenvalues only (X is None).
        With inplace=True, A and B must already be column-major buffers (as made by
        ``colmajor``); they are then destroyed / overwritten by L."""
        self._sync_stream()
        n = A.shape[0]
        iu = n if iu is None else iu
        m = iu - il + 1
        Ac = A if inplace else colmajor(A)
        Bc = B if inplace else colmajor(B)
        opts = _opts(precision, nb, max_refine_iters, refine_tol, values_only, one_stage)
        W = torch.zeros(max(m, 1), dtype=torch.float64, device=self.device)
        Xc = None if values_only else torch.zeros((max(m, 1), max(n, 1)), dtype=torch.complex128, device=self.device)
        w = self._work(hgv_zhegvx_bufsize(self.handle, n, il, iu, opts))
        info = self._info()
        st = Stats() if stats else None
        hgv_zhegvx(self.handle, n, _ptr(Ac), max(n, 1), _ptr(Bc), max(n, 1), il, iu, _ptr(W), _ptr(Xc), max(n, 1),
                   _ptr(w), w.numel(), opts, _ptr(info), st)
        X = None if values_only else from_colmajor(Xc)[:n, :m]
        return W[:m], X, int(info.item()), (st.as_dict() if st is not None else None)

    def chegvx(self, A, B, il=1, iu=None, nb=0, stats=False, values_only=False):
        """Complex64 pencil: eigenpairs il..iu.  Returns (W float32, X complex64 or None, info, stats)."""
        self._sync_stream()
        n = A.shape[0]
        iu = n if iu is None else iu
        m = iu - il + 1
        Ac, Bc = colmajor(A, torch.complex64), colmajor(B, torch.complex64)
        opts = _opts("fp64", nb, 0, 0.0, values_only)
        W = torch.zeros(max(m, 1), dtype=torch.float32, device=self.device)
        Xc = None if values_only else torch.zeros((max(m, 1), max(n, 1)), dtype=torch.complex64, device=self.device)
        w = self._work(hgv_chegvx_bufsize(self.handle, n, il, iu, opts))
        info = self._info()
        st = Stats() if stats else None
        hgv_chegvx(self.handle, n, _ptr(Ac), max(n, 1), _ptr(Bc), max(n, 1), il, iu, _ptr(W), _ptr(Xc), max(n, 1),
                   _ptr(w), w.numel(), opts, _ptr(info), st)
        X = None if values_only else from_colmajor(Xc)[:n, :m]
        return W[:m], X, int(info.item()), (st.as_dict() if st is not None else None)

    def dsygvx(self, A, B, il=1, iu=None, precision="fp64", nb=0, stats=False, values_only=False):
        """Real symmetric-definite pencil: eigenpairs il..iu.  Returns (W, X float64 or None, info,
        stats, L) where L is the Cholesky factor left in B's lower triangle."""
        self._sync_stream()
        n = A.shape[0]
        iu = n if iu is None else iu
        m = iu - il + 1
        Ac, Bc = colmajor(A, torch.float64), colmajor(B, torch.float64)
        opts = _opts(precision, nb, 0, 0.0, values_only)
        W = torch.zeros(max(m, 1), dtype=torch.float64, device=self.device)
        Xc = None if values_only else torch.zeros((max(m, 1), max(n, 1)), dtype=torch.float64, device=self.device)
        w = self._work(hgv_dsygvx_bufsize(self.handle, n, il, iu, opts))
        info = self._info()
        st = Stats() if stats else None
        hgv_dsygvx(self.handle, n, _ptr(Ac), max(n, 1), _ptr(Bc), max(n, 1), il, iu, _ptr(W), _ptr(Xc), max(n, 1),
                   _ptr(w), w.numel(), opts, _ptr(info), st)
        X = None if values_only else from_colmajor(Xc)[:n, :m]
        return W[:m], X, int(info.item()), (st.as_dict() if st is not None else None), torch.tril(from_colmajor(Bc))

    def zhegvx_range(self, A, B, vl, vu, mmax=None, nb=0, stats=False, inplace=False, values_only=False):
        """Eigenpairs with eigenvalues in (vl, vu], at most mmax of them (default n).
        Returns (W, X, m, info, stats): W and X hold min(m, mmax) pairs, m is the number
        of eigenvalues in the interval (counted on the device)."""
        self._sync_stream()
        n = A.shape[0]
        mmax = n if mmax is None else mmax
        Ac = A if inplace else colmajor(A)
        Bc = B if inplace else colmajor(B)
        opts = _opts("fp64", nb, 0, 0.0, values_only)
        W = torch.zeros(max(mmax, 1), dtype=torch.float64, device=self.device)
        Xc = None if values_only else torch.zeros((max(mmax, 1), max(n, 1)), dtype=torch.complex128,
                                                  device=self.device)
        w = self._work(hgv_zhegvx_range_bufsize(self.handle, n, mmax, opts))
        info = self._info()
        dm = self._info()
        st = Stats() if stats else None
        hgv_zhegvx_range(self.handle, n, _ptr(Ac), max(n, 1), _ptr(Bc), max(n, 1), float(vl), float(vu), mmax,
                         _ptr(W), _ptr(Xc), max(n, 1), _ptr(dm), _ptr(w), w.numel(), opts, _ptr(info), st)
        m = int(dm.item())
        X = None if values_only else from_colmajor(Xc)[:n, :mmax]
        return W[:mmax], X, m, int(info.item()), (st.as_dict() if st is not None else None)


_closing = False


@atexit.register
def _close_cached_contexts():
    """Destroy the cached contexts at exit, after the device has drained, before
    the interpreter (and with it torch and the HIP runtime) shuts down."""
    global _closing
    _closing = True
    for key, ctx in list(Context._cache.items()):
        try:
            with torch.cuda.device(ctx.device):
                torch.cuda.synchronize()
            ctx.close()
        except Exception:
            pass
    Context._cache.clear()


def _opts(precision, nb=0, max_refine_iters=0, refine_tol=0.0, values_only=False, one_stage=False):
    if precision not in ("fp64", "mixed"):
        raise ValueError("precision must be 'fp64' or 'mixed'")
    return Opts(HGV_FP64 if precision == "fp64" else HGV_MIXED, int(nb), int(max_refine_iters), float(refine_tol),
                int(bool(values_only)), int(bool(one_stage)))


class BatchedSolve:
    """Buffers of one batched solve: column-major inputs (kept pristine), working copies,
    outputs and the workspace.  run() restores the working copies and launches
    hgv_zhegvx_batched on the current stream; it allocates nothing, so it can be captured
    in a HIP graph and replayed."""

    def __init__(self, ctx, As, Bs, il, iu, nb=None, precision="fp64", max_refine_iters=0, refine_tol=0.0):
        self.ctx = ctx
        self.opts = _opts(precision, 0, max_refine_iters, refine_tol)
        dev = ctx.device
        self.n = [int(A.shape[0]) for A in As]
        self.il = list(il)
        self.iu = list(iu)
        self.nb = list(nb) if nb is not None else None
        self.A0 = [colmajor(A.to(dev)) for A in As]
        self.B0 = [colmajor(B.to(dev)) for B in Bs]
        self.A = [a.clone() for a in self.A0]
        self.B = [b.clone() for b in self.B0]
        m = [u - l + 1 for l, u in zip(self.il, self.iu)]
        self.W = [torch.zeros(max(k, 1), dtype=torch.float64, device=dev) for k in m]
        self.X = [torch.zeros((max(k, 1), max(nn, 1)), dtype=torch.complex128, device=dev)
                  for k, nn in zip(m, self.n)]
        self.info = torch.zeros(max(len(self.n), 1), dtype=torch.int32, device=dev)
        self.work = ctx._work(hgv_zhegvx_batched_bufsize(ctx.handle, self.n, self.il, self.iu, self.nb, self.opts))
        self.m = m

    def run(self):
        for a, a0 in zip(self.A, self.A0):
            a.copy_(a0)
        for b, b0 in zip(self.B, self.B0):
            b.copy_(b0)
        self.ctx._sync_stream()
        P = lambda ts: [t.data_ptr() for t in ts]
        ld = [max(x, 1) for x in self.n]
        hgv_zhegvx_batched(self.ctx.handle, self.n, P(self.A), ld, P(self.B), ld, self.il, self.iu, P(self.W),
                           P(self.X), ld, self.nb, ctypes.c_void_p(self.work.data_ptr()), self.work.numel(),
                           ctypes.c_void_p(self.info.data_ptr()), self.opts)

    def results(self):
        return ([w[:k] for w, k in zip(self.W, self.m)],
                [from_colmajor(x)[:nn, :k] for x, nn, k in zip(self.X, self.n, self.m)],
                self.info[:len(self.n)].tolist())


def eigh(A, B, il=1, iu=None, precision="fp64", nb=0):
    """Eigenpairs il..iu (1-based, inclusive) of A x = lambda B x for Hermitian A and
    Hermitian positive definite B (torch complex tensors on a GPU).  Returns (W, X)."""
    ctx = Context.get(A.device)
    W, X, info, _ = ctx.zhegvx(A, B, il, iu, precision, nb)
    if info != 0:
        raise RuntimeError("hgv_zhegvx failed: info = %d" % info)
    return W, X
