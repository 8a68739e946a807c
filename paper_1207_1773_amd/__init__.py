"""Python binding of libhgv.so, the gfx950 Hermitian-definite generalized eigensolver.

The ``hgv_*`` functions mirror the C ABI in ``include/hgv.h`` one to one (raw device
pointers as integers, status codes turned into exceptions).  ``eigh`` and friends
marshal torch tensors: they make column-major copies of the inputs, allocate the
workspace the library asks for, pass the current HIP stream and view the outputs.
Every arithmetic step of the solve runs in the library's HIP kernels; when the
library is not built this module raises instead of computing anything itself.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhgv.so")

HGV_OK = 0
HGV_E_HIP = 1001
HGV_E_WORKSPACE = 1002
HGV_E_CTX = 1003
HGV_E_NOTSUP = 1004
HGV_FP64 = 0
HGV_MIXED = 1
(HGV_ST_POTRF, HGV_ST_HEGST, HGV_ST_HE2HB, HGV_ST_HB2ST, HGV_ST_STEDC, HGV_ST_Q2, HGV_ST_Q1,
 HGV_ST_TRSM, HGV_ST_REFINE, HGV_NSTAGES) = range(10)
STAGE_NAMES = ["potrf", "hegst", "he2hb", "hb2st", "stedc", "q2", "q1", "trsm", "refine"]

EXPORTS = [
    "hgv_create", "hgv_destroy", "hgv_set_stream", "hgv_status_string", "hgv_last_hip_error",
    "hgv_default_nb", "hgv_zhegvx_bufsize", "hgv_zhegvx", "hgv_stage_bufsize", "hgv_zpotrf",
    "hgv_zhegst", "hgv_zhe2hb", "hgv_zhb2st", "hgv_v2_elems", "hgv_v2_taus", "hgv_dstedc",
    "hgv_zunmtr_q2", "hgv_zunmtr_q1", "hgv_ztrsm_lh", "hgv_zgemm", "hgv_device_peaks", "hgv_gauge_fix",
    "hgv_zhegvx_backward_bufsize", "hgv_zhegvx_backward", "hgv_zhegvx_batched_bufsize", "hgv_zhegvx_batched",
    "hgv_test_hooks", "hgv_zhegvx_range_bufsize", "hgv_zhegvx_range", "hgv_dstebz_bufsize", "hgv_dstebz",
    "hgv_chegvx_bufsize", "hgv_chegvx", "hgv_dsygvx_bufsize", "hgv_dsygvx", "hgv_dstebz_noalloc",
    "hgv_zhetrd_bufsize", "hgv_zhetrd", "hgv_zunmtr_tr",
]
HGV_DSTEBZ_NOALLOC_MAX = 262144
HGV_TEST_WAIT_FAIL = 1
HGV_TEST_NAN_RESIDUAL = 2
HGV_TEST_HB2ST_SWEEPS = 4
HGV_TEST_HOUSEHOLDER_PANELS = 8


class c128(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("nb", ctypes.c_int),
                ("max_refine_iters", ctypes.c_int), ("refine_tol", ctypes.c_double),
                ("values_only", ctypes.c_int), ("one_stage", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_float * HGV_NSTAGES), ("flops", ctypes.c_double * HGV_NSTAGES),
                ("gemm_ms", ctypes.c_double), ("gemm_flops", ctypes.c_double),
                ("gemm_launches", ctypes.c_int), ("refine_iters", ctypes.c_int), ("nb", ctypes.c_int),
                ("refine_resid", ctypes.c_double), ("fallback", ctypes.c_int)]

    def as_dict(self):
        return {
            "ms": {STAGE_NAMES[i]: float(self.ms[i]) for i in range(HGV_NSTAGES)},
            "flops": {STAGE_NAMES[i]: float(self.flops[i]) for i in range(HGV_NSTAGES)},
            "gemm_ms": float(self.gemm_ms), "gemm_flops": float(self.gemm_flops),
            "gemm_launches": int(self.gemm_launches), "refine_iters": int(self.refine_iters),
            "nb": int(self.nb), "refine_resid": float(self.refine_resid), "fallback": int(self.fallback),
        }


class HgvError(RuntimeError):
    def __init__(self, status, where=""):
        self.status = status
        msg = _lib.hgv_status_string(status).decode() if _lib is not None else str(status)
        super().__init__("%s: status %d (%s)" % (where, status, msg))


_lib = None
P = ctypes.c_void_p
I = ctypes.c_int
SZ = ctypes.c_size_t


def load():
    """Load libhgv.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libhgv.so is not built (run paper_1207_1773_amd.build.build())")
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "hgv_create": (I, [ctypes.POINTER(P), I]),
        "hgv_destroy": (I, [P]),
        "hgv_set_stream": (I, [P, P]),
        "hgv_status_string": (ctypes.c_char_p, [I]),
        "hgv_last_hip_error": (I, [P]),
        "hgv_default_nb": (I, [I, I]),
        "hgv_zhegvx_bufsize": (I, [P, I, I, I, ctypes.POINTER(Opts), ctypes.POINTER(SZ)]),
        "hgv_zhegvx": (I, [P, I, P, I, P, I, I, I, P, P, I, P, SZ, ctypes.POINTER(Opts), P,
                           ctypes.POINTER(Stats)]),
        "hgv_stage_bufsize": (I, [P, I, I, I, I, ctypes.POINTER(SZ)]),
        "hgv_zpotrf": (I, [P, I, P, I, P, SZ, P]),
        "hgv_zhegst": (I, [P, I, P, I, P, I, P, SZ]),
        "hgv_zhe2hb": (I, [P, I, I, P, I, P, P, SZ, P]),
        "hgv_zhb2st": (I, [P, I, I, P, I, P, P, P, P, P, SZ, P]),
        "hgv_test_hooks": (I, [P, I]),
        "hgv_zhegvx_range_bufsize": (I, [P, I, I, ctypes.POINTER(Opts), ctypes.POINTER(SZ)]),
        "hgv_zhegvx_range": (I, [P, I, P, I, P, I, ctypes.c_double, ctypes.c_double, I, P, P, I, P, P, SZ,
                                 ctypes.POINTER(Opts), P, ctypes.POINTER(Stats)]),
        "hgv_dstebz_bufsize": (I, [P, I, ctypes.POINTER(SZ)]),
        "hgv_chegvx_bufsize": (I, [P, I, I, I, ctypes.POINTER(Opts), ctypes.POINTER(SZ)]),
        "hgv_chegvx": (I, [P, I, P, I, P, I, I, I, P, P, I, P, SZ, ctypes.POINTER(Opts), P,
                           ctypes.POINTER(Stats)]),
        "hgv_dsygvx_bufsize": (I, [P, I, I, I, ctypes.POINTER(Opts), ctypes.POINTER(SZ)]),
        "hgv_dsygvx": (I, [P, I, P, I, P, I, I, I, P, P, I, P, SZ, ctypes.POINTER(Opts), P,
                           ctypes.POINTER(Stats)]),
        "hgv_dstebz": (I, [P, I, P, P, I, I, P, P, SZ]),
        "hgv_dstebz_noalloc": (I, [P, I, P, P, I, I, P]),
        "hgv_zhetrd_bufsize": (I, [P, I, I, ctypes.POINTER(SZ)]),
        "hgv_zhetrd": (I, [P, I, I, P, I, P, P, P, P, SZ]),
        "hgv_zunmtr_tr": (I, [P, ctypes.c_char, I, I, I, P, I, P, P, I, P, SZ]),
        "hgv_v2_elems": (SZ, [I, I]),
        "hgv_v2_taus": (SZ, [I, I]),
        "hgv_dstedc": (I, [P, I, P, P, I, I, P, P, I, P, SZ, P]),
        "hgv_zunmtr_q2": (I, [P, ctypes.c_char, I, I, I, P, P, P, I, P, SZ]),
        "hgv_zunmtr_q1": (I, [P, ctypes.c_char, I, I, I, P, I, P, P, I, P, SZ]),
        "hgv_ztrsm_lh": (I, [P, I, I, P, I, P, I, P, SZ]),
        "hgv_zgemm": (I, [P, ctypes.c_char, ctypes.c_char, I, I, I, c128, P, I, P, I, c128, P, I]),
        "hgv_device_peaks": (I, [P, P, SZ, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
        "hgv_gauge_fix": (I, [P, I, I, P, I]),
        "hgv_zhegvx_backward_bufsize": (I, [P, I, I, I, ctypes.POINTER(SZ)]),
        "hgv_zhegvx_backward": (I, [P, I, I, I, P, P, I, P, P, I, P, I, P, I, P, SZ]),
        "hgv_zhegvx_batched_bufsize": (I, [P, I, P, P, P, P, ctypes.POINTER(Opts), ctypes.POINTER(SZ)]),
        "hgv_zhegvx_batched": (I, [P, I, P, P, P, P, P, P, P, P, P, P, P, ctypes.POINTER(Opts), P, SZ, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(status, where):
    if status != HGV_OK:
        raise HgvError(status, where)


# ---- one-to-one wrappers of the C ABI (pointers as Python ints) ------------------------
def hgv_create(device=0):
    h = P()
    _check(load().hgv_create(ctypes.byref(h), device), "hgv_create")
    return h


def hgv_destroy(ctx):
    _check(load().hgv_destroy(ctx), "hgv_destroy")


def hgv_set_stream(ctx, stream):
    _check(load().hgv_set_stream(ctx, stream), "hgv_set_stream")


def hgv_status_string(status):
    return load().hgv_status_string(status).decode()


def hgv_last_hip_error(ctx):
    return load().hgv_last_hip_error(ctx)


def hgv_default_nb(n, precision=HGV_FP64):
    return load().hgv_default_nb(n, precision)


def hgv_zhegvx_bufsize(ctx, n, il, iu, opts=None):
    out = SZ()
    _check(load().hgv_zhegvx_bufsize(ctx, n, il, iu, ctypes.byref(opts) if opts else None, ctypes.byref(out)),
           "hgv_zhegvx_bufsize")
    return out.value


def hgv_zhegvx(ctx, n, A, lda, B, ldb, il, iu, W, X, ldx, work, work_bytes, opts=None, d_info=None, stats=None):
    st = load().hgv_zhegvx(ctx, n, A, lda, B, ldb, il, iu, W, X, ldx, work, work_bytes,
                           ctypes.byref(opts) if opts else None, d_info,
                           ctypes.byref(stats) if stats is not None else None)
    _check(st, "hgv_zhegvx")


def hgv_stage_bufsize(ctx, stage, n, nb=0, m=0):
    out = SZ()
    _check(load().hgv_stage_bufsize(ctx, stage, n, nb, m, ctypes.byref(out)), "hgv_stage_bufsize")
    return out.value


def hgv_zpotrf(ctx, n, B, ldb, work, work_bytes, d_info):
    _check(load().hgv_zpotrf(ctx, n, B, ldb, work, work_bytes, d_info), "hgv_zpotrf")


def hgv_zhegst(ctx, n, A, lda, L, ldl, work, work_bytes):
    _check(load().hgv_zhegst(ctx, n, A, lda, L, ldl, work, work_bytes), "hgv_zhegst")


def hgv_zhe2hb(ctx, n, nb, A, lda, T1, work, work_bytes, d_info=None):
    _check(load().hgv_zhe2hb(ctx, n, nb, A, lda, T1, work, work_bytes, d_info), "hgv_zhe2hb")


def hgv_zhb2st(ctx, n, nb, A, lda, d, e, V2, tau2, work, work_bytes, d_info=None):
    _check(load().hgv_zhb2st(ctx, n, nb, A, lda, d, e, V2, tau2, work, work_bytes, d_info), "hgv_zhb2st")


def hgv_test_hooks(ctx, mask):
    _check(load().hgv_test_hooks(ctx, mask), "hgv_test_hooks")


def hgv_zhegvx_range_bufsize(ctx, n, mmax, opts=None):
    out = SZ()
    _check(load().hgv_zhegvx_range_bufsize(ctx, n, mmax, ctypes.byref(opts) if opts else None, ctypes.byref(out)),
           "hgv_zhegvx_range_bufsize")
    return out.value


def hgv_zhegvx_range(ctx, n, A, lda, B, ldb, vl, vu, mmax, W, X, ldx, d_m, work, work_bytes, opts=None,
                     d_info=None, stats=None):
    _check(load().hgv_zhegvx_range(ctx, n, A, lda, B, ldb, vl, vu, mmax, W, X, ldx, d_m, work, work_bytes,
                                   ctypes.byref(opts) if opts else None, d_info,
                                   ctypes.byref(stats) if stats is not None else None), "hgv_zhegvx_range")


def hgv_chegvx_bufsize(ctx, n, il, iu, opts=None):
    out = SZ()
    _check(load().hgv_chegvx_bufsize(ctx, n, il, iu, ctypes.byref(opts) if opts else None, ctypes.byref(out)),
           "hgv_chegvx_bufsize")
    return out.value


def hgv_chegvx(ctx, n, A, lda, B, ldb, il, iu, W, X, ldx, work, work_bytes, opts=None, d_info=None, stats=None):
    _check(load().hgv_chegvx(ctx, n, A, lda, B, ldb, il, iu, W, X, ldx, work, work_bytes,
                             ctypes.byref(opts) if opts else None, d_info,
                             ctypes.byref(stats) if stats is not None else None), "hgv_chegvx")


def hgv_dsygvx_bufsize(ctx, n, il, iu, opts=None):
    out = SZ()
    _check(load().hgv_dsygvx_bufsize(ctx, n, il, iu, ctypes.byref(opts) if opts else None, ctypes.byref(out)),
           "hgv_dsygvx_bufsize")
    return out.value


def hgv_dsygvx(ctx, n, A, lda, B, ldb, il, iu, W, X, ldx, work, work_bytes, opts=None, d_info=None, stats=None):
    _check(load().hgv_dsygvx(ctx, n, A, lda, B, ldb, il, iu, W, X, ldx, work, work_bytes,
                             ctypes.byref(opts) if opts else None, d_info,
                             ctypes.byref(stats) if stats is not None else None), "hgv_dsygvx")


def hgv_dstebz_bufsize(ctx, n):
    out = SZ()
    _check(load().hgv_dstebz_bufsize(ctx, n, ctypes.byref(out)), "hgv_dstebz_bufsize")
    return out.value


def hgv_dstebz(ctx, n, d, e, il, iu, W, work, work_bytes):
    _check(load().hgv_dstebz(ctx, n, d, e, il, iu, W, work, work_bytes), "hgv_dstebz")


def hgv_zhetrd_bufsize(ctx, n, nb):
    out = SZ()
    _check(load().hgv_zhetrd_bufsize(ctx, n, nb, ctypes.byref(out)), "hgv_zhetrd_bufsize")
    return out.value


def hgv_zhetrd(ctx, n, nb, A, lda, d, e, T1, work, work_bytes):
    _check(load().hgv_zhetrd(ctx, n, nb, A, lda, d, e, T1, work, work_bytes), "hgv_zhetrd")


def hgv_zunmtr_tr(ctx, trans, n, nb, m, A, lda, T1, Y, ldy, work, work_bytes):
    _check(load().hgv_zunmtr_tr(ctx, trans.encode() if isinstance(trans, str) else trans, n, nb, m, A, lda, T1, Y,
                                ldy, work, work_bytes), "hgv_zunmtr_tr")


def hgv_dstebz_noalloc(ctx, n, d, e, il, iu, W):
    _check(load().hgv_dstebz_noalloc(ctx, n, d, e, il, iu, W), "hgv_dstebz_noalloc")


def hgv_v2_elems(n, nb):
    return load().hgv_v2_elems(n, nb)


def hgv_v2_taus(n, nb):
    return load().hgv_v2_taus(n, nb)


def hgv_dstedc(ctx, n, d, e, il, iu, lam, Z, ldz, work, work_bytes, d_info):
    _check(load().hgv_dstedc(ctx, n, d, e, il, iu, lam, Z, ldz, work, work_bytes, d_info), "hgv_dstedc")


def hgv_zunmtr_q2(ctx, trans, n, nb, m, V2, tau2, Y, ldy, work, work_bytes):
    _check(load().hgv_zunmtr_q2(ctx, trans.encode() if isinstance(trans, str) else trans, n, nb, m, V2, tau2, Y,
                                ldy, work, work_bytes), "hgv_zunmtr_q2")


def hgv_zunmtr_q1(ctx, trans, n, nb, m, A, lda, T1, Y, ldy, work, work_bytes):
    _check(load().hgv_zunmtr_q1(ctx, trans.encode() if isinstance(trans, str) else trans, n, nb, m, A, lda, T1, Y,
                                ldy, work, work_bytes), "hgv_zunmtr_q1")


def hgv_ztrsm_lh(ctx, n, m, L, ldl, X, ldx, work, work_bytes):
    _check(load().hgv_ztrsm_lh(ctx, n, m, L, ldl, X, ldx, work, work_bytes), "hgv_ztrsm_lh")


def hgv_zgemm(ctx, opa, opb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc):
    a = c128(alpha.real, alpha.imag)
    b = c128(beta.real, beta.imag)
    _check(load().hgv_zgemm(ctx, opa.encode(), opb.encode(), m, n, k, a, A, lda, B, ldb, b, C, ldc), "hgv_zgemm")


def hgv_device_peaks(ctx, work, work_bytes):
    """Measured FP64 MFMA TFLOP/s and copy GB/s (read + write) of the context's device."""
    t = ctypes.c_double(0.0)
    g = ctypes.c_double(0.0)
    _check(load().hgv_device_peaks(ctx, work, work_bytes, ctypes.byref(t), ctypes.byref(g)), "hgv_device_peaks")
    return t.value, g.value


def hgv_gauge_fix(ctx, n, m, X, ldx):
    _check(load().hgv_gauge_fix(ctx, n, m, X, ldx), "hgv_gauge_fix")


def hgv_zhegvx_backward_bufsize(ctx, n, il, iu):
    out = SZ()
    _check(load().hgv_zhegvx_backward_bufsize(ctx, n, il, iu, ctypes.byref(out)), "hgv_zhegvx_backward_bufsize")
    return out.value


def hgv_zhegvx_backward(ctx, n, il, iu, lam, Xall, ldxa, Wbar, Xbar, ldxb, Abar, ldab, Bbar, ldbb, work, work_bytes):
    _check(load().hgv_zhegvx_backward(ctx, n, il, iu, lam, Xall, ldxa, Wbar, Xbar, ldxb, Abar, ldab, Bbar, ldbb,
                                      work, work_bytes), "hgv_zhegvx_backward")


def _iarr(vals):
    return (ctypes.c_int * len(vals))(*vals)


def _parr(vals):
    return (ctypes.c_void_p * len(vals))(*vals)


def hgv_zhegvx_batched_bufsize(ctx, n, il, iu, nb=None, opts=None):
    out = SZ()
    _check(load().hgv_zhegvx_batched_bufsize(ctx, len(n), _iarr(n), _iarr(il), _iarr(iu),
                                             _iarr(nb) if nb is not None else None,
                                             ctypes.byref(opts) if opts is not None else None, ctypes.byref(out)),
           "hgv_zhegvx_batched_bufsize")
    return out.value


def hgv_zhegvx_batched(ctx, n, A, lda, B, ldb, il, iu, W, X, ldx, nb, work, work_bytes, d_info, opts=None):
    _check(load().hgv_zhegvx_batched(ctx, len(n), _iarr(n), _parr(A), _iarr(lda), _parr(B), _iarr(ldb), _iarr(il),
                                     _iarr(iu), _parr(W), _parr(X), _iarr(ldx),
                                     _iarr(nb) if nb is not None else None,
                                     ctypes.byref(opts) if opts is not None else None, work, work_bytes, d_info),
           "hgv_zhegvx_batched")


# ---- torch marshalling ---------------------------------------------------------------------
from . import tensors  # noqa: E402  (torch-facing helpers)
from .tensors import Context, eigh, colmajor, from_colmajor  # noqa: E402,F401
from .autograd import EighGeneralized, eigh_differentiable  # noqa: E402,F401
