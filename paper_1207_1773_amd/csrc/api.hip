// api.hip -- the extern "C" entry points declared in include/hgv.h: argument
// checks (before any launch), workspace planning, stage sequencing for the
// full solve of Algorithm 1, optional per-stage event timing.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <new>

#include "hgv_internal.h"

using namespace hgv;

namespace {

constexpr int kMagic = 0x68677631;

bool ctx_ok(hgv_ctx_t c) { return c != nullptr && c->magic == kMagic; }

struct NotSupported {};

// Wraps an entry point body: selects the device, converts internal
// exceptions into status codes.
template <class F>
int guarded(hgv_ctx_t ctx, F &&body) {
    if (!ctx_ok(ctx)) return HGV_E_CTX;
    try {
        HGV_HIP(hipSetDevice(ctx->device));
        return body();
    } catch (const HipFail &f) {
        ctx->last_hip_error = (int)f.err;
        return HGV_E_HIP;
    } catch (const WorkspaceShort &) {
        return HGV_E_WORKSPACE;
    } catch (const NotSupported &) {
        return HGV_E_NOTSUP;
    } catch (const std::bad_alloc &) {
        return HGV_E_HIP;
    }
}

int resolve_nb(int n, const hgv_opts *o) {
    int nb = (o && o->nb > 0) ? o->nb : hgv_default_nb(n, o ? o->precision : HGV_FP64);
    return std::max(1, nb);
}

// Complex copy of a real n x m matrix (Z -> Y).
__global__ void real_to_complex_kernel(int n, int m, const double *Z, int ldz, double2 *Y, int ldy) {
    int i = blockIdx.x * 64 + (threadIdx.x & 63);
    int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i < n && j < m) Y[i + (size_t)j * ldy] = make_double2(Z[i + (size_t)j * ldz], 0.0);
}

__global__ void copy_doubles_kernel(int n, const double *a, double *b) {
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) b[i] = a[i];
}

// W[s] = lambda[range[0] - 1 + s] for s < range[2], 0 for the other slots.
__global__ void select_vals_kernel(int nslot, const double *lambda, const int *range, double *W) {
    int s = blockIdx.x * 256 + threadIdx.x;
    if (s < nslot) W[s] = s < range[2] ? lambda[range[0] - 1 + s] : 0.0;
}

__global__ void copy_int_kernel(const int *src, int *dst) { *dst = *src; }

}  // namespace

namespace hgv {

void standard_fp64(hgv_ctx_s *ctx, int n, double2 *A, int lda, int il, int iu, double *W, double2 *X, int ldx,
                   Arena &ar, int nb, int *d_info, StageTimer *tm, const ValueRange *vr, bool values_only,
                   bool one_stage) {
    const int m = iu - il + 1;
    const int np = cdiv(n, nb);
    const size_t mk0 = ar.mark();
    const double N = n, M = m;
    if (one_stage) {
        // Sec. 4.1: one-stage tridiagonalisation, then the tridiagonal solve and a
        // single back-transformation (reported as the band-reduction and Q1 stages)
        double2 *T1 = ar.take<double2>((size_t)np * nb * nb);
        double *d = ar.take<double>(n);
        double *e = ar.take<double>(std::max(n - 1, 1));
        double *lambda = values_only ? nullptr : ar.take<double>(n);
        double *Z = values_only ? nullptr : ar.take<double>((size_t)n * m);
        const size_t mk = ar.mark();
        const bool run = !ar.measuring();
        if (tm) tm->begin(HGV_ST_HE2HB);
        hetrd_run(ctx, n, nb, A, lda, d, e, T1, ar);
        ar.release(mk);
        if (tm) tm->end(HGV_ST_HE2HB, 16.0 / 3.0 * N * N * N);
        if (vr) sturm_range_run(ctx, n, d, e, vr->vl, vr->vu, m, vr->range, ar);
        ar.release(mk);
        const int *d_range = vr ? vr->range : nullptr;
        if (tm) tm->begin(HGV_ST_STEDC);
        if (values_only) {
            stebz_run(ctx, n, d, e, il, m, d_range, W, ar);
            ar.release(mk);
            if (tm) tm->end(HGV_ST_STEDC, 0.0);
            ar.release(mk0);
            return;
        }
        stedc_run(ctx, n, d, e, il, iu, lambda, Z, n, ar, d_info, {}, d_range);
        ar.release(mk);
        if (run) {
            if (d_range)
                hipLaunchKernelGGL(select_vals_kernel, dim3(cdiv(m, 256)), dim3(256), 0, ctx->stream, m, lambda,
                                   d_range, W);
            else
                hipLaunchKernelGGL(copy_doubles_kernel, dim3(cdiv(m, 256)), dim3(256), 0, ctx->stream, m,
                                   lambda + (il - 1), W);
            HGV_LAUNCH_CHECK();
            hipLaunchKernelGGL(real_to_complex_kernel, dim3(cdiv(n, 64), cdiv(m, 4)), dim3(256), 0, ctx->stream, n,
                               m, Z, n, X, ldx);
            HGV_LAUNCH_CHECK();
        }
        if (tm) tm->end(HGV_ST_STEDC, 4.0 / 3.0 * N * N * N);
        if (tm) tm->begin(HGV_ST_Q1);
        unmtr_q1_t<double2>(ctx, n, nb, m, A, lda, T1, X, ldx, false, ar, 1);
        ar.release(mk);
        if (tm) tm->end(HGV_ST_Q1, 8.0 * N * N * M);
        ar.release(mk0);
        return;
    }
    if (values_only) {
        // Band reduction and bulge chasing without keeping the second-stage
        // reflectors, eigenvalues by Sturm-count multisection, no back-transformation.
        double2 *T1 = ar.take<double2>((size_t)np * nb * nb);
        double *d = ar.take<double>(n);
        double *e = ar.take<double>(std::max(n - 1, 1));
        const size_t mk = ar.mark();
        if (tm) tm->begin(HGV_ST_HE2HB);
        he2hb_run(ctx, n, nb, A, lda, T1, ar, d_info);
        ar.release(mk);
        if (tm) tm->end(HGV_ST_HE2HB, 16.0 / 3.0 * N * N * N);
        if (tm) tm->begin(HGV_ST_HB2ST);
        hb2st_run(ctx, n, nb, A, lda, d, e, nullptr, nullptr, ar, d_info);
        ar.release(mk);
        if (tm) tm->end(HGV_ST_HB2ST, 24.0 * N * N * nb);
        if (tm) tm->begin(HGV_ST_STEDC);
        if (vr) sturm_range_run(ctx, n, d, e, vr->vl, vr->vu, m, vr->range, ar);
        ar.release(mk);
        stebz_run(ctx, n, d, e, il, m, vr ? vr->range : nullptr, W, ar);
        ar.release(mk);
        if (tm) tm->end(HGV_ST_STEDC, 0.0);
        ar.release(mk0);
        return;
    }
    double2 *T1 = ar.take<double2>((size_t)np * nb * nb);
    double *d = ar.take<double>(n);
    double *e = ar.take<double>(std::max(n - 1, 1));
    double *lambda = ar.take<double>(n);
    double2 *V2 = ar.take<double2>(v2_elems(n, nb));
    double2 *tau2 = ar.take<double2>(v2_taus(n, nb));
    double2 *T2 = ar.take<double2>(q2_t_elems(n, nb));   // Q2's group T factors (built during stedc)
    double *Z = ar.take<double>((size_t)n * m);
    const size_t mk = ar.mark();
    const bool run = !ar.measuring();

    if (tm) tm->begin(HGV_ST_HE2HB);
    he2hb_run(ctx, n, nb, A, lda, T1, ar, d_info);
    ar.release(mk);
    if (tm) tm->end(HGV_ST_HE2HB, 16.0 / 3.0 * N * N * N);

    if (tm) tm->begin(HGV_ST_HB2ST);
    hb2st_run(ctx, n, nb, A, lda, d, e, V2, tau2, ar, d_info);
    ar.release(mk);
    if (tm) tm->end(HGV_ST_HB2ST, 24.0 * N * N * nb);
    // selection by value: the index range from Sturm counts of T, on the device
    if (vr) sturm_range_run(ctx, n, d, e, vr->vl, vr->vu, m, vr->range, ar);
    ar.release(mk);
    const int *d_range = vr ? vr->range : nullptr;

    // the T factors of Q2's reflector groups need only the bulge chasing's
    // reflectors: built on a side stream while the tridiagonal solver runs the
    // serial kernels of its last merge level (beside its small, latency-bound
    // levels the build slowed them down)
    const bool side = run && !ctx->concurrent;
    hipStream_t main = ctx->stream;
    bool built = false;
    auto build_t_side = [&]() {
        ensure_lookahead_stream(ctx);
        HGV_HIP(hipEventRecord(ctx->la_ev[1], ctx->stream));
        HGV_HIP(hipStreamWaitEvent(ctx->la_stream[1], ctx->la_ev[1], 0));
        hipStream_t cur = ctx->stream;
        ctx->stream = ctx->la_stream[1];
        try {
            q2_build_t<double2>(ctx, n, nb, V2, tau2, T2);
        } catch (...) {
            ctx->stream = cur;
            throw;
        }
        ctx->stream = cur;
        HGV_HIP(hipEventRecord(ctx->la_ev[1], ctx->la_stream[1]));
        built = true;
    };
    if (run && !side) {
        q2_build_t<double2>(ctx, n, nb, V2, tau2, T2);
        built = true;
    }

    if (tm) tm->begin(HGV_ST_STEDC);
    if (side) stedc_run(ctx, n, d, e, il, iu, lambda, Z, n, ar, d_info, build_t_side, d_range);
    else stedc_run(ctx, n, d, e, il, iu, lambda, Z, n, ar, d_info, {}, d_range);
    if (side && !built) build_t_side();   // no merge level (n within one leaf)
    ar.release(mk);
    if (run) {
        if (d_range)
            hipLaunchKernelGGL(select_vals_kernel, dim3(cdiv(m, 256)), dim3(256), 0, ctx->stream, m, lambda,
                               d_range, W);
        else
            hipLaunchKernelGGL(copy_doubles_kernel, dim3(cdiv(m, 256)), dim3(256), 0, ctx->stream, m,
                               lambda + (il - 1), W);
        HGV_LAUNCH_CHECK();
        hipLaunchKernelGGL(real_to_complex_kernel, dim3(cdiv(n, 64), cdiv(m, 4)), dim3(256), 0, ctx->stream, n,
                           m, Z, n, X, ldx);
        HGV_LAUNCH_CHECK();
    }
    if (tm) tm->end(HGV_ST_STEDC, 4.0 / 3.0 * N * N * N);

    if (side) HGV_HIP(hipStreamWaitEvent(main, ctx->la_ev[1], 0));
    if (tm) tm->begin(HGV_ST_Q2);
    if (run) q2_apply_t<double2>(ctx, n, nb, m, V2, T2, X, ldx, false);
    ar.release(mk);
    if (tm) tm->end(HGV_ST_Q2, 8.0 * N * N * M);

    if (tm) tm->begin(HGV_ST_Q1);
    unmtr_q1_run(ctx, n, nb, m, A, lda, T1, X, ldx, ar);
    ar.release(mk);
    if (tm) tm->end(HGV_ST_Q1, 8.0 * N * N * M);
    ar.release(mk0);
}

}  // namespace hgv

namespace {

// Full solve (Algorithm 1 with the two-stage Algorithm 2): potrf and hegst in
// FP64, the standard eigensolve in FP64 or mixed precision, x = L^-H y in
// FP64 (skipped for eigenvalues only).  With vr the pairs in (vl, vu] are
// chosen on the device and il..iu only give the number of slots.  Shared by
// the size query (arena without base) and the run.
void zhegvx_full(hgv_ctx_s *ctx, int n, double2 *A, int lda, double2 *B, int ldb, int il, int iu, double *W,
                 double2 *X, int ldx, Arena &ar, int nb, const hgv_opts *opts, int *d_info, StageTimer *tm,
                 MixedResult *mres, bool fixed_iters, const ValueRange *vr = nullptr) {
    const int m = iu - il + 1;
    const size_t mk = ar.mark();
    const bool run = !ar.measuring();
    const double N = n, M = m;

    if (run) set_info(ctx, d_info, 0);
    // potrf, then hegst; the reduction of the leading block overlaps the
    // factorisation of the trailing one
    if (tm) tm->begin(HGV_ST_POTRF);
    potrf_hegst_run(ctx, n, B, ldb, A, lda, ar, d_info, n, tm, 4.0 / 3.0 * N * N * N);
    ar.release(mk);
    if (tm) tm->end(HGV_ST_HEGST, 4.0 * N * N * N);

    if (opts && opts->precision == HGV_MIXED) {
        int iters = opts->max_refine_iters > 0 ? opts->max_refine_iters : 3;
        double tol = opts->refine_tol > 0.0 ? opts->refine_tol : 32.0 * DBL_EPSILON * std::sqrt((double)n);
        MixedResult local;
        mixed_standard(ctx, n, A, lda, il, iu, W, X, ldx, ar, nb, opts->max_refine_iters < 0 ? 0 : iters, tol,
                       fixed_iters, d_info, tm, mres ? mres : &local);
    } else {
        standard_fp64(ctx, n, A, lda, il, iu, W, X, ldx, ar, nb, d_info, tm, vr, opts && opts->values_only,
                      opts && opts->one_stage);
    }
    ar.release(mk);
    if (opts && opts->values_only) return;

    if (tm) tm->begin(HGV_ST_TRSM);
    trsm_lh_run(ctx, n, m, B, ldb, X, ldx, ar);
    ar.release(mk);
    if (tm) tm->end(HGV_ST_TRSM, 4.0 * N * N * M);
}

}  // namespace

extern "C" {

int hgv_create(hgv_ctx_t *ctx, int device) {
    if (!ctx) return -1;
    *ctx = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return -2;
    // the allocation-free entry point's device array: its address is looked up
    // here, once per device, with that device current
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) return HGV_E_HIP;
    try {
        if (hipSetDevice(device) != hipSuccess) return HGV_E_HIP;
        stebz_scratch_init(device);
    } catch (const HipFail &) {
        (void)hipSetDevice(prev);
        return HGV_E_HIP;
    }
    if (hipSetDevice(prev) != hipSuccess) return HGV_E_HIP;
    hgv_ctx_s *c = new (std::nothrow) hgv_ctx_s();
    if (!c) return HGV_E_HIP;
    c->device = device;
    c->magic = kMagic;
    *ctx = c;
    return HGV_OK;
}

int hgv_destroy(hgv_ctx_t ctx) {
    if (!ctx_ok(ctx)) return HGV_E_CTX;
    (void)hipSetDevice(ctx->device);
    for (hipStream_t st : ctx->side) (void)hipStreamDestroy(st);
    for (hipEvent_t e : ctx->side_ev) (void)hipEventDestroy(e);
    for (hipStream_t st : ctx->la_stream)
        if (st) (void)hipStreamDestroy(st);
    for (hipEvent_t e : ctx->la_ev)
        if (e) (void)hipEventDestroy(e);
    if (ctx->fork_ev) (void)hipEventDestroy(ctx->fork_ev);
    for (hipEvent_t e : ctx->ev_free) (void)hipEventDestroy(e);
    for (auto &p : ctx->ev_pending) {
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
    }
    ctx->magic = 0;
    delete ctx;
    return HGV_OK;
}

int hgv_set_stream(hgv_ctx_t ctx, void *stream) {
    if (!ctx_ok(ctx)) return HGV_E_CTX;
    ctx->stream = static_cast<hipStream_t>(stream);
    return HGV_OK;
}

int hgv_last_hip_error(hgv_ctx_t ctx) { return ctx_ok(ctx) ? ctx->last_hip_error : 0; }

int hgv_test_hooks(hgv_ctx_t ctx, int mask) {
    if (!ctx_ok(ctx)) return HGV_E_CTX;
    if (mask & ~(HGV_TEST_WAIT_FAIL | HGV_TEST_NAN_RESIDUAL | HGV_TEST_HB2ST_SWEEPS | HGV_TEST_HOUSEHOLDER_PANELS))
        return -2;
    ctx->test_hooks = mask;
    return HGV_OK;
}

const char *hgv_status_string(int status) {
    if (status == HGV_OK) return "success";
    if (status < 0) return "invalid argument";
    switch (status) {
        case HGV_E_HIP: return "HIP runtime error";
        case HGV_E_WORKSPACE: return "workspace too small";
        case HGV_E_CTX: return "invalid context";
        case HGV_E_NOTSUP: return "unsupported option";
    }
    return "unknown status";
}

int hgv_default_nb(int n, int precision) {
    (void)precision;
    if (n <= 1024) return 32;
    return 64;
}

int hgv_zhegvx_bufsize(hgv_ctx_t ctx, int n, int il, int iu, const hgv_opts *opts, size_t *bytes) {
    if (!ctx_ok(ctx)) return HGV_E_CTX;
    if (n < 0) return -2;
    if (n > 0 && (il < 1 || il > n)) return -3;
    if (n > 0 && (iu < il || iu > n)) return -4;
    if (!bytes) return -6;
    *bytes = 0;
    if (n == 0) return HGV_OK;
    if (opts && opts->precision != HGV_FP64 && opts->precision != HGV_MIXED) return -5;
    if (opts && opts->values_only && opts->precision == HGV_MIXED) return HGV_E_NOTSUP;
    if (opts && opts->one_stage && opts->precision == HGV_MIXED) return HGV_E_NOTSUP;
    return guarded(ctx, [&]() {
        Arena ar;
        zhegvx_full(ctx, n, nullptr, n, nullptr, n, il, iu, nullptr, nullptr, n, ar, resolve_nb(n, opts), opts,
                    nullptr, nullptr, nullptr, false);
        *bytes = ar.peak + 256;
        return HGV_OK;
    });
}

int hgv_zhegvx(hgv_ctx_t ctx, int n, hgv_c128 *A, int lda, hgv_c128 *B, int ldb, int il, int iu, double *W,
               hgv_c128 *X, int ldx, void *work, size_t work_bytes, const hgv_opts *opts, int *d_info,
               hgv_stats *stats) {
    if (!ctx_ok(ctx)) return HGV_E_CTX;
    if (n < 0) return -2;
    const int nn = std::max(1, n);
    if (n > 0 && !A) return -3;
    if (lda < nn) return -4;
    if (n > 0 && !B) return -5;
    if (ldb < nn) return -6;
    if (n > 0 && (il < 1 || il > n)) return -7;
    if (n > 0 && (iu < il || iu > n)) return -8;
    const bool vals = opts && opts->values_only;
    if (n > 0 && !W) return -9;
    if (n > 0 && !X && !vals) return -10;
    if (!vals && ldx < nn) return -11;
    if (opts && opts->precision != HGV_FP64 && opts->precision != HGV_MIXED) return -14;
    if (opts && opts->nb < 0) return -14;
    if (vals && opts->precision == HGV_MIXED) return HGV_E_NOTSUP;
    if (opts && opts->one_stage && opts->precision == HGV_MIXED) return HGV_E_NOTSUP;
    if (opts && opts->one_stage && opts->nb > 64) return -14;
    if (n == 0) return guarded(ctx, [&]() {
        set_info(ctx, d_info, 0);
        return HGV_OK;
    });
    size_t need = 0;
    int st = hgv_zhegvx_bufsize(ctx, n, il, iu, opts, &need);
    if (st != HGV_OK) return st;
    if (n > 0 && !work) return -12;
    if (work_bytes < need) return HGV_E_WORKSPACE;
    if (reinterpret_cast<uintptr_t>(work) & 255) return -12;
    return guarded(ctx, [&]() {
        // under stream capture the refinement runs a fixed number of
        // iterations (no host-side convergence check)
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        HGV_HIP(hipStreamIsCapturing(ctx->stream, &cap));
        const bool fixed = cap != hipStreamCaptureStatusNone;
        StageTimer tm(ctx, stats);
        Arena ar(work, work_bytes);
        int nb = resolve_nb(n, opts);
        MixedResult mres;
        zhegvx_full(ctx, n, reinterpret_cast<double2 *>(A), lda, reinterpret_cast<double2 *>(B), ldb, il, iu, W,
                    reinterpret_cast<double2 *>(X), ldx, ar, nb, opts, d_info, stats ? &tm : nullptr, &mres, fixed);
        if (stats) {
            tm.finish();
            stats->nb = nb;
            stats->refine_iters = mres.iters;
            stats->refine_resid = mres.rho;
            stats->fallback = mres.fallback;
        }
        return HGV_OK;
    });
}

// ---- complex64 and real front ends (variants.hip) --------------------------------------
int hgv_chegvx_bufsize(hgv_ctx_t ctx, int n, int il, int iu, const hgv_opts *opts, size_t *bytes) {
    if (!ctx_ok(ctx)) return HGV_E_CTX;
    if (n < 0) return -2;
    if (n > 0 && (il < 1 || il > n)) return -3;
    if (n > 0 && (iu < il || iu > n)) return -4;
    if (!bytes) return -6;
    *bytes = 0;
    if (opts && opts->precision != HGV_FP64) return opts->precision == HGV_MIXED ? HGV_E_NOTSUP : -5;
    if (opts && opts->one_stage) return HGV_E_NOTSUP;
    if (n == 0) return HGV_OK;
    return guarded(ctx, [&]() {
        Arena ar;
        chegvx_full(ctx, n, nullptr, n, nullptr, n, il, iu, nullptr, nullptr, n, ar, resolve_nb(n, opts),
                    opts && opts->values_only, nullptr, nullptr);
        *bytes = ar.peak + 256;
        return HGV_OK;
    });
}

int hgv_chegvx(hgv_ctx_t ctx, int n, hgv_c64 *A, int lda, hgv_c64 *B, int ldb, int il, int iu, float *W, hgv_c64 *X,
               int ldx, void *work, size_t work_bytes, const hgv_opts *opts, int *d_info, hgv_stats *stats) {
    if (!ctx_ok(ctx)) return HGV_E_CTX;
    if (n < 0) return -2;
    const int nn = std::max(1, n);
    const bool vals = opts && opts->values_only;
    if (n > 0 && !A) return -3;
    if (lda < nn) return -4;
    if (n > 0 && !B) return -5;
    if (ldb < nn) return -6;
    if (n > 0 && (il < 1 || il > n)) return -7;
    if (n > 0 && (iu < il || iu > n)) return -8;
    if (n > 0 && !W) return -9;
    if (n > 0 && !X && !vals) return -10;
    if (!vals && ldx < nn) return -11;
    if (opts && opts->precision != HGV_FP64) return opts->precision == HGV_MIXED ? HGV_E_NOTSUP : -14;
    if (opts && opts->nb < 0) return -14;
    if (opts && opts->one_stage) return HGV_E_NOTSUP;
    if (n == 0) return guarded(ctx, [&]() {
        set_info(ctx, d_info, 0);
        return HGV_OK;
    });
    size_t need = 0;
    int st = hgv_chegvx_bufsize(ctx, n, il, iu, opts, &need);
    if (st != HGV_OK) return st;
    if (!work || (reinterpret_cast<uintptr_t>(work) & 255)) return -12;
    if (work_bytes < need) return HGV_E_WORKSPACE;
    return guarded(ctx, [&]() {
        StageTimer tm(ctx, stats);
        Arena ar(work, work_bytes);
        const int nb = resolve_nb(n, opts);
        chegvx_full(ctx, n, reinterpret_cast<float2 *>(A), lda, reinterpret_cast<float2 *>(B), ldb, il, iu, W,
                    reinterpret_cast<float2 *>(X), ldx, ar, nb, vals, d_info, stats ? &tm : nullptr);
        if (stats) {
            tm.finish();
            stats->nb = nb;
        }
        return HGV_OK;
    });
}

// Real pencils: complex copies in the workspace, the complex-double solve,
// real parts back (see variants.hip).
static void dsygvx_plan(hgv_ctx_s *ctx, int n, double *A, int lda, double *B, int ldb, int il, int iu, double *W,
                        double *X, int ldx, Arena &ar, int nb, const hgv_opts *opts, int *d_info, StageTimer *tm,
                        MixedResult *mres, bool fixed) {
    const int m = iu - il + 1;
    const bool vals = opts && opts->values_only;
    double2 *Az = ar.take<double2>((size_t)n * n);
    double2 *Bz = ar.take<double2>((size_t)n * n);
    double2 *Xz = vals ? nullptr : ar.take<double2>((size_t)n * m);
    const bool run = !ar.measuring();
    if (run) {
        real_to_complex(ctx, n, n, A, lda, Az, n);
        real_to_complex(ctx, n, n, B, ldb, Bz, n);
    }
    zhegvx_full(ctx, n, Az, n, Bz, n, il, iu, W, Xz, n, ar, nb, opts, d_info, tm, mres, fixed);
    if (run) {
        complex_real_part(ctx, n, n, Bz, n, B, ldb, true);
        if (!vals) complex_real_part(ctx, n, m, Xz, n, X, ldx, false);
    }
}

int hgv_dsygvx_bufsize(hgv_ctx_t ctx, int n, int il, int iu, const hgv_opts *opts, size_t *bytes) {
    if (!ctx_ok(ctx)) return HGV_E_CTX;
    if (n < 0) return -2;
    if (n > 0 && (il < 1 || il > n)) return -3;
    if (n > 0 && (iu < il || iu > n)) return -4;
    if (!bytes) return -6;
    *bytes = 0;
    if (opts && opts->precision != HGV_FP64 && opts->precision != HGV_MIXED) return -5;
    if (opts && opts->values_only && opts->precision == HGV_MIXED) return HGV_E_NOTSUP;
    if (n == 0) return HGV_OK;
    return guarded(ctx, [&]() {
        Arena ar;
        dsygvx_plan(ctx, n, nullptr, n, nullptr, n, il, iu, nullptr, nullptr, n, ar, resolve_nb(n, opts), opts,
                    nullptr, nullptr, nullptr, false);
        *bytes = ar.peak + 256;
        return HGV_OK;
    });
}

int hgv_dsygvx(hgv_ctx_t ctx, int n, double *A, int lda, double *B, int ldb, int il, int iu, double *W, double *X,
               int ldx, void *work, size_t work_bytes, const hgv_opts *opts, int *d_info, hgv_stats *stats) {
    if (!ctx_ok(ctx)) return HGV_E_CTX;
    if (n < 0) return -2;
    const int nn = std::max(1, n);
    const bool vals = opts && opts->values_only;
    if (n > 0 && !A) return -3;
    if (lda < nn) return -4;
    if (n > 0 && !B) return -5;
    if (ldb < nn) return -6;
    if (n > 0 && (il < 1 || il > n)) return -7;
    if (n > 0 && (iu < il || iu > n)) return -8;
    if (n > 0 && !W) return -9;
    if (n > 0 && !X && !vals) return -10;
    if (!vals && ldx < nn) return -11;
    if (opts && opts->precision != HGV_FP64 && opts->precision != HGV_MIXED) return -14;
    if (opts && opts->nb < 0) return -14;
    if (vals && opts->precision == HGV_MIXED) return HGV_E_NOTSUP;
    if (n == 0) return guarded(ctx, [&]() {
        set_info(ctx, d_info, 0);
        return HGV_OK;
    });
    size_t need = 0;
    int st = hgv_dsygvx_bufsize(ctx, n, il, iu, opts, &need);
    if (st != HGV_OK) return st;
    if (!work || (reinterpret_cast<uintptr_t>(work) & 255)) return -12;
    if (work_bytes < need) return HGV_E_WORKSPACE;
    return guarded(ctx, [&]() {
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        HGV_HIP(hipStreamIsCapturing(ctx->stream, &cap));
        StageTimer tm(ctx, stats);
        Arena ar(work, work_bytes);
        const int nb = resolve_nb(n, opts);
        MixedResult mres;
        dsygvx_plan(ctx, n, A, lda, B, ldb, il, iu, W, X, ldx, ar, nb, opts, d_info, stats ? &tm : nullptr, &mres,
                    cap != hipStreamCaptureStatusNone);
        if (stats) {
            tm.finish();
            stats->nb = nb;
            stats->refine_iters = mres.iters;
            stats->refine_resid = mres.rho;
            stats->fallback = mres.fallback;
        }
        return HGV_OK;
    });
}

// ---- stage entry points -----------------------------------------------------------
static void stage_plan(hgv_ctx_s *ctx, int stage, int n, int nb, int m, Arena &ar) {
    switch (stage) {
        case HGV_ST_POTRF: potrf_run(ctx, n, nullptr, n, ar, nullptr, 0); break;
        case HGV_ST_HEGST: hegst_run(ctx, n, nullptr, n, nullptr, n, ar); break;
        case HGV_ST_HE2HB: he2hb_run(ctx, n, nb, nullptr, n, nullptr, ar); break;
        case HGV_ST_HB2ST: hb2st_run(ctx, n, nb, nullptr, n, nullptr, nullptr, nullptr, nullptr, ar); break;
        case HGV_ST_STEDC: stedc_run(ctx, n, nullptr, nullptr, 1, std::max(m, 1), nullptr, nullptr, n, ar, nullptr); break;
        case HGV_ST_Q2: unmtr_q2_run(ctx, n, nb, m, nullptr, nullptr, nullptr, n, ar); break;
        case HGV_ST_Q1: unmtr_q1_run(ctx, n, nb, m, nullptr, n, nullptr, nullptr, n, ar); break;
        case HGV_ST_TRSM: trsm_lh_run(ctx, n, m, nullptr, n, nullptr, n, ar); break;
        default: throw NotSupported{};
    }
}

int hgv_stage_bufsize(hgv_ctx_t ctx, int stage, int n, int nb, int m, size_t *bytes) {
    if (!ctx_ok(ctx)) return HGV_E_CTX;
    if (stage < 0 || stage >= HGV_NSTAGES) return -2;
    if (n < 0) return -3;
    if (nb < 0) return -4;
    if (m < 0) return -5;
    if (!bytes) return -6;
    *bytes = 0;
    if (n == 0) return HGV_OK;
    if (nb == 0) nb = hgv_default_nb(n, HGV_FP64);
    return guarded(ctx, [&]() {
        Arena ar;
        stage_plan(ctx, stage, n, nb, m, ar);
        *bytes = ar.peak + 256;
        return HGV_OK;
    });
}

static int check_work(hgv_ctx_t ctx, int stage, int n, int nb, int m, void *work, size_t work_bytes,
                      int argno) {
    size_t need = 0;
    int st = hgv_stage_bufsize(ctx, stage, n, nb, m, &need);
    if (st != HGV_OK) return st;
    if (need > 256 && !work) return -argno;
    if (work && (reinterpret_cast<uintptr_t>(work) & 255)) return -argno;
    if (work_bytes < need && need > 256) return HGV_E_WORKSPACE;
    return HGV_OK;
}

int hgv_zpotrf(hgv_ctx_t ctx, int n, hgv_c128 *B, int ldb, void *work, size_t work_bytes, int *d_info) {
    if (!ctx_ok(ctx)) return HGV_E_CTX;
    if (n < 0) return -2;
    if (n > 0 && !B) return -3;
    if (ldb < std::max(1, n)) return -4;
    int st = check_work(ctx, HGV_ST_POTRF, n, 0, 0, work, work_bytes, 5);
    if (st) return st;
    return guarded(ctx, [&]() {
        set_info(ctx, d_info, 0);
        Arena ar(work, work_bytes);
        potrf_run(ctx, n, reinterpret_cast<double2 *>(B), ldb, ar, d_info, 0);
        return HGV_OK;
    });
}

int hgv_zhegst(hgv_ctx_t ctx, int n, hgv_c128 *A, int lda, const hgv_c128 *L, int ldl, void *work,
               size_t work_bytes) {
    if (!ctx_ok(ctx)) return HGV_E_CTX;
    if (n < 0) return -2;
    if (n > 0 && !A) return -3;
    if (lda < std::max(1, n)) return -4;
    if (n > 0 && !L) return -5;
    if (ldl < std::max(1, n)) return -6;
    int st = check_work(ctx, HGV_ST_HEGST, n, 0, 0, work, work_bytes, 7);
    if (st) return st;
    return guarded(ctx, [&]() {
        Arena ar(work, work_bytes);
        hegst_run(ctx, n, reinterpret_cast<double2 *>(A), lda, reinterpret_cast<const double2 *>(L), ldl, ar);
        return HGV_OK;
    });
}

int hgv_zhe2hb(hgv_ctx_t ctx, int n, int nb, hgv_c128 *A, int lda, hgv_c128 *T1, void *work,
               size_t work_bytes, int *d_info) {
    if (!ctx_ok(ctx)) return HGV_E_CTX;
    if (n < 0) return -2;
    if (nb < 1) return -3;
    if (n > 0 && !A) return -4;
    if (lda < std::max(1, n)) return -5;
    if (n > 0 && !T1) return -6;
    int st = check_work(ctx, HGV_ST_HE2HB, n, nb, 0, work, work_bytes, 7);
    if (st) return st;
    return guarded(ctx, [&]() {
        set_info(ctx, d_info, 0);
        Arena ar(work, work_bytes);
        he2hb_run(ctx, n, nb, reinterpret_cast<double2 *>(A), lda, reinterpret_cast<double2 *>(T1), ar, d_info);
        return HGV_OK;
    });
}

int hgv_zhetrd_bufsize(hgv_ctx_t ctx, int n, int nb, size_t *bytes) {
    if (!ctx_ok(ctx)) return HGV_E_CTX;
    if (n < 0) return -2;
    if (nb < 1 || nb > 64) return -3;
    if (!bytes) return -4;
    *bytes = 0;
    if (n == 0) return HGV_OK;
    return guarded(ctx, [&]() {
        Arena ar;
        hetrd_run(ctx, n, nb, nullptr, n, nullptr, nullptr, nullptr, ar);
        *bytes = ar.peak + 256;
        return HGV_OK;
    });
}

int hgv_zhetrd(hgv_ctx_t ctx, int n, int nb, hgv_c128 *A, int lda, double *d, double *e, hgv_c128 *T1, void *work,
               size_t work_bytes) {
    if (!ctx_ok(ctx)) return HGV_E_CTX;
    if (n < 0) return -2;
    if (nb < 1 || nb > 64) return -3;
    if (n > 0 && !A) return -4;
    if (lda < std::max(1, n)) return -5;
    if (n > 0 && !d) return -6;
    if (n > 1 && !e) return -7;
    if (n > 0 && !T1) return -8;
    if (n == 0) return HGV_OK;
    size_t need = 0;
    int st = hgv_zhetrd_bufsize(ctx, n, nb, &need);
    if (st != HGV_OK) return st;
    if (!work || (reinterpret_cast<uintptr_t>(work) & 255)) return -9;
    if (work_bytes < need) return HGV_E_WORKSPACE;
    return guarded(ctx, [&]() {
        Arena ar(work, work_bytes);
        hetrd_run(ctx, n, nb, reinterpret_cast<double2 *>(A), lda, d, e, reinterpret_cast<double2 *>(T1), ar);
        return HGV_OK;
    });
}

int hgv_zunmtr_tr(hgv_ctx_t ctx, char trans, int n, int nb, int m, const hgv_c128 *A, int lda, const hgv_c128 *T1,
                  hgv_c128 *Y, int ldy, void *work, size_t work_bytes) {
    if (!ctx_ok(ctx)) return HGV_E_CTX;
    if (trans != 'N' && trans != 'C') return -2;
    if (n < 0) return -3;
    if (nb < 1 || nb > 64) return -4;
    if (m < 0) return -5;
    if (n > 0 && !A) return -6;
    if (lda < std::max(1, n)) return -7;
    if (n > 0 && !T1) return -8;
    if (n > 0 && m > 0 && !Y) return -9;
    if (ldy < std::max(1, n)) return -10;
    int st = check_work(ctx, HGV_ST_Q1, n, nb, m, work, work_bytes, 11);
    if (st) return st;
    return guarded(ctx, [&]() {
        Arena ar(work, work_bytes);
        unmtr_q1_t<double2>(ctx, n, nb, m, reinterpret_cast<const double2 *>(A), lda,
                            reinterpret_cast<const double2 *>(T1), reinterpret_cast<double2 *>(Y), ldy, trans == 'C',
                            ar, 1);
        return HGV_OK;
    });
}

size_t hgv_v2_elems(int n, int nb) { return (n > 0 && nb > 0) ? v2_elems(n, nb) : 0; }
size_t hgv_v2_taus(int n, int nb) { return (n > 0 && nb > 0) ? v2_taus(n, nb) : 0; }

int hgv_zhb2st(hgv_ctx_t ctx, int n, int nb, const hgv_c128 *A, int lda, double *d, double *e, hgv_c128 *V2,
               hgv_c128 *tau2, void *work, size_t work_bytes, int *d_info) {
    if (!ctx_ok(ctx)) return HGV_E_CTX;
    if (n < 0) return -2;
    if (nb < 1) return -3;
    if (n > 0 && !A) return -4;
    if (lda < std::max(1, n)) return -5;
    if (n > 0 && !d) return -6;
    if (n > 1 && !e) return -7;
    if (n > 0 && !V2) return -8;
    if (n > 0 && !tau2) return -9;
    int st = check_work(ctx, HGV_ST_HB2ST, n, nb, 0, work, work_bytes, 10);
    if (st) return st;
    return guarded(ctx, [&]() {
        set_info(ctx, d_info, 0);
        Arena ar(work, work_bytes);
        hb2st_run(ctx, n, nb, reinterpret_cast<const double2 *>(A), lda, d, e, reinterpret_cast<double2 *>(V2),
                  reinterpret_cast<double2 *>(tau2), ar, d_info);
        return HGV_OK;
    });
}

int hgv_dstedc(hgv_ctx_t ctx, int n, const double *d, const double *e, int il, int iu, double *lambda, double *Z,
               int ldz, void *work, size_t work_bytes, int *d_info) {
    if (!ctx_ok(ctx)) return HGV_E_CTX;
    if (n < 0) return -2;
    if (n > 0 && !d) return -3;
    if (n > 1 && !e) return -4;
    if (n > 0 && (il < 1 || il > n)) return -5;
    if (n > 0 && (iu < il || iu > n)) return -6;
    if (n > 0 && !lambda) return -7;
    if (n > 0 && !Z) return -8;
    if (ldz < std::max(1, n)) return -9;
    const int m = n > 0 ? iu - il + 1 : 0;
    int st = check_work(ctx, HGV_ST_STEDC, n, 0, m, work, work_bytes, 10);
    if (st) return st;
    return guarded(ctx, [&]() {
        set_info(ctx, d_info, 0);
        if (n == 0) return HGV_OK;
        Arena ar(work, work_bytes);
        stedc_run(ctx, n, d, e, il, iu, lambda, Z, ldz, ar, d_info);
        return HGV_OK;
    });
}

int hgv_zunmtr_q2(hgv_ctx_t ctx, char trans, int n, int nb, int m, const hgv_c128 *V2, const hgv_c128 *tau2,
                  hgv_c128 *Y, int ldy, void *work, size_t work_bytes) {
    if (!ctx_ok(ctx)) return HGV_E_CTX;
    if (trans != 'N' && trans != 'C') return -2;
    if (n < 0) return -3;
    if (nb < 1) return -4;
    if (m < 0) return -5;
    if (n > 0 && !V2) return -6;
    if (n > 0 && !tau2) return -7;
    if (n > 0 && m > 0 && !Y) return -8;
    if (ldy < std::max(1, n)) return -9;
    int st = check_work(ctx, HGV_ST_Q2, n, nb, m, work, work_bytes, 10);
    if (st) return st;
    return guarded(ctx, [&]() {
        Arena ar(work, work_bytes);
        unmtr_q2_t<double2>(ctx, n, nb, m, reinterpret_cast<const double2 *>(V2),
                            reinterpret_cast<const double2 *>(tau2), reinterpret_cast<double2 *>(Y), ldy, trans == 'C',
                            ar);
        return HGV_OK;
    });
}
int hgv_zunmtr_q1(hgv_ctx_t ctx, char trans, int n, int nb, int m, const hgv_c128 *A, int lda, const hgv_c128 *T1,
                  hgv_c128 *Y, int ldy, void *work, size_t work_bytes) {
    if (!ctx_ok(ctx)) return HGV_E_CTX;
    if (trans != 'N' && trans != 'C') return -2;
    if (n < 0) return -3;
    if (nb < 1) return -4;
    if (m < 0) return -5;
    if (n > 0 && !A) return -6;
    if (lda < std::max(1, n)) return -7;
    if (n > 0 && !T1) return -8;
    if (n > 0 && m > 0 && !Y) return -9;
    if (ldy < std::max(1, n)) return -10;
    int st = check_work(ctx, HGV_ST_Q1, n, nb, m, work, work_bytes, 11);
    if (st) return st;
    return guarded(ctx, [&]() {
        Arena ar(work, work_bytes);
        unmtr_q1_t<double2>(ctx, n, nb, m, reinterpret_cast<const double2 *>(A), lda,
                            reinterpret_cast<const double2 *>(T1), reinterpret_cast<double2 *>(Y), ldy, trans == 'C',
                            ar);
        return HGV_OK;
    });
}

int hgv_ztrsm_lh(hgv_ctx_t ctx, int n, int m, const hgv_c128 *L, int ldl, hgv_c128 *X, int ldx, void *work,
                 size_t work_bytes) {
    if (!ctx_ok(ctx)) return HGV_E_CTX;
    if (n < 0) return -2;
    if (m < 0) return -3;
    if (n > 0 && !L) return -4;
    if (ldl < std::max(1, n)) return -5;
    if (n > 0 && m > 0 && !X) return -6;
    if (ldx < std::max(1, n)) return -7;
    int st = check_work(ctx, HGV_ST_TRSM, n, 0, m, work, work_bytes, 8);
    if (st) return st;
    return guarded(ctx, [&]() {
        Arena ar(work, work_bytes);
        trsm_lh_run(ctx, n, m, reinterpret_cast<const double2 *>(L), ldl, reinterpret_cast<double2 *>(X), ldx, ar);
        return HGV_OK;
    });
}

int hgv_device_peaks(hgv_ctx_t ctx, void *work, size_t work_bytes, double *fp64_mfma_tflops, double *copy_gbs) {
    if (!ctx_ok(ctx)) return HGV_E_CTX;
    if (!work || (reinterpret_cast<uintptr_t>(work) & 255)) return -2;
    if (!fp64_mfma_tflops) return -4;
    if (!copy_gbs) return -5;
    return guarded(ctx, [&]() {
        device_peaks(ctx, work, work_bytes, fp64_mfma_tflops, copy_gbs);
        return HGV_OK;
    });
}

int hgv_zgemm(hgv_ctx_t ctx, char opa, char opb, int m, int n, int k, hgv_c128 alpha, const hgv_c128 *A, int lda,
              const hgv_c128 *B, int ldb, hgv_c128 beta, hgv_c128 *C, int ldc) {
    if (!ctx_ok(ctx)) return HGV_E_CTX;
    auto okop = [](char o) { return o == 'N' || o == 'T' || o == 'C'; };
    if (!okop(opa)) return -2;
    if (!okop(opb)) return -3;
    if (m < 0) return -4;
    if (n < 0) return -5;
    if (k < 0) return -6;
    const int ra = (opa == 'N') ? m : k, rb = (opb == 'N') ? k : n;
    if (m > 0 && k > 0 && !A) return -8;
    if (lda < std::max(1, ra)) return -9;
    if (n > 0 && k > 0 && !B) return -10;
    if (ldb < std::max(1, rb)) return -11;
    if (m > 0 && n > 0 && !C) return -13;
    if (ldc < std::max(1, m)) return -14;
    return guarded(ctx, [&]() {
        ZGemm g;
        g.m = m; g.n = n; g.k = k;
        g.opa = opa; g.opb = opb;
        g.A = reinterpret_cast<const double2 *>(A); g.lda = lda;
        g.B = reinterpret_cast<const double2 *>(B); g.ldb = ldb;
        g.alpha = make_double2(alpha.re, alpha.im);
        g.beta = make_double2(beta.re, beta.im);
        g.C = reinterpret_cast<double2 *>(C); g.ldc = ldc;
        zgemm(ctx, g, nullptr, 0);
        return HGV_OK;
    });
}

// ---- batched solves ----------------------------------------------------------------------
static size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

static int batch_nb(const int *nb, int i, int n) {
    return (nb && nb[i] > 0) ? nb[i] : hgv_default_nb(n, HGV_FP64);
}

// One problem of an FP64 batched solve.  The solve runs in three phases over
// the whole batch: (A) per problem on the side streams: Cholesky, reduction to
// standard form, band reduction, band copy for the bulge chasing; (B) one
// grouped bulge-chasing kernel over the (problem, sweep) pairs of all problems;
// (C) per problem on the side streams: tridiagonal solve (or the eigenvalues
// alone), Q2, Q1, back-substitution.  The buffers that cross the phases are
// taken first from the problem's workspace slice; each stage's own scratch
// follows them and is released when the stage returns.
struct BatchProb {
    int n = 0, il = 1, iu = 1, nb = 32;
    bool vals = false;
    double2 *A = nullptr, *B = nullptr, *X = nullptr;
    int lda = 1, ldb = 1, ldx = 1;
    double *W = nullptr;
    int *d_info = nullptr;
    double2 *T1 = nullptr, *V2 = nullptr, *tau2 = nullptr, *T2 = nullptr;
    double *d = nullptr, *e = nullptr, *lambda = nullptr, *Z = nullptr;
    HbBatchProblem hb;
    size_t mark = 0;
};

static void batch_take(BatchProb &p, Arena &ar) {
    const int n = p.n, m = p.iu - p.il + 1;
    p.T1 = ar.take<double2>((size_t)cdiv(n, p.nb) * p.nb * p.nb);
    p.d = ar.take<double>(n);
    p.e = ar.take<double>(std::max(n - 1, 1));
    if (!p.vals) {
        p.lambda = ar.take<double>(n);
        p.V2 = ar.take<double2>(v2_elems(n, p.nb));
        p.tau2 = ar.take<double2>(v2_taus(n, p.nb));
        p.T2 = ar.take<double2>(q2_t_elems(n, p.nb));
        p.Z = ar.take<double>((size_t)n * m);
    }
    hb2st_batch_plan<double2>(n, p.nb, ar, p.hb);
    p.hb.V2 = p.V2;
    p.hb.tau2 = p.tau2;
    p.hb.d_info = p.d_info;
    p.mark = ar.mark();
}

static void batch_phase_a(hgv_ctx_s *ctx, BatchProb &p, Arena &ar) {
    const bool run = !ar.measuring();
    if (run) set_info(ctx, p.d_info, 0);
    potrf_hegst_run(ctx, p.n, p.B, p.ldb, p.A, p.lda, ar, p.d_info, p.n, nullptr, 0.0);
    ar.release(p.mark);
    he2hb_run(ctx, p.n, p.nb, p.A, p.lda, p.T1, ar, p.d_info);
    ar.release(p.mark);
    if (run) hb2st_batch_prep<double2>(ctx, p.hb, p.A, p.lda);
}

static void batch_phase_c(hgv_ctx_s *ctx, BatchProb &p, Arena &ar) {
    const bool run = !ar.measuring();
    const int n = p.n, m = p.iu - p.il + 1;
    if (run) hb2st_batch_finish<double2>(ctx, p.hb, p.d, p.e);
    if (p.vals) {
        stebz_run(ctx, n, p.d, p.e, p.il, m, nullptr, p.W, ar);
        ar.release(p.mark);
        return;
    }
    if (run) q2_build_t<double2>(ctx, n, p.nb, p.V2, p.tau2, p.T2);
    stedc_run(ctx, n, p.d, p.e, p.il, p.iu, p.lambda, p.Z, n, ar, p.d_info);
    ar.release(p.mark);
    if (run) {
        hipLaunchKernelGGL(copy_doubles_kernel, dim3(cdiv(m, 256)), dim3(256), 0, ctx->stream, m,
                           p.lambda + (p.il - 1), p.W);
        HGV_LAUNCH_CHECK();
        hipLaunchKernelGGL(real_to_complex_kernel, dim3(cdiv(n, 64), cdiv(m, 4)), dim3(256), 0, ctx->stream, n, m,
                           p.Z, n, p.X, p.ldx);
        HGV_LAUNCH_CHECK();
        q2_apply_t<double2>(ctx, n, p.nb, m, p.V2, p.T2, p.X, p.ldx, false);
    }
    unmtr_q1_run(ctx, n, p.nb, m, p.A, p.lda, p.T1, p.X, p.ldx, ar);
    ar.release(p.mark);
    trsm_lh_run(ctx, n, m, p.B, p.ldb, p.X, p.ldx, ar);
    ar.release(p.mark);
}

// Workspace of one problem of the grouped FP64 path (measured by running its
// phases in planning mode).
static size_t batch_prob_bytes(hgv_ctx_s *ctx, BatchProb p) {
    Arena ar;
    batch_take(p, ar);
    batch_phase_a(ctx, p, ar);
    batch_phase_c(ctx, p, ar);
    return align256(ar.peak);
}

static bool batch_grouped(const hgv_opts *opts) {
    return !opts || (opts->precision == HGV_FP64 && !opts->one_stage);
}
// mixed precision: the same three phases (complex64 band reduction, grouped
// complex64 bulge chasing, then the rest with the refinement)
static bool batch_grouped_mixed(const hgv_opts *opts) {
    return opts && opts->precision == HGV_MIXED && !opts->one_stage && !opts->values_only;
}

int hgv_zhegvx_batched_bufsize(hgv_ctx_t ctx, int batch, const int *n, const int *il, const int *iu, const int *nb,
                               const hgv_opts *opts, size_t *bytes) {
    if (!ctx_ok(ctx)) return HGV_E_CTX;
    if (batch < 0) return -2;
    if (batch > 0 && (!n || !il || !iu)) return -3;
    if (!bytes) return -8;
    if (opts && opts->precision != HGV_FP64 && opts->precision != HGV_MIXED) return -7;
    if (opts && opts->values_only && opts->precision == HGV_MIXED) return HGV_E_NOTSUP;
    *bytes = 0;
    size_t total = 512;   // the grouped path's give-up flag, then the problems' slices
    for (int i = 0; i < batch; ++i) {
        if (n[i] < 0) return -3;
        if (n[i] == 0) continue;
        if (il[i] < 1 || il[i] > n[i] || iu[i] < il[i] || iu[i] > n[i]) return -4;
        int b = batch_nb(nb, i, n[i]);
        if (b > 64) return -6;
        if (batch_grouped(opts)) {
            BatchProb p;
            p.n = n[i]; p.il = il[i]; p.iu = iu[i]; p.nb = b; p.vals = opts && opts->values_only;
            int st = guarded(ctx, [&]() {
                total += batch_prob_bytes(ctx, p);
                return HGV_OK;
            });
            if (st != HGV_OK) return st;
        } else {
            hgv_opts o = *opts;
            o.nb = b;
            size_t need = 0;
            int st = hgv_zhegvx_bufsize(ctx, n[i], il[i], iu[i], &o, &need);
            if (st != HGV_OK) return st;
            total += align256(need);
        }
    }
    *bytes = total;
    return HGV_OK;
}

int hgv_zhegvx_batched(hgv_ctx_t ctx, int batch, const int *n, hgv_c128 *const *A, const int *lda,
                       hgv_c128 *const *B, const int *ldb, const int *il, const int *iu, double *const *W,
                       hgv_c128 *const *X, const int *ldx, const int *nb, const hgv_opts *opts, void *work,
                       size_t work_bytes, int *d_info) {
    if (!ctx_ok(ctx)) return HGV_E_CTX;
    if (batch < 0) return -2;
    if (batch == 0) return HGV_OK;
    if (!n || !A || !lda || !B || !ldb || !il || !iu || !W || !X || !ldx) return -3;
    const bool vals = opts && opts->values_only;
    for (int i = 0; i < batch; ++i) {
        const int nn = std::max(1, n[i]);
        if (n[i] < 0) return -3;
        if (lda[i] < nn || ldb[i] < nn || (!vals && ldx[i] < nn)) return -5;
        if (n[i] > 0 && (!A[i] || !B[i] || !W[i] || (!X[i] && !vals))) return -4;
    }
    size_t need = 0;
    if (opts && opts->precision != HGV_FP64 && opts->precision != HGV_MIXED) return -14;
    int st = hgv_zhegvx_batched_bufsize(ctx, batch, n, il, iu, nb, opts, &need);
    if (st != HGV_OK) return st == -7 ? -14 : st;
    if (!work || (reinterpret_cast<uintptr_t>(work) & 255)) return -15;
    if (work_bytes < need) return HGV_E_WORKSPACE;
    return guarded(ctx, [&]() {
        const int K = 8;
        if (ctx->side.empty()) {
            for (int k = 0; k < K; ++k) {
                hipStream_t s;
                hipEvent_t e;
                HGV_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
                HGV_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
                ctx->side.push_back(s);
                ctx->side_ev.push_back(e);
            }
            HGV_HIP(hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming));
        }
        const bool grouped = batch_grouped(opts);
        char *base = static_cast<char *>(work);
        int *err = reinterpret_cast<int *>(base);
        // workspace slices in problem order; problems dealt longest first to the
        // least loaded stream (estimated cost ~ n^3)
        std::vector<size_t> off(batch, 0);
        std::vector<BatchProb> probs(batch);
        size_t at = 512;
        for (int i = 0; i < batch; ++i) {
            off[i] = at;
            if (n[i] == 0) continue;
            if (grouped) {
                BatchProb &p = probs[i];
                p.n = n[i]; p.il = il[i]; p.iu = iu[i]; p.nb = batch_nb(nb, i, n[i]); p.vals = vals;
                at += batch_prob_bytes(ctx, p);
            } else {
                hgv_opts o = *opts;
                o.nb = batch_nb(nb, i, n[i]);
                size_t b = 0;
                (void)hgv_zhegvx_bufsize(ctx, n[i], il[i], iu[i], &o, &b);
                at += align256(b);
            }
        }
        std::vector<int> order(batch);
        for (int i = 0; i < batch; ++i) order[i] = i;
        std::sort(order.begin(), order.end(), [&](int x, int y) { return n[x] > n[y]; });
        hipStream_t user = ctx->stream;
        // every problem of `order` on the least loaded side stream, then join
        auto fan_out = [&](const std::function<void(int)> &body) {
            std::vector<double> load(K, 0.0);
            HGV_HIP(hipEventRecord(ctx->fork_ev, user));
            for (int k = 0; k < K; ++k) HGV_HIP(hipStreamWaitEvent(ctx->side[k], ctx->fork_ev, 0));
            ctx->concurrent = true;
            try {
                for (int idx : order) {
                    int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
                    load[k] += (double)n[idx] * n[idx] * n[idx];
                    ctx->stream = ctx->side[k];
                    body(idx);
                }
            } catch (...) {
                ctx->stream = user;
                ctx->concurrent = false;
                ctx->panel_share = 0;
                throw;
            }
            ctx->stream = user;
            ctx->concurrent = false;
            for (int k = 0; k < K; ++k) {
                HGV_HIP(hipEventRecord(ctx->side_ev[k], ctx->side[k]));
                HGV_HIP(hipStreamWaitEvent(user, ctx->side_ev[k], 0));
            }
        };
        if (batch_grouped_mixed(opts)) {
            const int iters = opts->max_refine_iters > 0 ? opts->max_refine_iters : 3;
            const int its = opts->max_refine_iters < 0 ? 0 : iters;
            std::vector<HbBatchProblem> hbm(batch);
            // (A) FP64 factorisation and reduction to standard form, complex64 band reduction
            ctx->panel_share = K;
            fan_out([&](int idx) {
                int *inf = d_info ? d_info + idx : nullptr;
                if (n[idx] == 0) {
                    set_info(ctx, inf, 0);
                    return;
                }
                Arena ar(base + off[idx], work_bytes - off[idx]);
                const int nbi = batch_nb(nb, idx, n[idx]);
                const double tol = opts->refine_tol > 0.0 ? opts->refine_tol
                                                         : 32.0 * DBL_EPSILON * std::sqrt((double)n[idx]);
                set_info(ctx, inf, 0);
                potrf_hegst_run(ctx, n[idx], reinterpret_cast<double2 *>(B[idx]), ldb[idx],
                                reinterpret_cast<double2 *>(A[idx]), lda[idx], ar, inf, n[idx], nullptr, 0.0);
                ar.release(0);
                MixedResult mr;
                mixed_standard(ctx, n[idx], reinterpret_cast<double2 *>(A[idx]), lda[idx], il[idx], iu[idx], W[idx],
                               reinterpret_cast<double2 *>(X[idx]), ldx[idx], ar, nbi, its, tol, true, inf, nullptr,
                               &mr, 1, &hbm[idx]);
            });
            ctx->panel_share = 0;
            // (B) one grouped complex64 bulge chasing
            std::vector<HbBatchProblem> hbs;
            for (int i = 0; i < batch; ++i)
                if (n[i] > 0) hbs.push_back(hbm[i]);
            hb2st_batch_run<float2>(ctx, hbs, err);
            // (C) tridiagonal solves, complex64 back-transformations, FP64 refinement, back-substitution
            fan_out([&](int idx) {
                if (n[idx] == 0) return;
                int *inf = d_info ? d_info + idx : nullptr;
                Arena ar(base + off[idx], work_bytes - off[idx]);
                const int nbi = batch_nb(nb, idx, n[idx]);
                const double tol = opts->refine_tol > 0.0 ? opts->refine_tol
                                                         : 32.0 * DBL_EPSILON * std::sqrt((double)n[idx]);
                MixedResult mr;
                mixed_standard(ctx, n[idx], reinterpret_cast<double2 *>(A[idx]), lda[idx], il[idx], iu[idx], W[idx],
                               reinterpret_cast<double2 *>(X[idx]), ldx[idx], ar, nbi, its, tol, true, inf, nullptr,
                               &mr, 2, &hbm[idx]);
                ar.release(0);
                trsm_lh_run(ctx, n[idx], iu[idx] - il[idx] + 1, reinterpret_cast<double2 *>(B[idx]), ldb[idx],
                            reinterpret_cast<double2 *>(X[idx]), ldx[idx], ar);
            });
            return HGV_OK;
        }
        if (!grouped) {
            fan_out([&](int idx) {
                int *inf = d_info ? d_info + idx : nullptr;
                if (n[idx] == 0) {
                    set_info(ctx, inf, 0);
                    return;
                }
                Arena ar(base + off[idx], work_bytes - off[idx]);
                hgv_opts o = *opts;
                o.nb = batch_nb(nb, idx, n[idx]);
                zhegvx_full(ctx, n[idx], reinterpret_cast<double2 *>(A[idx]), lda[idx],
                            reinterpret_cast<double2 *>(B[idx]), ldb[idx], il[idx], iu[idx], W[idx],
                            reinterpret_cast<double2 *>(X[idx]), ldx[idx], ar, o.nb, &o, inf, nullptr, nullptr, true);
            });
            return HGV_OK;
        }
        std::vector<Arena> arenas;
        arenas.reserve(batch);
        for (int i = 0; i < batch; ++i) {
            arenas.emplace_back(base + off[i], work_bytes - off[i]);
            BatchProb &p = probs[i];
            p.A = reinterpret_cast<double2 *>(A[i]); p.lda = lda[i];
            p.B = reinterpret_cast<double2 *>(B[i]); p.ldb = ldb[i];
            p.X = reinterpret_cast<double2 *>(X[i]); p.ldx = ldx[i];
            p.W = W[i];
            p.d_info = d_info ? d_info + i : nullptr;
            if (n[i] > 0) batch_take(p, arenas[i]);
        }
        // (A) factorisations and band reductions (persistent panels side by side)
        ctx->panel_share = K;
        fan_out([&](int idx) {
            if (n[idx] == 0) {
                set_info(ctx, probs[idx].d_info, 0);
                return;
            }
            batch_phase_a(ctx, probs[idx], arenas[idx]);
        });
        ctx->panel_share = 0;
        // (B) one grouped bulge chasing over every problem
        std::vector<HbBatchProblem> hbs;
        for (int i = 0; i < batch; ++i)
            if (n[i] > 0) hbs.push_back(probs[i].hb);
        hb2st_batch_run<double2>(ctx, hbs, err);
        // (C) tridiagonal solves and back-transformations
        fan_out([&](int idx) {
            if (n[idx] > 0) batch_phase_c(ctx, probs[idx], arenas[idx]);
        });
        return HGV_OK;
    });
}

// ---- selection by value ------------------------------------------------------------------
static void zhegvx_range_plan(hgv_ctx_s *ctx, int n, double2 *A, int lda, double2 *B, int ldb, double vl, double vu,
                              int mmax, double *W, double2 *X, int ldx, int *d_m, Arena &ar, int nb,
                              const hgv_opts *opts, int *d_info, StageTimer *tm) {
    int *range = ar.take<int>(4);
    ValueRange vr{vl, vu, range};
    zhegvx_full(ctx, n, A, lda, B, ldb, 1, mmax, W, X, ldx, ar, nb, opts, d_info, tm, nullptr, true, &vr);
    if (!ar.measuring()) {
        hipLaunchKernelGGL(copy_int_kernel, dim3(1), dim3(1), 0, ctx->stream, range + 1, d_m);
        HGV_LAUNCH_CHECK();
    }
}

int hgv_zhegvx_range_bufsize(hgv_ctx_t ctx, int n, int mmax, const hgv_opts *opts, size_t *bytes) {
    if (!ctx_ok(ctx)) return HGV_E_CTX;
    if (n < 0) return -2;
    if (n > 0 && (mmax < 1 || mmax > n)) return -3;
    if (!bytes) return -5;
    *bytes = 0;
    if (opts && opts->precision != HGV_FP64) return opts->precision == HGV_MIXED ? HGV_E_NOTSUP : -4;
    if (n == 0) return HGV_OK;
    return guarded(ctx, [&]() {
        Arena ar;
        zhegvx_range_plan(ctx, n, nullptr, n, nullptr, n, 0.0, 1.0, mmax, nullptr, nullptr, n, nullptr, ar,
                          resolve_nb(n, opts), opts, nullptr, nullptr);
        *bytes = ar.peak + 256;
        return HGV_OK;
    });
}

int hgv_zhegvx_range(hgv_ctx_t ctx, int n, hgv_c128 *A, int lda, hgv_c128 *B, int ldb, double vl, double vu,
                     int mmax, double *W, hgv_c128 *X, int ldx, int *d_m, void *work, size_t work_bytes,
                     const hgv_opts *opts, int *d_info, hgv_stats *stats) {
    if (!ctx_ok(ctx)) return HGV_E_CTX;
    if (n < 0) return -2;
    const int nn = std::max(1, n);
    const bool vals = opts && opts->values_only;
    if (n > 0 && !A) return -3;
    if (lda < nn) return -4;
    if (n > 0 && !B) return -5;
    if (ldb < nn) return -6;
    if (!(vl == vl)) return -7;
    if (!(vu > vl)) return -8;
    if (n > 0 && (mmax < 1 || mmax > n)) return -9;
    if (n > 0 && !W) return -10;
    if (n > 0 && !X && !vals) return -11;
    if (!vals && ldx < nn) return -12;
    if (!d_m) return -13;
    if (opts && opts->precision != HGV_FP64) return opts->precision == HGV_MIXED ? HGV_E_NOTSUP : -16;
    if (opts && opts->nb < 0) return -16;
    if (n == 0) return guarded(ctx, [&]() {
        set_info(ctx, d_info, 0);
        set_info(ctx, d_m, 0);
        return HGV_OK;
    });
    size_t need = 0;
    int st = hgv_zhegvx_range_bufsize(ctx, n, mmax, opts, &need);
    if (st != HGV_OK) return st;
    if (!work || (reinterpret_cast<uintptr_t>(work) & 255)) return -14;
    if (work_bytes < need) return HGV_E_WORKSPACE;
    return guarded(ctx, [&]() {
        StageTimer tm(ctx, stats);
        Arena ar(work, work_bytes);
        const int nb = resolve_nb(n, opts);
        zhegvx_range_plan(ctx, n, reinterpret_cast<double2 *>(A), lda, reinterpret_cast<double2 *>(B), ldb, vl, vu,
                          mmax, W, reinterpret_cast<double2 *>(X), ldx, d_m, ar, nb, opts, d_info,
                          stats ? &tm : nullptr);
        if (stats) {
            tm.finish();
            stats->nb = nb;
        }
        return HGV_OK;
    });
}

// ---- tridiagonal eigenvalues by Sturm counts --------------------------------------------
int hgv_dstebz_bufsize(hgv_ctx_t ctx, int n, size_t *bytes) {
    if (!ctx_ok(ctx)) return HGV_E_CTX;
    if (n < 0) return -2;
    if (!bytes) return -3;
    Arena ar;
    stebz_run(ctx, n, nullptr, nullptr, 1, n, nullptr, nullptr, ar);
    *bytes = ar.peak + 256;
    return HGV_OK;
}

int hgv_dstebz(hgv_ctx_t ctx, int n, const double *d, const double *e, int il, int iu, double *W, void *work,
               size_t work_bytes) {
    if (!ctx_ok(ctx)) return HGV_E_CTX;
    if (n < 0) return -2;
    if (n > 0 && !d) return -3;
    if (n > 1 && !e) return -4;
    if (n > 0 && (il < 1 || il > n)) return -5;
    if (n > 0 && (iu < il || iu > n)) return -6;
    if (n > 0 && !W) return -7;
    if (n == 0) return HGV_OK;
    size_t need = 0;
    hgv_dstebz_bufsize(ctx, n, &need);
    if (!work || (reinterpret_cast<uintptr_t>(work) & 255)) return -8;
    if (work_bytes < need) return HGV_E_WORKSPACE;
    return guarded(ctx, [&]() {
        Arena ar(work, work_bytes);
        stebz_run(ctx, n, d, e, il, iu - il + 1, nullptr, W, ar);
        return HGV_OK;
    });
}

int hgv_dstebz_noalloc(hgv_ctx_t ctx, int n, const double *d, const double *e, int il, int iu, double *W) {
    if (!ctx_ok(ctx)) return HGV_E_CTX;
    if (n < 0 || n > HGV_DSTEBZ_NOALLOC_MAX) return -2;
    if (n > 0 && !d) return -3;
    if (n > 1 && !e) return -4;
    if (n > 0 && (il < 1 || il > n)) return -5;
    if (n > 0 && (iu < il || iu > n)) return -6;
    if (n > 0 && !W) return -7;
    if (n == 0) return HGV_OK;
    return guarded(ctx, [&]() {
        stebz_noalloc_run(ctx, n, d, e, il, iu - il + 1, W);
        return HGV_OK;
    });
}

int hgv_gauge_fix(hgv_ctx_t ctx, int n, int m, hgv_c128 *X, int ldx) {
    if (!ctx_ok(ctx)) return HGV_E_CTX;
    if (n < 0) return -2;
    if (m < 0) return -3;
    if (n > 0 && m > 0 && !X) return -4;
    if (ldx < std::max(1, n)) return -5;
    return guarded(ctx, [&]() {
        gauge_fix_run(ctx, n, m, reinterpret_cast<double2 *>(X), ldx);
        return HGV_OK;
    });
}

int hgv_zhegvx_backward_bufsize(hgv_ctx_t ctx, int n, int il, int iu, size_t *bytes) {
    if (!ctx_ok(ctx)) return HGV_E_CTX;
    if (n < 0) return -2;
    if (n > 0 && (il < 1 || il > n)) return -3;
    if (n > 0 && (iu < il || iu > n)) return -4;
    if (!bytes) return -5;
    *bytes = 0;
    if (n == 0) return HGV_OK;
    return guarded(ctx, [&]() {
        Arena ar;
        adjoint_run(ctx, n, il, iu, nullptr, nullptr, n, nullptr, nullptr, n, nullptr, n, nullptr, n, ar);
        *bytes = ar.peak + 256;
        return HGV_OK;
    });
}

int hgv_zhegvx_backward(hgv_ctx_t ctx, int n, int il, int iu, const double *lambda, const hgv_c128 *Xall, int ldxa,
                        const double *Wbar, const hgv_c128 *Xbar, int ldxb, hgv_c128 *Abar, int ldab, hgv_c128 *Bbar,
                        int ldbb, void *work, size_t work_bytes) {
    if (!ctx_ok(ctx)) return HGV_E_CTX;
    if (n < 0) return -2;
    const int nn = std::max(1, n);
    if (n > 0 && (il < 1 || il > n)) return -3;
    if (n > 0 && (iu < il || iu > n)) return -4;
    if (n > 0 && !lambda) return -5;
    if (n > 0 && !Xall) return -6;
    if (ldxa < nn) return -7;
    if (n > 0 && !Wbar) return -8;
    if (n > 0 && !Xbar) return -9;
    if (ldxb < nn) return -10;
    if (n > 0 && !Abar) return -11;
    if (ldab < nn) return -12;
    if (n > 0 && !Bbar) return -13;
    if (ldbb < nn) return -14;
    size_t need = 0;
    int st = hgv_zhegvx_backward_bufsize(ctx, n, il, iu, &need);
    if (st != HGV_OK) return st;
    if (n == 0) return HGV_OK;
    if (!work || (reinterpret_cast<uintptr_t>(work) & 255)) return -15;
    if (work_bytes < need) return HGV_E_WORKSPACE;
    return guarded(ctx, [&]() {
        Arena ar(work, work_bytes);
        adjoint_run(ctx, n, il, iu, lambda, reinterpret_cast<const double2 *>(Xall), ldxa, Wbar,
                    reinterpret_cast<const double2 *>(Xbar), ldxb, reinterpret_cast<double2 *>(Abar), ldab,
                    reinterpret_cast<double2 *>(Bbar), ldbb, ar);
        return HGV_OK;
    });
}

}  // extern "C"
