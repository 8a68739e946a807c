// hgv_internal.h -- shared declarations of the gfx950 solver library (not part
// of the public ABI).  Device complex numbers are double2 (x = re, y = im) or
// float2 for the complex64 path; matrices are column-major.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <functional>
#include <vector>

#include "hgv.h"

struct hgv_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    int last_hip_error = 0;
    // Optional per-call accounting of the MFMA GEMM launches (events around
    // every launch; enabled only while a call fills hgv_stats).
    bool time_gemm = false;
    std::vector<hipEvent_t> ev_free;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending;
    std::vector<double> ev_flops;
    double gemm_ms = 0.0, gemm_flops = 0.0;
    int gemm_launches = 0;
    // Streams and events of batched solves (created on first use, default
    // priority); problems of a batch run concurrently on them.
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> side_ev;
    hipEvent_t fork_ev = nullptr;
    // Set while problems run concurrently on the side streams: kernels whose
    // workgroups wait for each other (and so need to be resident together)
    // then use their launch-per-step forms where they have one.
    bool concurrent = false;
    // While problems run concurrently: the number of band-reduction panels that
    // may run side by side (one per side stream) when nothing else that waits
    // on other workgroups runs beside them (the factorisation and band-reduction
    // phase of a grouped batch); each panel's persistent grid then takes at most
    // that share of the device, so all of them fit at once.  0: panels use their
    // launch-per-step form while concurrent.
    int panel_share = 0;
    // workgroups of the 64 x 64 (128 x 128 for real) GEMM tile kernel resident on
    // the device at once, per element type (complex double, complex float, real
    // double); 0 until the first product of that type
    int gemm_slots[3] = {0, 0, 0};
    // Side streams of one solve (created on first use, default priority) and
    // their events: [0] runs the next panel of the band reduction under the
    // current update (events 0, 1), [1] the left triangular solves of the
    // reduction to standard form under its recursion (events 2, 3).
    hipStream_t la_stream[2] = {nullptr, nullptr};
    hipEvent_t la_ev[4] = {nullptr, nullptr, nullptr, nullptr};
    // Test hooks (hgv_test_hooks, HGV_TEST_* bits): HGV_TEST_WAIT_FAIL starts
    // the give-up flags of the kernels with bounded waits set, so every wait
    // returns at once and the stage reports d_info = 2n+2; HGV_TEST_NAN_RESIDUAL
    // makes the mixed-precision refinement see a NaN residual.
    int test_hooks = 0;
    int magic = 0x68677631;
};

namespace hgv {

// ---- errors -------------------------------------------------------------
struct HipFail {
    hipError_t err;
};

#define HGV_HIP(call)                                             \
    do {                                                          \
        hipError_t e_ = (call);                                   \
        if (e_ != hipSuccess) throw ::hgv::HipFail{e_};           \
    } while (0)

#define HGV_LAUNCH_CHECK() HGV_HIP(hipGetLastError())

struct WorkspaceShort {
    size_t need;
};

// ---- scratch arena ---------------------------------------------------------
// Carves 256-byte aligned pieces out of the caller's workspace.  With a null
// base it only measures (the *_bufsize queries run the same planning code).
// Stages run one after another on one stream, so a stage's private scratch
// is released (reset to a mark) when it returns; `peak` is the size needed.
struct Arena {
    char *base = nullptr;
    size_t cap = 0;
    size_t off = 0;
    size_t peak = 0;
    Arena() = default;
    Arena(void *b, size_t c) : base(static_cast<char *>(b)), cap(c) {}
    template <class T>
    T *take(size_t count) {
        size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
        size_t at = off;
        off += bytes;
        if (off > peak) peak = off;
        if (!base) return nullptr;
        if (off > cap) throw WorkspaceShort{off};
        return reinterpret_cast<T *>(base + at);
    }
    bool measuring() const { return base == nullptr; }
    size_t mark() const { return off; }
    void release(size_t m) { off = m; }
};

// ---- device complex helpers ---------------------------------------------------
__host__ __device__ inline double2 zmk(double r, double i) { return make_double2(r, i); }
// c ? a : b per component (a ternary on the vector type itself may be compiled
// as a select between two addresses and a load through scratch memory)
__host__ __device__ inline double2 zsel(bool c, double2 a, double2 b) {
    return make_double2(c ? a.x : b.x, c ? a.y : b.y);
}
__host__ __device__ inline double2 zadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline double2 zsub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline double2 zmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__host__ __device__ inline double2 zcmul(double2 a, double2 b) {
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__host__ __device__ inline double2 zconj(double2 a) { return make_double2(a.x, -a.y); }
__host__ __device__ inline double2 zscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
__host__ __device__ inline double zabs2(double2 a) { return a.x * a.x + a.y * a.y; }
// a += b * c
__host__ __device__ inline void zfma(double2 &a, double2 b, double2 c) {
    a.x = fma(b.x, c.x, fma(-b.y, c.y, a.x));
    a.y = fma(b.x, c.y, fma(b.y, c.x, a.y));
}
// a += conj(b) * c
__host__ __device__ inline void zcfma(double2 &a, double2 b, double2 c) {
    a.x = fma(b.x, c.x, fma(b.y, c.y, a.x));
    a.y = fma(b.x, c.y, fma(-b.y, c.x, a.y));
}
__host__ __device__ inline double2 zdiv(double2 a, double2 b) {
    double s = 1.0 / (b.x * b.x + b.y * b.y);
    return make_double2((a.x * b.x + a.y * b.y) * s, (a.y * b.x - a.x * b.y) * s);
}

// A double moved between the lanes of a wave by a DPP control (as its two 32-bit
// halves): the cross-lane step of the reductions that avoid LDS round trips.
template <int CTRL>
__device__ inline double dpp_f64(double x) {
    const long long v = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(v & 0xffffffffll), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// The value of a double in lane l of the wave (l wave-uniform), as its two
// 32-bit halves.
__device__ inline double lane_f64(double x, int l) {
    const long long v = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(v & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane((int)(v >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

inline int cdiv(int a, int b) { return (a + b - 1) / b; }
inline size_t cdivz(size_t a, size_t b) { return (a + b - 1) / b; }

// ---- GEMM (gemm.hip) -------------------------------------------------------
// C <- alpha * (opA(A) opB(B) [+ opA2(A2) opB2(B2)]) + beta * C, complex double.
// op: 'N', 'T', 'C'; for A also 'H': A is Hermitian (m == k) with only its
// lower triangle stored (diagonal taken real).  lower != 0 restricts the
// output to the elements i >= j (tiles entirely above the diagonal are
// skipped, elements above it are not written).
struct ZGemm {
    int m = 0, n = 0, k = 0;
    char opa = 'N', opb = 'N';
    const double2 *A = nullptr; int lda = 1;
    const double2 *B = nullptr; int ldb = 1;
    char opa2 = 'N', opb2 = 'N';
    const double2 *A2 = nullptr; int lda2 = 1;
    const double2 *B2 = nullptr; int ldb2 = 1;
    double2 alpha = {1.0, 0.0}, beta = {0.0, 0.0};
    double2 *C = nullptr; int ldc = 1;
    int lower = 0;
    int allow_split = 1;   // 0: C may alias A or B: K is never split and one tile spans
                           // the aliased operand's other dimension
    const int *gate = nullptr;   // non-null: the product runs only if *gate == gate_val
    int gate_val = 0;            // (a device flag set by an earlier kernel on the stream)
};
// Workspace for split-K partial sums reserved by every stage that calls zgemm.
size_t zgemm_splitk_bytes(int n);
void zgemm(hgv_ctx_s *ctx, const ZGemm &g, double2 *splitk_ws, size_t splitk_bytes);

// Real double GEMM (divide-and-conquer merges): C <- A B (+ beta C), 'N' ops only.
void dgemm_nn(hgv_ctx_s *ctx, int m, int n, int k, double alpha, const double *A, int lda,
              const double *B, int ldb, double beta, double *C, int ldc);

// Complex float GEMM for the mixed-precision path (same conventions as ZGemm).
struct CGemm {
    int m = 0, n = 0, k = 0;
    char opa = 'N', opb = 'N';
    const float2 *A = nullptr; int lda = 1;
    const float2 *B = nullptr; int ldb = 1;
    char opa2 = 'N', opb2 = 'N';
    const float2 *A2 = nullptr; int lda2 = 1;
    const float2 *B2 = nullptr; int ldb2 = 1;
    float2 alpha = {1.0f, 0.0f}, beta = {0.0f, 0.0f};
    float2 *C = nullptr; int ldc = 1;
    int lower = 0;
    int allow_split = 1;
    const int *gate = nullptr;
    int gate_val = 0;
};
void cgemm(hgv_ctx_s *ctx, const CGemm &g, float2 *splitk_ws, size_t splitk_bytes);

// Storage-type traits: every stage that also runs in complex64 (the mixed-
// precision path) is a template on the storage type E; arithmetic that the
// method keeps in FP64 (norms, reflector scalars, T factors) converts through
// these.
template <class E>
struct El;
template <>
struct El<double2> {
    typedef ZGemm Gemm;
    __host__ __device__ static double2 to(double2 a) { return a; }
    __host__ __device__ static double2 from(double2 a) { return a; }
    __host__ __device__ static double2 mk(double r, double i) { return make_double2(r, i); }
};
template <>
struct El<float2> {
    typedef CGemm Gemm;
    __host__ __device__ static double2 to(float2 a) { return make_double2(a.x, a.y); }
    __host__ __device__ static float2 from(double2 a) { return make_float2((float)a.x, (float)a.y); }
    __host__ __device__ static float2 mk(double r, double i) { return make_float2((float)r, (float)i); }
};
inline void gemm_any(hgv_ctx_s *ctx, const ZGemm &g, void *ws, size_t wsb) {
    zgemm(ctx, g, static_cast<double2 *>(ws), wsb);
}
inline void gemm_any(hgv_ctx_s *ctx, const CGemm &g, void *ws, size_t wsb) {
    cgemm(ctx, g, static_cast<float2 *>(ws), wsb);
}

// ---- small helpers (misc.hip) ---------------------------------------------------
void fill_upper_from_lower(hgv_ctx_s *ctx, int n, double2 *A, int lda);
void zero_strict_upper(hgv_ctx_s *ctx, int n, double2 *A, int lda);
void copy_matrix(hgv_ctx_s *ctx, int m, int n, const double2 *A, int lda, double2 *B, int ldb);
// Y += alpha X (m x n, alpha real)
void add_scaled(hgv_ctx_s *ctx, int m, int n, double alpha, const double2 *X, int ldx, double2 *Y, int ldy);
void set_info(hgv_ctx_s *ctx, int *d_info, int value);
// measured FP64 MFMA rate (TFLOP/s) and copy bandwidth (GB/s, read + write)
// of the context's device; work: device buffer, the copy uses most of it
void device_peaks(hgv_ctx_s *ctx, void *work, size_t work_bytes, double *tflops, double *gbs);
// creates ctx->la_stream and ctx->la_ev on first use
void ensure_lookahead_stream(hgv_ctx_s *ctx);
// *d_info = code if *err != 0 and *d_info == 0 (device words; d_info may be null)
void report_wait_fail(hgv_ctx_s *ctx, const int *err, int *d_info, int code);

// ---- stages ----------------------------------------------------------------------
// Every stage has a plan (arena-driven size) and a run with the same arena.
void potrf_run(hgv_ctx_s *ctx, int n, double2 *B, int ldb, Arena &ar, int *d_info, int info_offset);
void hegst_run(hgv_ctx_s *ctx, int n, double2 *A, int lda, const double2 *L, int ldl, Arena &ar);
struct StageTimer;
void potrf_hegst_run(hgv_ctx_s *ctx, int n, double2 *B, int ldb, double2 *A, int lda, Arena &ar, int *d_info,
                     int info_offset, StageTimer *tm, double potrf_flops);
void trsm_lh_run(hgv_ctx_s *ctx, int n, int m, const double2 *L, int ldl, double2 *X, int ldx, Arena &ar);
// The same stages in the storage type E (double2 or float2; the 64 x 64 leaves
// compute in FP64 whatever E is, the GEMMs run in E's precision).
template <class E>
void trsm_lh_t(hgv_ctx_s *ctx, int n, int m, const E *L, int ldl, E *X, int ldx, Arena &ar);
template <class E>
void potrf_hegst_t(hgv_ctx_s *ctx, int n, E *B, int ldb, E *A, int lda, Arena &ar, int *d_info, int info_offset,
                   StageTimer *tm, double potrf_flops);
// Triangular solves used by the recursive stages (L lower n x n):
//   right_lc:  X <- X L^-H      (X m x n)
//   left_ln:   X <- L^-1 X      (X n x m)
//   left_lc:   X <- L^-H X      (X n x m)
void trsm_right_lc(hgv_ctx_s *ctx, int m, int n, const double2 *L, int ldl, double2 *X, int ldx, Arena &ar);
void trsm_left_ln(hgv_ctx_s *ctx, int n, int m, const double2 *L, int ldl, double2 *X, int ldx, Arena &ar);
void trsm_left_lc(hgv_ctx_s *ctx, int n, int m, const double2 *L, int ldl, double2 *X, int ldx, Arena &ar);

// d_info (device, may be null) receives 2n+2 if a bounded wait of a
// persistent kernel gave up (the result is then not valid)
template <class E>
void he2hb_t(hgv_ctx_s *ctx, int n, int nb, E *A, int lda, E *T1, Arena &ar, int *d_info = nullptr);
// Y <- Q1 Y (adj = false) or Y <- Q1^H Y (adj = true)
// voff: first reflector row of panel p is p*nb + voff (0: nb, the band reduction;
// 1: the one-stage tridiagonalisation)
template <class E>
void unmtr_q1_t(hgv_ctx_s *ctx, int n, int nb, int m, const E *A, int lda, const E *T1, E *Y, int ldy, bool adj,
                Arena &ar, int voff = 0);
// T factor of a panel of r reflectors held in P (N x r, unit diagonal implicit)
void panel_t_build(hgv_ctx_s *ctx, int N, int r, const double2 *P, int ldp, const double2 *tau, double2 *Vw,
                   double2 *Gm, double2 *T, int ldt, void *ws, size_t wsb);
// One-stage tridiagonalisation (hetrd.hip): A = Q T Q^H with T real (d, e),
// the reflectors of panel p (columns p*nb ..) below the first subdiagonal of A
// and their compact-WY factors in T1 (as the band reduction's, voff = 1).
void hetrd_run(hgv_ctx_s *ctx, int n, int nb, double2 *A, int lda, double *d, double *e, double2 *T1, Arena &ar);
template <class E>
void hb2st_t(hgv_ctx_s *ctx, int n, int nb, const E *A, int lda, double *d, double *e, E *V2, E *tau2, Arena &ar,
             int *d_info = nullptr);
// Grouped bulge chasing of the problems of a batched solve: plan takes each
// problem's band storage and progress counters from its arena; prep (on the
// problem's stream) copies its band and clears its counters and reflectors;
// run launches one persistent kernel over the (problem, sweep) pairs of up to
// 32 problems at a time (on ctx->stream, after every prep has been joined) and
// reports a given-up wait through each d_info; finish writes (d, e).
struct HbBatchProblem {
    int n = 0, nb = 0;
    void *AB = nullptr, *V2 = nullptr, *tau2 = nullptr;
    int *prog = nullptr;
    int *d_info = nullptr;
};
template <class E>
void hb2st_batch_plan(int n, int nb, Arena &ar, HbBatchProblem &pb);
template <class E>
void hb2st_batch_prep(hgv_ctx_s *ctx, const HbBatchProblem &pb, const E *A, int lda);
template <class E>
void hb2st_batch_run(hgv_ctx_s *ctx, const std::vector<HbBatchProblem> &pbs, int *err);
template <class E>
void hb2st_batch_finish(hgv_ctx_s *ctx, const HbBatchProblem &pb, double *d, double *e);
template <class E>
void unmtr_q2_t(hgv_ctx_s *ctx, int n, int nb, int m, const E *V2, const E *tau2, E *Y, int ldy, bool adj,
                Arena &ar);
// the two halves of unmtr_q2_t, for callers that apply the same Q2 repeatedly:
// the T factors of every reflector group (q2_t_elems(n, nb) elements), then
// their application
size_t q2_t_elems(int n, int nb);
template <class E>
void q2_build_t(hgv_ctx_s *ctx, int n, int nb, const E *V2, const E *tau2, E *T2);
template <class E>
void q2_apply_t(hgv_ctx_s *ctx, int n, int nb, int m, const E *V2, const E *T2, E *Y, int ldy, bool adj);
inline void he2hb_run(hgv_ctx_s *ctx, int n, int nb, double2 *A, int lda, double2 *T1, Arena &ar,
                      int *d_info = nullptr) {
    he2hb_t<double2>(ctx, n, nb, A, lda, T1, ar, d_info);
}
inline void hb2st_run(hgv_ctx_s *ctx, int n, int nb, const double2 *A, int lda, double *d, double *e,
                      double2 *V2, double2 *tau2, Arena &ar, int *d_info = nullptr) {
    hb2st_t<double2>(ctx, n, nb, A, lda, d, e, V2, tau2, ar, d_info);
}
size_t v2_elems(int n, int nb);
size_t v2_taus(int n, int nb);
// at_last_level (may be empty) is called once, on the host, when the work of
// the last merge level is about to be enqueued (not at all without merges).
// d_range (device int[3], may be null): the wanted columns are chosen on the
// device, range[0] = first index (1-based), range[2] = count; the m = iu-il+1
// columns of Z are slots, those beyond range[2] are zeroed.
void stedc_run(hgv_ctx_s *ctx, int n, const double *d, const double *e, int il, int iu,
               double *lambda, double *Z, int ldz, Arena &ar, int *d_info,
               const std::function<void()> &at_last_level = {}, const int *d_range = nullptr);

// ---- eigenvalues by Sturm counts (stebz.hip) ------------------------------------------
// W[s] = eigenvalue il + s (1-based, ascending) of T = (d, e) for s < nslot; with
// d_range (device int[3]) the first index is range[0] and slots s >= range[2]
// are zeroed.
void stebz_run(hgv_ctx_s *ctx, int n, const double *d, const double *e, int il, int nslot, const int *d_range,
               double *W, Arena &ar);
// The same with its scratch in a file-scope device array (no workspace):
// n <= STEBZ_NOALLOC_MAX; stebz_scratch_init looks the array's address up once
// per device (the device must be current).
constexpr int STEBZ_NOALLOC_MAX = HGV_DSTEBZ_NOALLOC_MAX;
void stebz_scratch_init(int device);
void stebz_noalloc_run(hgv_ctx_s *ctx, int n, const double *d, const double *e, int il, int nslot, double *W);
// range[0] = 1 + #{eigenvalues <= vl}, range[1] = m = #{eigenvalues in (vl, vu]},
// range[2] = min(m, mmax), from Sturm counts of T = (d, e) (device int[3]).
void sturm_range_run(hgv_ctx_s *ctx, int n, const double *d, const double *e, double vl, double vu, int mmax,
                     int *d_range, Arena &ar);
// A selection of eigenpairs by value: (vl, vu], at most mmax of them returned.
struct ValueRange {
    double vl, vu;
    int *range;   // device int[3] (see sturm_range_run)
};
inline void unmtr_q2_run(hgv_ctx_s *ctx, int n, int nb, int m, const double2 *V2, const double2 *tau2,
                         double2 *Y, int ldy, Arena &ar) {
    unmtr_q2_t<double2>(ctx, n, nb, m, V2, tau2, Y, ldy, false, ar);
}
inline void unmtr_q1_run(hgv_ctx_s *ctx, int n, int nb, int m, const double2 *A, int lda,
                         const double2 *T1, double2 *Y, int ldy, Arena &ar) {
    unmtr_q1_t<double2>(ctx, n, nb, m, A, lda, T1, Y, ldy, false, ar);
}

// ---- full-solve drivers (api.hip, refine.hip) -------------------------------------
// Event pairs around stages when statistics are requested.
struct StageTimer {
    hgv_ctx_s *ctx;
    hgv_stats *st;
    hipEvent_t ev[HGV_NSTAGES + 1][2] = {};
    bool used[HGV_NSTAGES] = {};
    StageTimer(hgv_ctx_s *c, hgv_stats *s) : ctx(c), st(s) {
        if (!st) return;
        std::memset(st, 0, sizeof(*st));
        for (int i = 0; i < HGV_NSTAGES; ++i) {
            HGV_HIP(hipEventCreate(&ev[i][0]));
            HGV_HIP(hipEventCreate(&ev[i][1]));
        }
        ctx->time_gemm = true;
        ctx->gemm_ms = 0.0;
        ctx->gemm_flops = 0.0;
        ctx->gemm_launches = 0;
    }
    void begin(int s) {
        if (st) HGV_HIP(hipEventRecord(ev[s][0], ctx->stream));
    }
    void end(int s, double flops) {
        if (!st) return;
        HGV_HIP(hipEventRecord(ev[s][1], ctx->stream));
        used[s] = true;
        st->flops[s] += flops;
    }
    void finish() {
        if (!st) return;
        HGV_HIP(hipStreamSynchronize(ctx->stream));
        for (int i = 0; i < HGV_NSTAGES; ++i) {
            if (used[i]) HGV_HIP(hipEventElapsedTime(&st->ms[i], ev[i][0], ev[i][1]));
        }
        double ms = 0.0, fl = 0.0;
        for (size_t i = 0; i < ctx->ev_pending.size(); ++i) {
            float t = 0.f;
            HGV_HIP(hipEventElapsedTime(&t, ctx->ev_pending[i].first, ctx->ev_pending[i].second));
            ms += t;
            fl += ctx->ev_flops[i];
            ctx->ev_free.push_back(ctx->ev_pending[i].first);
            ctx->ev_free.push_back(ctx->ev_pending[i].second);
        }
        st->gemm_ms = ms;
        st->gemm_flops = fl;
        st->gemm_launches = (int)ctx->ev_pending.size();
        ctx->ev_pending.clear();
        ctx->ev_flops.clear();
        ctx->time_gemm = false;
    }
    ~StageTimer() {
        if (!st) return;
        ctx->time_gemm = false;
        for (int i = 0; i < HGV_NSTAGES; ++i) {
            (void)hipEventDestroy(ev[i][0]);
            (void)hipEventDestroy(ev[i][1]);
        }
    }
};

// Standard eigensolve of the lower triangle of A (n x n, destroyed) in FP64:
// he2hb, hb2st, stedc for pairs il..iu, then Y = Q1 Q2 Z into Y (n x m).  The
// eigenvalues il..iu go to W (device).  Used by the generalized solve, by the
// Rayleigh-Ritz step of the refinement and as its fallback.  With vr the
// pairs are those in (vr->vl, vr->vu], chosen on the device (il..iu then only
// give the number m of slots); with values_only Y is not referenced: no
// second-stage reflectors are kept, the eigenvalues come from Sturm-count
// multisection and nothing is back-transformed.
void standard_fp64(hgv_ctx_s *ctx, int n, double2 *A, int lda, int il, int iu, double *W, double2 *Y, int ldy,
                   Arena &ar, int nb, int *d_info, StageTimer *tm, const ValueRange *vr = nullptr,
                   bool values_only = false, bool one_stage = false);
// Mixed precision standard eigensolve of A' (n x n, FP64, lower triangle;
// kept intact unless the refinement falls back to standard_fp64): complex64
// band reduction, bulge chasing and back-transforms, FP64 tridiagonal solve,
// then FP64 refinement of the eigenpairs il..iu to the residual tolerance.
struct MixedResult {
    int iters = 0;       // corrections applied
    int fallback = 0;    // 1: the FP64 path produced the result
    double rho = 0.0;    // final max_i ||A' y_i - theta_i y_i||_2 / ||A'||_2 (host-checked runs)
};
// phase: 0 the whole solve; for batched solves 1 = up to the band copy of the
// bulge chasing (hb receives its buffers), 2 = the rest after the grouped bulge
// chasing (called with an arena in the same state as for phase 1).
struct HbBatchProblem;
void mixed_standard(hgv_ctx_s *ctx, int n, double2 *A, int lda, int il, int iu, double *W, double2 *Y, int ldy,
                    Arena &ar, int nb, int max_iters, double tol, bool fixed_iters, int *d_info, StageTimer *tm,
                    MixedResult *res, int phase = 0, HbBatchProblem *hb = nullptr);

// ---- other storage types (variants.hip) ---------------------------------------------
// Complex64 generalized solve (every stage on complex64 storage, FP32 MFMA
// GEMMs, FP64 leaves / reflector scalars / tridiagonal solve); W in FP32;
// values_only: W only (X not referenced).
void chegvx_full(hgv_ctx_s *ctx, int n, float2 *A, int lda, float2 *B, int ldb, int il, int iu, float *W, float2 *X,
                 int ldx, Arena &ar, int nb, bool values_only, int *d_info, StageTimer *tm);
// C = R (+ 0 i), n x m; R = Re C (lower triangle only when lower)
void real_to_complex(hgv_ctx_s *ctx, int n, int m, const double *R, int lr, double2 *C, int lc);
void complex_real_part(hgv_ctx_s *ctx, int n, int m, const double2 *C, int lc, double *R, int lr, bool lower);

// ---- adjoint (adjoint.hip) --------------------------------------------------------
void gauge_fix_run(hgv_ctx_s *ctx, int n, int m, double2 *X, int ldx);
void adjoint_run(hgv_ctx_s *ctx, int n, int il, int iu, const double *lam, const double2 *Xall, int ldxa,
                 const double *wbar, const double2 *Xbar, int ldxb, double2 *Abar, int ldab, double2 *Bbar, int ldbb,
                 Arena &ar);

}  // namespace hgv
