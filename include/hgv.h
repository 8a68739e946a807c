/*
 * hgv.h -- C ABI of the MI355X (gfx950) Hermitian-definite generalized
 * eigensolver:  A x = lambda B x,  A Hermitian, B Hermitian positive definite.
 *
 * The solve follows Algorithm 1 of the paper (Cholesky of B, reduction to the
 * standard form A' = L^-1 A L^-H, standard eigensolve, back-substitution
 * x = L^-H y) with the two-stage standard eigensolver of Algorithm 2 /
 * Sec. 4.2 (dense -> band by block Householder panels, band -> tridiagonal
 * by column-wise bulge chasing), the divide-and-conquer tridiagonal solver of
 * Sec. 4.3 (only the wanted eigenvectors at the last merge), and the two-step
 * eigenvector back-transformation of Sec. 4.2 (through Q2, then Q1).
 *
 * Conventions shared by every call
 *  - Matrices are column-major: element (i, j) of a matrix with leading
 *    dimension ld is at index i + j*ld.  Complex numbers are interleaved
 *    (re, im) pairs (hgv_c128 / hgv_c64).
 *  - Every matrix/vector pointer is a DEVICE pointer owned by the caller.  The
 *    library never allocates or frees caller memory and allocates no device
 *    memory of its own: scratch space is the caller's `work` buffer, whose
 *    size comes from the matching *_bufsize query.  `work` must be 256-byte
 *    aligned.
 *  - All calls are asynchronous on the stream set with hgv_set_stream (the
 *    null stream by default) and return once the work is enqueued.  Only the
 *    optional hgv_stats output synchronizes the stream.
 *  - Return value = host status: HGV_OK, a negative value -i when argument i
 *    (1-based, counting the context as argument 1) is invalid (checked on the
 *    host before anything is launched), or one of the HGV_E_* codes.
 *    Numerical failures are written to the device integer *d_info with the
 *    LAPACK xHEGV meaning (0 ok; k in [1,n]: the tridiagonal solver failed on
 *    eigenvalue k; n+k: the leading minor of order k of B is not positive
 *    definite).  d_info = 2n+2 reports that a bounded wait inside a
 *    persistent kernel gave up (the device was held by other work for
 *    seconds); the outputs are then not valid.  d_info may be NULL.
 *  - Only the lower triangles of A and B are read; their strict upper
 *    triangles may be overwritten (they are workspace).
 */
#ifndef HGV_H
#define HGV_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double re, im; } hgv_c128;
typedef struct { float re, im; } hgv_c64;

typedef struct hgv_ctx_s *hgv_ctx_t;

enum {
    HGV_OK = 0,
    HGV_E_HIP = 1001,        /* a HIP runtime call failed (see hgv_last_hip_error) */
    HGV_E_WORKSPACE = 1002,  /* work_bytes smaller than the *_bufsize query */
    HGV_E_CTX = 1003,        /* null or destroyed context */
    HGV_E_NOTSUP = 1004      /* option combination not supported */
};

enum { HGV_FP64 = 0, HGV_MIXED = 1 };

/* Solver options.  A NULL opts pointer means all defaults. */
typedef struct {
    int precision;         /* HGV_FP64 (default) or HGV_MIXED: complex64 band
                              reduction / back-transforms + fp64 refinement */
    int nb;                /* band width = panel width; 0 picks the tuned default */
    int max_refine_iters;  /* HGV_MIXED only: corrections before the FP64
                              fallback; 0 -> 3; < 0 -> none (forces the
                              fallback unless the first check passes) */
    double refine_tol;     /* HGV_MIXED only: target of max_i ||A'y_i -
                              theta_i y_i||_2 / ||A'||_2 (A' = L^-1 A L^-H);
                              0 -> 32 eps sqrt(n) */
    int values_only;       /* 1: eigenvalues only (Sec. 1: a fraction of the
                              spectrum; Sec. 4.3 builds only the needed vectors,
                              here none): X is not referenced and may be NULL,
                              the second-stage reflectors are not stored, the
                              tridiagonal eigenvalues come from Sturm-count
                              multisection (see hgv_dstebz) and neither back-
                              transformation nor the back-substitution runs.
                              HGV_FP64 only (HGV_MIXED -> HGV_E_NOTSUP). */
    int one_stage;         /* 1: one-stage tridiagonalisation (Sec. 4.1; hgv_zhetrd,
                              hemv-based, bound by memory bandwidth) and one
                              back-transformation (hgv_zunmtr_tr) in place of
                              the two-stage reduction (Sec. 4.2); nb <= 64 is its
                              panel width.  HGV_FP64 only. */
} hgv_opts;

/* Stage indices of hgv_stats.ms / flops. */
enum {
    HGV_ST_POTRF = 0, HGV_ST_HEGST, HGV_ST_HE2HB, HGV_ST_HB2ST, HGV_ST_STEDC,
    HGV_ST_Q2, HGV_ST_Q1, HGV_ST_TRSM, HGV_ST_REFINE, HGV_NSTAGES
};

/* Optional per-call statistics.  Filling it records HIP events on the stream
 * and synchronizes it at the end of the call. */
typedef struct {
    float ms[HGV_NSTAGES];       /* elapsed time per stage (HIP events)           */
    double flops[HGV_NSTAGES];   /* algorithmic flops per stage (LAPACK counts)   */
    double gemm_ms;              /* summed duration of the complex-double MFMA
                                    GEMM tile kernel launches (HIP events around
                                    each launch, split-K reductions excluded)    */
    double gemm_flops;           /* algorithmic flops of those launches           */
    int gemm_launches;
    int refine_iters;            /* HGV_MIXED: refinement corrections applied     */
    int nb;                      /* band width used                               */
    double refine_resid;         /* HGV_MIXED: final residual measure (refine_tol) */
    int fallback;                /* HGV_MIXED: 1 if the FP64 path gave the result */
} hgv_stats;

/* ---- context ------------------------------------------------------------ */
/* Binds a context to HIP device `device` (made current by every call). */
int hgv_create(hgv_ctx_t *ctx, int device);
int hgv_destroy(hgv_ctx_t ctx);
/* `stream` is a hipStream_t (e.g. torch.cuda.current_stream().cuda_stream). */
int hgv_set_stream(hgv_ctx_t ctx, void *stream);
const char *hgv_status_string(int status);
/* Last HIP error code seen by the context (0 if none). */
int hgv_last_hip_error(hgv_ctx_t ctx);
/* Band width the solver uses for order n and precision when opts->nb == 0. */
int hgv_default_nb(int n, int precision);

/* Test hooks (for the library's own failure-path tests; 0 = off, the default).
 * HGV_TEST_WAIT_FAIL: the give-up flags of the kernels with bounded waits
 *   (band reduction panel, bulge chasing) start set, so every wait returns at
 *   once, every kernel still runs to its end, and the stage reports
 *   d_info = 2n+2 (its outputs are then not valid).
 * HGV_TEST_NAN_RESIDUAL: the mixed-precision refinement sees a NaN residual,
 *   so it never meets its tolerance (FP64 fallback, or d_info = 2n+1 under
 *   graph capture).
 * HGV_TEST_HB2ST_SWEEPS: the bulge chasing of single solves runs the
 *   sweep-per-workgroup schedule (otherwise used only when the windows of the
 *   window-owner pipeline do not all fit on the device at once), so that both
 *   schedules can be tested.
 * HGV_TEST_HOUSEHOLDER_PANELS: every band-reduction panel is factored by the
 *   Householder column steps (otherwise a complex double panel of full column
 *   rank and condition number at most 1e5 is factored by Cholesky QR twice
 *   with Householder reconstruction), so that both forms can be tested.
 * Returns -2 for unknown bits. */
enum { HGV_TEST_WAIT_FAIL = 1, HGV_TEST_NAN_RESIDUAL = 2, HGV_TEST_HB2ST_SWEEPS = 4, HGV_TEST_HOUSEHOLDER_PANELS = 8 };
int hgv_test_hooks(hgv_ctx_t ctx, int mask);

/* ---- full generalized solve (Algorithm 1) -------------------------------- */
/* Workspace bytes needed by hgv_zhegvx for these arguments. */
int hgv_zhegvx_bufsize(hgv_ctx_t ctx, int n, int il, int iu, const hgv_opts *opts,
                       size_t *bytes);

/* Eigenpairs il..iu (1-based, inclusive; 1 <= il <= iu <= n; ascending
 * eigenvalues) of the pencil (A, B), n >= 0.
 *   A [in, destroyed]  n x n, lda >= max(1,n); lower triangle read.
 *   B [in/out]         n x n, ldb >= max(1,n); lower triangle read; on exit
 *                      its lower triangle holds the Cholesky factor L.
 *   W [out]            m = iu-il+1 doubles.
 *   X [out]            n x m, ldx >= max(1,n); X^H B X = I.
 * opts->precision = HGV_MIXED: potrf / hegst in FP64; band reduction, bulge
 * chasing and both back-transforms in complex64 (FP32 MFMA, reflector norms
 * and scalars in FP64); tridiagonal solve in FP64; then FP64 refinement of the
 * pairs (Rayleigh-Ritz on the subspace widened by up to 32 guard pairs on each
 * side, corrections through the complex64 factorisation) until
 * max_i ||A'y_i - theta_i y_i||_2 <= refine_tol ||A'||_2.  The check reads one
 * double back to the host per iteration; if max_refine_iters corrections do
 * not reach the tolerance the FP64 path recomputes the result.  While the
 * stream is being captured into a graph the iteration count is fixed
 * (max_refine_iters) and d_info = 2n+1 reports a missed tolerance.
 * With opts->values_only only W is written (X may be NULL, ldx is ignored).
 * Argument numbers for -i: ctx 1, n 2, A 3, lda 4, B 5, ldb 6, il 7, iu 8,
 * W 9, X 10, ldx 11, work 12, work_bytes 13, opts 14. */
int hgv_zhegvx(hgv_ctx_t ctx, int n, hgv_c128 *A, int lda, hgv_c128 *B, int ldb,
               int il, int iu, double *W, hgv_c128 *X, int ldx,
               void *work, size_t work_bytes, const hgv_opts *opts, int *d_info,
               hgv_stats *stats);

/* ---- other storage types ------------------------------------------------------ */
/* Complex64 pencils (the paper's method for Hermitian pencils in single
 * precision): every stage of hgv_zhegvx runs on complex64 storage with FP32
 * MFMA GEMMs; the 64 x 64 factorisation leaves, the reflector norms and
 * scalars and the tridiagonal divide and conquer run in FP64.  W in FP32.
 * Accuracy is that of a complex64 solver (residual and B-orthogonality
 * errors of order n * eps_fp32 * cond(B)).  Arguments as hgv_zhegvx (same
 * numbers for -i), with complex64 A, B, X and float W; opts->precision must
 * be HGV_FP64 (the default; HGV_MIXED -> HGV_E_NOTSUP: there is no
 * refinement here); opts->values_only is supported. */
int hgv_chegvx_bufsize(hgv_ctx_t ctx, int n, int il, int iu, const hgv_opts *opts, size_t *bytes);
int hgv_chegvx(hgv_ctx_t ctx, int n, hgv_c64 *A, int lda, hgv_c64 *B, int ldb, int il, int iu, float *W,
               hgv_c64 *X, int ldx, void *work, size_t work_bytes, const hgv_opts *opts, int *d_info,
               hgv_stats *stats);

/* Real symmetric-definite pencils (A symmetric, B symmetric positive
 * definite; the real case of the paper's Hermitian problem), FP64.  The pencil
 * is solved by the complex-double path on complex copies with zero imaginary
 * parts (held in the workspace); the solver's reflectors map real vectors onto
 * real multiples of e_1, so its eigenvectors come out real and their real
 * parts are returned.  On exit the lower triangle of B holds L.  Arguments as
 * hgv_zhegvx (same numbers for -i), with real A, B, X; both precisions and
 * opts->values_only are supported. */
int hgv_dsygvx_bufsize(hgv_ctx_t ctx, int n, int il, int iu, const hgv_opts *opts, size_t *bytes);
int hgv_dsygvx(hgv_ctx_t ctx, int n, double *A, int lda, double *B, int ldb, int il, int iu, double *W,
               double *X, int ldx, void *work, size_t work_bytes, const hgv_opts *opts, int *d_info,
               hgv_stats *stats);

/* ---- selection by value (LAPACK RANGE = 'V') ------------------------------- */
/* The eigenpairs whose eigenvalues lie in the half-open interval (vl, vu]
 * (Sec. 1: only a part of the spectrum is wanted).  After the reduction to the
 * real tridiagonal T (Alg. 1 steps 1-2, Alg. 2 step 1) the index range is taken
 * on the device from two Sturm counts of T, so nothing is read back to the host
 * and the whole call can be captured in a HIP graph.  An eigenvalue within a
 * few ulps of ||T|| of vl or vu may fall on either side.
 *   mmax [in]   capacity of W (doubles) and X (columns), 1 <= mmax <= n.
 *   d_m  [out]  device int: m, the number of eigenvalues in (vl, vu].  The
 *               lowest min(m, mmax) pairs go to W[0..] and X[:, 0..]; the
 *               remaining entries of W and columns of X (up to mmax) are set
 *               to zero.  m > mmax means the output was truncated.
 * Other arguments as hgv_zhegvx (opts->values_only: X may be NULL).
 * HGV_MIXED is not supported (HGV_E_NOTSUP).  Argument numbers: ctx 1, n 2,
 * A 3, lda 4, B 5, ldb 6, vl 7, vu 8, mmax 9, W 10, X 11, ldx 12, d_m 13,
 * work 14, work_bytes 15, opts 16. */
int hgv_zhegvx_range_bufsize(hgv_ctx_t ctx, int n, int mmax, const hgv_opts *opts, size_t *bytes);
int hgv_zhegvx_range(hgv_ctx_t ctx, int n, hgv_c128 *A, int lda, hgv_c128 *B, int ldb, double vl,
                     double vu, int mmax, double *W, hgv_c128 *X, int ldx, int *d_m, void *work,
                     size_t work_bytes, const hgv_opts *opts, int *d_info, hgv_stats *stats);

/* ---- batched solves ------------------------------------------------------- */
/* Many independent pencils of uneven orders (Sec. 1: the paper's target
 * applications, electronic-structure codes, solve such problems many times).  Arrays of length `batch` live in HOST
 * memory and hold per-problem sizes and DEVICE pointers with the meaning of
 * hgv_zhegvx; nb may be NULL (default band width per order) or hold a band
 * width per problem (e.g. from the autotuner of the Python package).  The
 * problems run concurrently on streams owned by the context, forked from and
 * joined back into the context's stream, so the whole call can be captured in
 * one HIP graph.  d_info is a device array of `batch` ints.  opts (NULL: FP64)
 * applies to every problem; with HGV_MIXED each problem runs exactly
 * max_refine_iters corrections (no host-side check inside a batch) and gets
 * d_info = 2n+1 when its final residual measure exceeds refine_tol. */
int hgv_zhegvx_batched_bufsize(hgv_ctx_t ctx, int batch, const int *n, const int *il, const int *iu,
                               const int *nb, const hgv_opts *opts, size_t *bytes);
int hgv_zhegvx_batched(hgv_ctx_t ctx, int batch, const int *n, hgv_c128 *const *A, const int *lda,
                       hgv_c128 *const *B, const int *ldb, const int *il, const int *iu, double *const *W,
                       hgv_c128 *const *X, const int *ldx, const int *nb, const hgv_opts *opts, void *work,
                       size_t work_bytes, int *d_info);

/* ---- stages (each one step of Algorithm 1 / Algorithm 2) ----------------- */
/* Workspace bytes of one stage call below (stage = HGV_ST_*; m = number of
 * eigenvector columns where it matters, nb = band width where it matters). */
int hgv_stage_bufsize(hgv_ctx_t ctx, int stage, int n, int nb, int m, size_t *bytes);

/* Alg. 1 step 1: B = L L^H in place (lower), L_ii real > 0.  d_info gets k
 * (1-based) when the leading minor of order k is not positive definite;
 * the factor is then incomplete. */
int hgv_zpotrf(hgv_ctx_t ctx, int n, hgv_c128 *B, int ldb, void *work, size_t work_bytes,
               int *d_info);

/* Alg. 1 step 2: A <- L^-1 A L^-H (lower triangle of A in/out, L from
 * hgv_zpotrf).  The strict upper triangle of A is used as scratch. */
int hgv_zhegst(hgv_ctx_t ctx, int n, hgv_c128 *A, int lda, const hgv_c128 *L, int ldl,
               void *work, size_t work_bytes);

/* Alg. 2 step 1, first stage (Sec. 4.2, Fig. 1): A = Q1 Band Q1^H.
 * On exit the lower band of A (0 <= i-j <= nb) holds Band; the Householder
 * vectors of panel p (columns p*nb .. p*nb+nb-1) sit below the band (unit
 * leading element implicit), and T1 (ceil(n/nb) blocks of nb x nb, block p at
 * T1 + p*nb*nb, column-major, upper triangular) holds the compact-WY factors:
 * panel p's transform is I - V_p T_p V_p^H.  Every reflector maps its column
 * onto a real multiple of e_1, so the band's first subdiagonal inside a panel
 * is real.  d_info (device int, may be NULL) is set to 0, or to 2n+2 when a
 * bounded wait of the panel kernel gave up (the result is then not valid). */
int hgv_zhe2hb(hgv_ctx_t ctx, int n, int nb, hgv_c128 *A, int lda, hgv_c128 *T1,
               void *work, size_t work_bytes, int *d_info);

/* Alg. 2 step 1, second stage (Sec. 4.2): column-wise bulge chasing of the
 * band held in the lower band of A (as left by hgv_zhe2hb; A is not modified)
 * to the real symmetric tridiagonal (d[n], e[n-1]) with Band = Q2 T Q2^H.
 * V2 receives the reflectors (hgv_v2_elems(n, nb) complex entries) and tau2
 * their scalars (hgv_v2_taus(n, nb) entries), in the layout hgv_zunmtr_q2
 * reads.  d_info (device int, may be NULL) is set to 0, or to 2n+2 when a
 * bounded wait of the bulge-chasing kernel gave up (outputs not valid). */
int hgv_zhb2st(hgv_ctx_t ctx, int n, int nb, const hgv_c128 *A, int lda, double *d,
               double *e, hgv_c128 *V2, hgv_c128 *tau2, void *work, size_t work_bytes,
               int *d_info);
size_t hgv_v2_elems(int n, int nb);
size_t hgv_v2_taus(int n, int nb);

/* Alg. 2 step 2 (Sec. 4.3): divide and conquer on the real symmetric
 * tridiagonal (d, e) -> all n eigenvalues ascending in lambda[n], and the
 * eigenvectors il..iu in Z (n x m real, ldz >= n; only the needed columns are
 * formed in the last merge).  d_info gets k in [1, n] on failure (a leaf
 * whose Jacobi sweeps did not converge: its first row; a secular root that
 * did not converge: its index in its merge); the first failure recorded wins. */
int hgv_dstedc(hgv_ctx_t ctx, int n, const double *d, const double *e, int il, int iu,
               double *lambda, double *Z, int ldz, void *work, size_t work_bytes,
               int *d_info);

/* Eigenvalues il..iu (1-based, ascending) of the real symmetric tridiagonal
 * (d, e) into W[0 .. iu-il] by multisection on Sturm counts (the eigenvalue-
 * only form of Alg. 2 step 2): each eigenvalue is bracketed independently by
 * 16 lanes that evaluate the count of eigenvalues below 16 points of its
 * interval per round, to an interval of width about 2 eps max|lambda| + eps
 * ||T||.  work: hgv_dstebz_bufsize bytes, 256-byte aligned.  Argument
 * numbers: ctx 1, n 2, d 3, e 4, il 5, iu 6, W 7, work 8. */
int hgv_dstebz_bufsize(hgv_ctx_t ctx, int n, size_t *bytes);
int hgv_dstebz(hgv_ctx_t ctx, int n, const double *d, const double *e, int il, int iu, double *W,
               void *work, size_t work_bytes);

/* Allocation-free form of hgv_dstebz, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  The multisection's scratch (e^2 and the bounds, at most
 * HGV_DSTEBZ_NOALLOC_MAX + 64 doubles, 2 MiB) lives in a device array that the
 * library holds on every device it runs on (its address is looked up by
 * hgv_create) until the process ends; the caller passes only d, e and W.
 * n <= HGV_DSTEBZ_NOALLOC_MAX, else -2.  Calls that overlap on one device
 * (several streams or contexts at once) race on that array; calls in one
 * stream are ordered.  Results equal hgv_dstebz's.  Argument numbers: ctx 1,
 * n 2, d 3, e 4, il 5, iu 6, W 7. */
#define HGV_DSTEBZ_NOALLOC_MAX 262144
int hgv_dstebz_noalloc(hgv_ctx_t ctx, int n, const double *d, const double *e, int il, int iu, double *W);

/* One-stage tridiagonalisation (Sec. 4.1): A = Q T Q^H with T real symmetric
 * tridiagonal (d[n], e[n-1]), by Householder reflectors H = I - tau v v^H with
 * H^H x = beta e_1 (beta real), blocked by panels of nb <= 64 columns: per
 * column a Hermitian matrix-vector product with the trailing matrix (its lower
 * triangle read once), then a rank-2nb update per panel on the MFMA tiles.  On
 * exit the reflector of column c sits in A below row c+1 (unit element at row
 * c+1 implicit; A[c+1, c] holds e[c]) and T1 (ceil(n/nb) blocks of nb x nb)
 * the compact-WY factors of each panel.  work: hgv_zhetrd_bufsize bytes.
 * Argument numbers: ctx 1, n 2, nb 3, A 4, lda 5, d 6, e 7, T1 8, work 9. */
int hgv_zhetrd_bufsize(hgv_ctx_t ctx, int n, int nb, size_t *bytes);
int hgv_zhetrd(hgv_ctx_t ctx, int n, int nb, hgv_c128 *A, int lda, double *d, double *e, hgv_c128 *T1,
               void *work, size_t work_bytes);
/* Y <- Q Y (trans 'N') or Q^H Y (trans 'C') with Q from hgv_zhetrd (A, T1, nb
 * as it left them); Y n x m.  work: hgv_stage_bufsize(HGV_ST_Q1, n, nb, m).
 * Argument numbers: ctx 1, trans 2, n 3, nb 4, m 5, A 6, lda 7, T1 8, Y 9,
 * ldy 10, work 11. */
int hgv_zunmtr_tr(hgv_ctx_t ctx, char trans, int n, int nb, int m, const hgv_c128 *A, int lda,
                  const hgv_c128 *T1, hgv_c128 *Y, int ldy, void *work, size_t work_bytes);

/* Alg. 2 step 3, first part: Y <- Q2 Y (trans 'N') or Y <- Q2^H Y (trans 'C');
 * Y n x m complex, ldy >= n.  Argument numbers for -i: ctx 1, trans 2, n 3,
 * nb 4, m 5, V2 6, tau2 7, Y 8, ldy 9, work 10. */
int hgv_zunmtr_q2(hgv_ctx_t ctx, char trans, int n, int nb, int m, const hgv_c128 *V2,
                  const hgv_c128 *tau2, hgv_c128 *Y, int ldy, void *work, size_t work_bytes);

/* Alg. 2 step 3, second part: Y <- Q1 Y (trans 'N') or Y <- Q1^H Y (trans 'C'),
 * with Q1 from hgv_zhe2hb (reflectors in A below the band, factors in T1).
 * Argument numbers: ctx 1, trans 2, n 3, nb 4, m 5, A 6, lda 7, T1 8, Y 9,
 * ldy 10, work 11. */
int hgv_zunmtr_q1(hgv_ctx_t ctx, char trans, int n, int nb, int m, const hgv_c128 *A, int lda,
                  const hgv_c128 *T1, hgv_c128 *Y, int ldy, void *work, size_t work_bytes);

/* Alg. 1 step 4: X <- L^-H X (X n x m, L lower from hgv_zpotrf). */
int hgv_ztrsm_lh(hgv_ctx_t ctx, int n, int m, const hgv_c128 *L, int ldl, hgv_c128 *X,
                 int ldx, void *work, size_t work_bytes);

/* ---- differentiable solve (reverse mode) ------------------------------------------ */
/* Gauge fixing used by the differentiable solve: every column of X (n x m) is
 * multiplied by a unit complex number so that its entry of largest modulus
 * (the first one on ties) becomes real and positive. */
int hgv_gauge_fix(hgv_ctx_t ctx, int n, int m, hgv_c128 *X, int ldx);

int hgv_zhegvx_backward_bufsize(hgv_ctx_t ctx, int n, int il, int iu, size_t *bytes);

/* Reverse mode of the selected pairs il..iu for the loss
 *   L = sum_i Wbar_i lambda_i + Re sum_i Xbar_i^H x_i
 * (first-order perturbation theory of A x = lambda B x with x^H B x = 1 and the
 * gauge of hgv_gauge_fix).  Inputs: lambda (all n eigenvalues, ascending),
 * Xall (n x n, all B-orthonormal eigenvectors; columns il..iu gauge fixed),
 * Wbar (m doubles), Xbar (n x m).  Outputs: Abar, Bbar (n x n, Hermitian, full
 * storage) such that dL = Re tr(Abar^H dA) + Re tr(Bbar^H dB) for Hermitian dA,
 * dB.  Argument numbers for -i: ctx 1, n 2, il 3, iu 4, lambda 5, Xall 6,
 * ldxa 7, Wbar 8, Xbar 9, ldxb 10, Abar 11, ldab 12, Bbar 13, ldbb 14, work 15. */
int hgv_zhegvx_backward(hgv_ctx_t ctx, int n, int il, int iu, const double *lambda, const hgv_c128 *Xall,
                        int ldxa, const double *Wbar, const hgv_c128 *Xbar, int ldxb, hgv_c128 *Abar, int ldab,
                        hgv_c128 *Bbar, int ldbb, void *work, size_t work_bytes);

/* ---- diagnostics ------------------------------------------------------------ */
/* Measures, on the context's device, the FP64 MFMA rate in TFLOP/s
 * (independent v_mfma_f64_16x16x4f64 chains with no memory traffic, 16 waves
 * per CU) and the copy bandwidth in GB/s (bytes read plus bytes written by
 * 16-byte loads and stores): the denominators of the roofline fractions,
 * measured next to the published peaks.  work: device buffer, 256-byte
 * aligned, work_bytes >= 4 MiB; the copy runs over all but its first few MiB
 * (half source, half destination), so pass well over the 256 MB on-package
 * cache (e.g. 2 GiB) to measure HBM.  The contents of work are overwritten.
 * Synchronizes the stream; results are host doubles.  HGV_E_WORKSPACE if
 * work_bytes is too small.  Argument numbers for -i: ctx 1, work 2,
 * work_bytes 3, fp64_mfma_tflops 4, copy_gbs 5. */
int hgv_device_peaks(hgv_ctx_t ctx, void *work, size_t work_bytes, double *fp64_mfma_tflops, double *copy_gbs);

/* ---- building block -------------------------------------------------------- */
/* C <- alpha op(A) op(B) + beta C on the MFMA tiles the stages use.
 * opa/opb: 'N', 'T' (transpose) or 'C' (conjugate transpose).  C is m x n,
 * op(A) m x k, op(B) k x n.  `work` (hgv_stage_bufsize(HGV_ST_NSTAGES...) not
 * needed: may be NULL) is unused for these shapes. */
int hgv_zgemm(hgv_ctx_t ctx, char opa, char opb, int m, int n, int k, hgv_c128 alpha,
              const hgv_c128 *A, int lda, const hgv_c128 *B, int ldb, hgv_c128 beta,
              hgv_c128 *C, int ldc);

#ifdef __cplusplus
}
#endif

#endif /* HGV_H */
