// variants.hip -- the generalized solve (Alg. 1 with the two-stage Alg. 2) for
// the other storage types of a Hermitian-definite pencil (the paper states the
// method for Hermitian pencils, the real symmetric case included):
//
//  * complex64: every stage runs on complex64 storage with the FP32 MFMA
//    GEMM tiles (Cholesky, reduction to standard form, band reduction, bulge
//    chasing, both back-transformations, back-substitution), the 64 x 64
//    leaves, reflector norms and scalars in FP64, the tridiagonal solve in
//    FP64; eigenvalues are returned in FP32.
//  * real double: the real symmetric pencil is solved as the complex Hermitian
//    pencil with zero imaginary parts.  Every reflector of the solver maps its
//    vector onto a real multiple of e_1, so for real data every reflector, band,
//    tridiagonal and eigenvector stays real: each complex product is formed from
//    three real MFMA products (Ar Br, Ai Bi, (Ar + Ai)(Br + Bi)), and with zero
//    imaginary parts the third accumulates exactly the operands of the first in
//    the same order, so the imaginary parts come out exactly zero.  The real
//    parts are returned.  (This reuses the complex-double kernels at about
//    four times the arithmetic of a real-storage path.)
#include <algorithm>

#include "hgv_internal.h"

namespace hgv {

namespace {

__global__ void real_to_c64_kernel(int n, int m, const double *Z, int ldz, float2 *X, int ldx) {
    int i = blockIdx.x * 64 + (threadIdx.x & 63);
    int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i < n && j < m) X[i + (size_t)j * ldx] = make_float2((float)Z[i + (size_t)j * ldz], 0.0f);
}

__global__ void to_float_kernel(int m, const double *a, float *b) {
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i < m) b[i] = (float)a[i];
}

// real n x m (ld lr) -> complex (ld lc) with zero imaginary parts
__global__ void real_to_z_kernel(int n, int m, const double *R, int lr, double2 *C, int lc) {
    int i = blockIdx.x * 64 + (threadIdx.x & 63);
    int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i < n && j < m) C[i + (size_t)j * lc] = make_double2(R[i + (size_t)j * lr], 0.0);
}

// real parts of a complex n x m matrix (lower triangle only when lower != 0)
__global__ void z_to_real_kernel(int n, int m, const double2 *C, int lc, double *R, int lr, int lower) {
    int i = blockIdx.x * 64 + (threadIdx.x & 63);
    int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i < n && j < m && (!lower || i >= j)) R[i + (size_t)j * lr] = C[i + (size_t)j * lc].x;
}

dim3 grid2(int n, int m) { return dim3(cdiv(n, 64), cdiv(std::max(m, 1), 4)); }

}  // namespace

// Complex64 generalized solve; W in FP32.  values_only: W only.
void chegvx_full(hgv_ctx_s *ctx, int n, float2 *A, int lda, float2 *B, int ldb, int il, int iu, float *W, float2 *X,
                 int ldx, Arena &ar, int nb, bool values_only, int *d_info, StageTimer *tm) {
    const int m = iu - il + 1;
    const int np = cdiv(n, nb);
    const size_t mk0 = ar.mark();
    const bool run = !ar.measuring();
    const double N = n, M = m;
    if (run) set_info(ctx, d_info, 0);
    if (tm) tm->begin(HGV_ST_POTRF);
    potrf_hegst_t<float2>(ctx, n, B, ldb, A, lda, ar, d_info, n, tm, 4.0 / 3.0 * N * N * N);
    ar.release(mk0);
    if (tm) tm->end(HGV_ST_HEGST, 4.0 * N * N * N);

    float2 *T1 = ar.take<float2>((size_t)np * nb * nb);
    double *d = ar.take<double>(n);
    double *e = ar.take<double>(std::max(n - 1, 1));
    double *Wd = ar.take<double>(std::max(m, 1));
    const size_t mk1 = ar.mark();
    if (tm) tm->begin(HGV_ST_HE2HB);
    he2hb_t<float2>(ctx, n, nb, A, lda, T1, ar, d_info);
    ar.release(mk1);
    if (tm) tm->end(HGV_ST_HE2HB, 16.0 / 3.0 * N * N * N);

    if (values_only) {
        if (tm) tm->begin(HGV_ST_HB2ST);
        hb2st_t<float2>(ctx, n, nb, A, lda, d, e, nullptr, nullptr, ar, d_info);
        ar.release(mk1);
        if (tm) tm->end(HGV_ST_HB2ST, 24.0 * N * N * nb);
        if (tm) tm->begin(HGV_ST_STEDC);
        stebz_run(ctx, n, d, e, il, m, nullptr, Wd, ar);
        ar.release(mk1);
        if (run) {
            hipLaunchKernelGGL(to_float_kernel, dim3(cdiv(m, 256)), dim3(256), 0, ctx->stream, m, Wd, W);
            HGV_LAUNCH_CHECK();
        }
        if (tm) tm->end(HGV_ST_STEDC, 0.0);
        ar.release(mk0);
        return;
    }

    float2 *V2 = ar.take<float2>(v2_elems(n, nb));
    float2 *tau2 = ar.take<float2>(v2_taus(n, nb));
    float2 *T2 = ar.take<float2>(q2_t_elems(n, nb));
    double *lambda = ar.take<double>(n);
    double *Z = ar.take<double>((size_t)n * m);
    const size_t mk2 = ar.mark();
    if (tm) tm->begin(HGV_ST_HB2ST);
    hb2st_t<float2>(ctx, n, nb, A, lda, d, e, V2, tau2, ar, d_info);
    ar.release(mk2);
    if (tm) tm->end(HGV_ST_HB2ST, 24.0 * N * N * nb);

    if (tm) tm->begin(HGV_ST_STEDC);
    stedc_run(ctx, n, d, e, il, iu, lambda, Z, n, ar, d_info);
    ar.release(mk2);
    if (run) {
        hipLaunchKernelGGL(to_float_kernel, dim3(cdiv(m, 256)), dim3(256), 0, ctx->stream, m, lambda + (il - 1), W);
        HGV_LAUNCH_CHECK();
        hipLaunchKernelGGL(real_to_c64_kernel, grid2(n, m), dim3(256), 0, ctx->stream, n, m, Z, n, X, ldx);
        HGV_LAUNCH_CHECK();
    }
    if (tm) tm->end(HGV_ST_STEDC, 4.0 / 3.0 * N * N * N);

    if (tm) tm->begin(HGV_ST_Q2);
    if (run) {
        q2_build_t<float2>(ctx, n, nb, V2, tau2, T2);
        q2_apply_t<float2>(ctx, n, nb, m, V2, T2, X, ldx, false);
    }
    if (tm) tm->end(HGV_ST_Q2, 8.0 * N * N * M);

    if (tm) tm->begin(HGV_ST_Q1);
    unmtr_q1_t<float2>(ctx, n, nb, m, A, lda, T1, X, ldx, false, ar);
    ar.release(mk2);
    if (tm) tm->end(HGV_ST_Q1, 8.0 * N * N * M);

    if (tm) tm->begin(HGV_ST_TRSM);
    trsm_lh_t<float2>(ctx, n, m, B, ldb, X, ldx, ar);
    ar.release(mk2);
    if (tm) tm->end(HGV_ST_TRSM, 4.0 * N * N * M);
    ar.release(mk0);
}

// Conversions of the real front end (the solve itself is the complex-double one).
void real_to_complex(hgv_ctx_s *ctx, int n, int m, const double *R, int lr, double2 *C, int lc) {
    if (n <= 0 || m <= 0) return;
    hipLaunchKernelGGL(real_to_z_kernel, grid2(n, m), dim3(256), 0, ctx->stream, n, m, R, lr, C, lc);
    HGV_LAUNCH_CHECK();
}

void complex_real_part(hgv_ctx_s *ctx, int n, int m, const double2 *C, int lc, double *R, int lr, bool lower) {
    if (n <= 0 || m <= 0) return;
    hipLaunchKernelGGL(z_to_real_kernel, grid2(n, m), dim3(256), 0, ctx->stream, n, m, C, lc, R, lr, lower ? 1 : 0);
    HGV_LAUNCH_CHECK();
}

}  // namespace hgv
