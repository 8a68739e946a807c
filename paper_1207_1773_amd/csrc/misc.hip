// misc.hip -- small element-wise kernels shared by the stages.
#include "hgv_internal.h"

namespace hgv {

// A[j, i] = conj(A[i, j]) for i > j (upper triangle made the mirror of the lower)
__global__ void fill_upper_kernel(int n, double2 *A, int lda) {
    int i = blockIdx.x * 16 + (threadIdx.x & 15);   // row of the lower element
    int j = blockIdx.y * 16 + (threadIdx.x >> 4);   // column of the lower element
    if (i < n && j < n && i > j) A[j + (size_t)i * lda] = zconj(A[i + (size_t)j * lda]);
}

__global__ void zero_upper_kernel(int n, double2 *A, int lda) {
    int i = blockIdx.x * 16 + (threadIdx.x & 15);
    int j = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (i < n && j < n && i < j) A[i + (size_t)j * lda] = make_double2(0.0, 0.0);
}

__global__ void copy_kernel(int m, int n, const double2 *A, int lda, double2 *B, int ldb) {
    int i = blockIdx.x * 64 + (threadIdx.x & 63);
    int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i < m && j < n) B[i + (size_t)j * ldb] = A[i + (size_t)j * lda];
}

__global__ void add_scaled_kernel(int m, int n, double alpha, const double2 *X, int ldx, double2 *Y, int ldy) {
    int i = blockIdx.x * 64 + (threadIdx.x & 63);
    int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i < m && j < n) {
        const double2 x = X[i + (size_t)j * ldx];
        double2 &y = Y[i + (size_t)j * ldy];
        y = make_double2(y.x + alpha * x.x, y.y + alpha * x.y);
    }
}

__global__ void set_int_kernel(int *p, int v) { *p = v; }

void fill_upper_from_lower(hgv_ctx_s *ctx, int n, double2 *A, int lda) {
    if (n <= 1) return;
    hipLaunchKernelGGL(fill_upper_kernel, dim3(cdiv(n, 16), cdiv(n, 16)), dim3(256), 0, ctx->stream, n, A, lda);
    HGV_LAUNCH_CHECK();
}

void zero_strict_upper(hgv_ctx_s *ctx, int n, double2 *A, int lda) {
    if (n <= 1) return;
    hipLaunchKernelGGL(zero_upper_kernel, dim3(cdiv(n, 16), cdiv(n, 16)), dim3(256), 0, ctx->stream, n, A, lda);
    HGV_LAUNCH_CHECK();
}

void copy_matrix(hgv_ctx_s *ctx, int m, int n, const double2 *A, int lda, double2 *B, int ldb) {
    if (m <= 0 || n <= 0) return;
    hipLaunchKernelGGL(copy_kernel, dim3(cdiv(m, 64), cdiv(n, 4)), dim3(256), 0, ctx->stream, m, n, A, lda, B, ldb);
    HGV_LAUNCH_CHECK();
}

void add_scaled(hgv_ctx_s *ctx, int m, int n, double alpha, const double2 *X, int ldx, double2 *Y, int ldy) {
    if (m <= 0 || n <= 0) return;
    hipLaunchKernelGGL(add_scaled_kernel, dim3(cdiv(m, 64), cdiv(n, 4)), dim3(256), 0, ctx->stream, m, n, alpha, X,
                       ldx, Y, ldy);
    HGV_LAUNCH_CHECK();
}

void set_info(hgv_ctx_s *ctx, int *d_info, int value) {
    if (!d_info) return;
    hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(1), 0, ctx->stream, d_info, value);
    HGV_LAUNCH_CHECK();
}

void ensure_lookahead_stream(hgv_ctx_s *ctx) {
    if (ctx->la_stream[0]) return;
    for (hipStream_t &st : ctx->la_stream) HGV_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    for (hipEvent_t &e : ctx->la_ev) HGV_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
}

__global__ void wait_fail_kernel(const int *err, int *d_info, int code) {
    if (*err != 0 && *d_info == 0) *d_info = code;
}

void report_wait_fail(hgv_ctx_s *ctx, const int *err, int *d_info, int code) {
    if (!d_info) return;
    hipLaunchKernelGGL(wait_fail_kernel, dim3(1), dim3(1), 0, ctx->stream, err, d_info, code);
    HGV_LAUNCH_CHECK();
}

}  // namespace hgv
