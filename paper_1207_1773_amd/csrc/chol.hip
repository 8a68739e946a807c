// chol.hip -- Cholesky factorisation B = L L^H (Alg. 1 step 1), the
// triangular solves with L, and the reduction to standard form
// A' = L^-1 A L^-H (Alg. 1 step 2, the xHEGST operation the paper runs with
// its level-3 work on the accelerator).
//
// All three are recursive: an order-n problem splits at n1 (a multiple of 64
// near n/2) into two halves joined by large MFMA GEMMs (herk / her2k / hemm /
// gemm updates with K up to n/2), so nearly all flops run in gemm.hip.  The
// leaves (order <= 64) are single-workgroup kernels working out of LDS and
// registers.
#include "hgv_internal.h"

namespace hgv {

constexpr int LEAF = 64;

static int split_point(int n) {
    int n1 = ((n / 2 + LEAF - 1) / LEAF) * LEAF;
    if (n1 >= n) n1 = n - LEAF;
    if (n1 <= 0) n1 = n / 2;
    return n1;
}

// ---- leaf Cholesky (n <= 64), one workgroup -----------------------------------
// Right-looking unblocked Cholesky of the lower triangle held in LDS.  A
// non-positive (or NaN) pivot at local column j records info = base + j + 1
// (first failure wins) and stops the factorisation of this block.
__global__ __launch_bounds__(256) void potf2_kernel(int n, double2 *A, int lda, int *info, int base) {
    __shared__ double2 S[LEAF][LEAF + 1];
    __shared__ int fail;
    const int tid = threadIdx.x;
    for (int t = tid; t < n * n; t += 256) {
        int i = t % n, j = t / n;
        if (i >= j) S[i][j] = A[i + (size_t)j * lda];
    }
    if (tid == 0) fail = 0;
    __syncthreads();
    for (int j = 0; j < n; ++j) {
        if (tid == 0) {
            double piv = S[j][j].x;
            if (!(piv > 0.0)) {
                fail = 1;
                if (info && *info == 0) *info = base + j + 1;
            } else {
                S[j][j] = make_double2(sqrt(piv), 0.0);
            }
        }
        __syncthreads();
        if (fail) break;
        double inv = 1.0 / S[j][j].x;
        for (int i = j + 1 + tid; i < n; i += 256) S[i][j] = zscale(inv, S[i][j]);
        __syncthreads();
        // trailing update of the lower triangle: S[i][k] -= S[i][j] conj(S[k][j]), j < k <= i
        int m = n - j - 1;
        for (int t = tid; t < m * m; t += 256) {
            int i = j + 1 + t % m, k = j + 1 + t / m;
            if (i >= k) {
                double2 a = S[i][j], b = S[k][j];
                double2 p = make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);  // a * conj(b)
                S[i][k] = zsub(S[i][k], p);
            }
        }
        __syncthreads();
    }
    for (int t = tid; t < n * n; t += 256) {
        int i = t % n, j = t / n;
        if (i >= j) A[i + (size_t)j * lda] = S[i][j];
    }
}

// ---- leaf triangular solves (order n <= 64), one wave per 64 right-hand sides --
// mode 0 (right, L^H):  X (rows) <- X L^-H : x_j = (b_j - sum_{k<j} x_k conj(L_jk)) / L_jj
// mode 1 (left,  L):    X (cols) <- L^-1 X : x_i = (b_i - sum_{k<i} L_ik x_k) / L_ii
// mode 2 (left,  L^H):  X (cols) <- L^-H X : x_i = (b_i - sum_{k>i} conj(L_ki) x_k) / L_ii
// Each lane keeps its right-hand side in registers; L is broadcast from LDS.
// Columns (modes 1, 2) are staged through LDS so global accesses coalesce.
template <int MODE>
__global__ __launch_bounds__(64) void trsm_leaf_kernel(int n, int nrhs, const double2 *L, int ldl,
                                                       double2 *X, int ldx) {
    __shared__ double2 Ls[LEAF][LEAF + 1];
    __shared__ double2 Xs[LEAF][LEAF + 1];
    const int lane = threadIdx.x;
    const int r0 = blockIdx.x * 64;
    for (int t = lane; t < n * n; t += 64) {
        int i = t % n, j = t / n;
        Ls[i][j] = (i >= j) ? L[i + (size_t)j * ldl] : make_double2(0.0, 0.0);
    }
    double2 x[LEAF];
    const int my = r0 + lane;
    if (MODE == 0) {
#pragma unroll
        for (int k = 0; k < LEAF; ++k)
            x[k] = (k < n && my < nrhs) ? X[my + (size_t)k * ldx] : make_double2(0.0, 0.0);
    } else {
        // stage columns r0..r0+63 (n rows each) through LDS: Xs[i][c]
        for (int t = lane; t < n * 64; t += 64) {
            int i = t % n, c = t / n;
            Xs[i][c] = (r0 + c < nrhs) ? X[i + (size_t)(r0 + c) * ldx] : make_double2(0.0, 0.0);
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < LEAF; ++k) x[k] = (k < n) ? Xs[k][lane] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    if (MODE == 0 || MODE == 1) {
#pragma unroll
        for (int j = 0; j < LEAF; ++j) {
            if (j < n) {
                double2 s = x[j];
#pragma unroll
                for (int k = 0; k < j; ++k) {
                    double2 l = Ls[j][k];
                    if (MODE == 0) s = zsub(s, zmul(x[k], zconj(l)));
                    else s = zsub(s, zmul(l, x[k]));
                }
                double2 d = Ls[j][j];
                x[j] = (MODE == 0) ? zdiv(s, zconj(d)) : zdiv(s, d);
            }
        }
    } else {
#pragma unroll
        for (int jj = LEAF - 1; jj >= 0; --jj) {
            if (jj < n) {
                double2 s = x[jj];
#pragma unroll
                for (int k = jj + 1; k < LEAF; ++k)
                    if (k < n) s = zsub(s, zmul(zconj(Ls[k][jj]), x[k]));
                x[jj] = zdiv(s, zconj(Ls[jj][jj]));
            }
        }
    }
    if (MODE == 0) {
        if (my < nrhs) {
#pragma unroll
            for (int k = 0; k < LEAF; ++k)
                if (k < n) X[my + (size_t)k * ldx] = x[k];
        }
    } else {
#pragma unroll
        for (int k = 0; k < LEAF; ++k)
            if (k < n) Xs[k][lane] = x[k];
        __syncthreads();
        for (int t = lane; t < n * 64; t += 64) {
            int i = t % n, c = t / n;
            if (r0 + c < nrhs) X[i + (size_t)(r0 + c) * ldx] = Xs[i][c];
        }
    }
}

// ---- leaf reduction to standard form (n <= 64), one workgroup ---------------------
// C = L^-1 A L^-H for the block: W = L^-1 A (A full Hermitian from its lower
// triangle), then C = L^-1 W^H; the lower triangle of (C + C^H)/2 is written.
__global__ __launch_bounds__(64) void hegs2_kernel(int n, double2 *A, int lda, const double2 *L, int ldl) {
    __shared__ double2 Ls[LEAF][LEAF + 1];
    __shared__ double2 Ws[LEAF][LEAF + 1];
    const int lane = threadIdx.x;
    for (int t = lane; t < n * n; t += 64) {
        int i = t % n, j = t / n;
        Ls[i][j] = (i >= j) ? L[i + (size_t)j * ldl] : make_double2(0.0, 0.0);
        double2 a;
        if (i > j) a = A[i + (size_t)j * lda];
        else if (i == j) a = make_double2(A[i + (size_t)i * lda].x, 0.0);
        else a = zconj(A[j + (size_t)i * lda]);
        Ws[i][j] = a;
    }
    __syncthreads();
    double2 x[LEAF];
    // pass 1: column `lane` of W = L^-1 A
#pragma unroll
    for (int k = 0; k < LEAF; ++k) x[k] = (k < n && lane < n) ? Ws[k][lane] : make_double2(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < LEAF; ++j) {
        if (j < n) {
            double2 s = x[j];
#pragma unroll
            for (int k = 0; k < j; ++k) s = zsub(s, zmul(Ls[j][k], x[k]));
            x[j] = zdiv(s, Ls[j][j]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < LEAF; ++k)
        if (k < n && lane < n) Ws[k][lane] = x[k];
    __syncthreads();
    // pass 2: column `lane` of C = L^-1 W^H, i.e. right-hand side conj(W[lane, :])
#pragma unroll
    for (int k = 0; k < LEAF; ++k) x[k] = (k < n && lane < n) ? zconj(Ws[lane][k]) : make_double2(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < LEAF; ++j) {
        if (j < n) {
            double2 s = x[j];
#pragma unroll
            for (int k = 0; k < j; ++k) s = zsub(s, zmul(Ls[j][k], x[k]));
            x[j] = zdiv(s, Ls[j][j]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < LEAF; ++k)
        if (k < n && lane < n) Ws[k][lane] = x[k];
    __syncthreads();
    for (int t = lane; t < n * n; t += 64) {
        int i = t % n, j = t / n;
        if (i > j) A[i + (size_t)j * lda] = zscale(0.5, zadd(Ws[i][j], zconj(Ws[j][i])));
        else if (i == j) A[i + (size_t)i * lda] = make_double2(Ws[i][i].x, 0.0);
    }
}

// ---- recursive drivers -----------------------------------------------------------------
static double2 *gemm_ws(Arena &ar, int n, size_t &bytes) {
    bytes = zgemm_splitk_bytes(n);
    return ar.take<double2>(bytes / sizeof(double2));
}

template <int MODE>
static void trsm_leaf(hgv_ctx_s *ctx, int n, int nrhs, const double2 *L, int ldl, double2 *X, int ldx) {
    if (n <= 0 || nrhs <= 0) return;
    hipLaunchKernelGGL((trsm_leaf_kernel<MODE>), dim3(cdiv(nrhs, 64)), dim3(64), 0, ctx->stream, n, nrhs, L,
                       ldl, X, ldx);
    HGV_LAUNCH_CHECK();
}

static void trsm_right_lc_rec(hgv_ctx_s *ctx, int m, int n, const double2 *L, int ldl, double2 *X, int ldx,
                              double2 *ws, size_t wsb) {
    if (m <= 0 || n <= 0) return;
    if (n <= LEAF) {
        trsm_leaf<0>(ctx, n, m, L, ldl, X, ldx);
        return;
    }
    int n1 = split_point(n), n2 = n - n1;
    trsm_right_lc_rec(ctx, m, n1, L, ldl, X, ldx, ws, wsb);
    ZGemm g;  // X2 -= X1 L21^H
    g.m = m; g.n = n2; g.k = n1;
    g.opa = 'N'; g.A = X; g.lda = ldx;
    g.opb = 'C'; g.B = L + n1; g.ldb = ldl;
    g.alpha = make_double2(-1.0, 0.0); g.beta = make_double2(1.0, 0.0);
    g.C = X + (size_t)n1 * ldx; g.ldc = ldx;
    zgemm(ctx, g, ws, wsb);
    trsm_right_lc_rec(ctx, m, n2, L + n1 + (size_t)n1 * ldl, ldl, X + (size_t)n1 * ldx, ldx, ws, wsb);
}

static void trsm_left_ln_rec(hgv_ctx_s *ctx, int n, int m, const double2 *L, int ldl, double2 *X, int ldx,
                             double2 *ws, size_t wsb) {
    if (m <= 0 || n <= 0) return;
    if (n <= LEAF) {
        trsm_leaf<1>(ctx, n, m, L, ldl, X, ldx);
        return;
    }
    int n1 = split_point(n), n2 = n - n1;
    trsm_left_ln_rec(ctx, n1, m, L, ldl, X, ldx, ws, wsb);
    ZGemm g;  // X2 -= L21 X1
    g.m = n2; g.n = m; g.k = n1;
    g.opa = 'N'; g.A = L + n1; g.lda = ldl;
    g.opb = 'N'; g.B = X; g.ldb = ldx;
    g.alpha = make_double2(-1.0, 0.0); g.beta = make_double2(1.0, 0.0);
    g.C = X + n1; g.ldc = ldx;
    zgemm(ctx, g, ws, wsb);
    trsm_left_ln_rec(ctx, n2, m, L + n1 + (size_t)n1 * ldl, ldl, X + n1, ldx, ws, wsb);
}

static void trsm_left_lc_rec(hgv_ctx_s *ctx, int n, int m, const double2 *L, int ldl, double2 *X, int ldx,
                             double2 *ws, size_t wsb) {
    if (m <= 0 || n <= 0) return;
    if (n <= LEAF) {
        trsm_leaf<2>(ctx, n, m, L, ldl, X, ldx);
        return;
    }
    int n1 = split_point(n), n2 = n - n1;
    trsm_left_lc_rec(ctx, n2, m, L + n1 + (size_t)n1 * ldl, ldl, X + n1, ldx, ws, wsb);
    ZGemm g;  // X1 -= L21^H X2
    g.m = n1; g.n = m; g.k = n2;
    g.opa = 'C'; g.A = L + n1; g.lda = ldl;
    g.opb = 'N'; g.B = X + n1; g.ldb = ldx;
    g.alpha = make_double2(-1.0, 0.0); g.beta = make_double2(1.0, 0.0);
    g.C = X; g.ldc = ldx;
    zgemm(ctx, g, ws, wsb);
    trsm_left_lc_rec(ctx, n1, m, L, ldl, X, ldx, ws, wsb);
}

void trsm_right_lc(hgv_ctx_s *ctx, int m, int n, const double2 *L, int ldl, double2 *X, int ldx, Arena &ar) {
    size_t b;
    double2 *ws = gemm_ws(ar, n, b);
    if (ar.measuring()) return;
    trsm_right_lc_rec(ctx, m, n, L, ldl, X, ldx, ws, b);
}
void trsm_left_ln(hgv_ctx_s *ctx, int n, int m, const double2 *L, int ldl, double2 *X, int ldx, Arena &ar) {
    size_t b;
    double2 *ws = gemm_ws(ar, n, b);
    if (ar.measuring()) return;
    trsm_left_ln_rec(ctx, n, m, L, ldl, X, ldx, ws, b);
}
void trsm_left_lc(hgv_ctx_s *ctx, int n, int m, const double2 *L, int ldl, double2 *X, int ldx, Arena &ar) {
    size_t b;
    double2 *ws = gemm_ws(ar, n, b);
    if (ar.measuring()) return;
    trsm_left_lc_rec(ctx, n, m, L, ldl, X, ldx, ws, b);
}
void trsm_lh_run(hgv_ctx_s *ctx, int n, int m, const double2 *L, int ldl, double2 *X, int ldx, Arena &ar) {
    trsm_left_lc(ctx, n, m, L, ldl, X, ldx, ar);
}

static void potrf_rec(hgv_ctx_s *ctx, int n, double2 *A, int lda, int *info, int base, double2 *ws,
                      size_t wsb) {
    if (n <= 0) return;
    if (n <= LEAF) {
        hipLaunchKernelGGL(potf2_kernel, dim3(1), dim3(256), 0, ctx->stream, n, A, lda, info, base);
        HGV_LAUNCH_CHECK();
        return;
    }
    int n1 = split_point(n), n2 = n - n1;
    potrf_rec(ctx, n1, A, lda, info, base, ws, wsb);
    trsm_right_lc_rec(ctx, n2, n1, A, lda, A + n1, lda, ws, wsb);  // L21 = A21 L11^-H
    ZGemm g;  // A22 -= L21 L21^H (lower)
    g.m = n2; g.n = n2; g.k = n1;
    g.opa = 'N'; g.A = A + n1; g.lda = lda;
    g.opb = 'C'; g.B = A + n1; g.ldb = lda;
    g.alpha = make_double2(-1.0, 0.0); g.beta = make_double2(1.0, 0.0);
    g.C = A + n1 + (size_t)n1 * lda; g.ldc = lda;
    g.lower = 1;
    zgemm(ctx, g, ws, wsb);
    potrf_rec(ctx, n2, A + n1 + (size_t)n1 * lda, lda, info, base + n1, ws, wsb);
}

void potrf_run(hgv_ctx_s *ctx, int n, double2 *B, int ldb, Arena &ar, int *d_info, int info_offset) {
    size_t b;
    double2 *ws = gemm_ws(ar, n, b);
    if (ar.measuring()) return;
    potrf_rec(ctx, n, B, ldb, d_info, info_offset, ws, b);
}

static void hegst_rec(hgv_ctx_s *ctx, int n, double2 *A, int lda, const double2 *L, int ldl, double2 *ws,
                      size_t wsb) {
    if (n <= 0) return;
    if (n <= LEAF) {
        hipLaunchKernelGGL(hegs2_kernel, dim3(1), dim3(64), 0, ctx->stream, n, A, lda, L, ldl);
        HGV_LAUNCH_CHECK();
        return;
    }
    int n1 = split_point(n), n2 = n - n1;
    double2 *A11 = A, *A21 = A + n1, *A22 = A + n1 + (size_t)n1 * lda;
    const double2 *L11 = L, *L21 = L + n1, *L22 = L + n1 + (size_t)n1 * ldl;
    hegst_rec(ctx, n1, A11, lda, L11, ldl, ws, wsb);
    trsm_right_lc_rec(ctx, n2, n1, L11, ldl, A21, lda, ws, wsb);  // A21 <- A21 L11^-H
    fill_upper_from_lower(ctx, n1, A11, lda);                      // A'11 as a full matrix
    ZGemm h;  // A21 -= 1/2 L21 A'11
    h.m = n2; h.n = n1; h.k = n1;
    h.opa = 'N'; h.A = L21; h.lda = ldl;
    h.opb = 'N'; h.B = A11; h.ldb = lda;
    h.alpha = make_double2(-0.5, 0.0); h.beta = make_double2(1.0, 0.0);
    h.C = A21; h.ldc = lda;
    zgemm(ctx, h, ws, wsb);
    ZGemm r;  // A22 -= A21 L21^H + L21 A21^H (lower)
    r.m = n2; r.n = n2; r.k = n1;
    r.opa = 'N'; r.A = A21; r.lda = lda;
    r.opb = 'C'; r.B = L21; r.ldb = ldl;
    r.opa2 = 'N'; r.A2 = L21; r.lda2 = ldl;
    r.opb2 = 'C'; r.B2 = A21; r.ldb2 = lda;
    r.alpha = make_double2(-1.0, 0.0); r.beta = make_double2(1.0, 0.0);
    r.C = A22; r.ldc = lda;
    r.lower = 1;
    zgemm(ctx, r, ws, wsb);
    zgemm(ctx, h, ws, wsb);                                        // A21 -= 1/2 L21 A'11
    trsm_left_ln_rec(ctx, n2, n1, L22, ldl, A21, lda, ws, wsb);   // A21 <- L22^-1 A21
    hegst_rec(ctx, n2, A22, lda, L22, ldl, ws, wsb);
}

void hegst_run(hgv_ctx_s *ctx, int n, double2 *A, int lda, const double2 *L, int ldl, Arena &ar) {
    size_t b;
    double2 *ws = gemm_ws(ar, n, b);
    if (ar.measuring()) return;
    hegst_rec(ctx, n, A, lda, L, ldl, ws, b);
}

}  // namespace hgv
