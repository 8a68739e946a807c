// adjoint.hip -- reverse-mode derivative of the selected eigenpairs of the
// pencil (A, B) (the differentiable solve).
//
// Loss L = sum_i wbar_i lambda_i + Re sum_i xbar_i^H x_i over the pairs il..iu,
// eigenvectors B-normalised and gauge fixed (the entry of largest modulus,
// first on ties, real and positive).  First-order perturbation of
// A x = lambda B x, x^H B x = 1 gives, with the gauge folded into the
// cotangent  g_i = xbar_i + i c_i e_{k_i},  c_i = Im(xbar_i^H x_i) / x_{k_i,i}:
//   Abar = herm( X diag(wbar) X^H + Z X^H ),
//   Bbar = -herm( X diag(wbar lambda + Re(g^H x)/2) X^H + Z diag(lambda) X^H ),
//   Z    = Xall (F o (Xall^H G)),  F_ji = 1 / (lambda_i - lambda_j), F_ii = 0,
// where Xall holds every eigenvector (the sum over j runs over the complement
// of the selected pairs too).  herm(M) = (M + M^H) / 2.  The products are MFMA
// GEMMs (gemm.hip); the element-wise steps are the kernels below.
#include <algorithm>

#include "hgv_internal.h"

namespace hgv {

// Per column: k = argmax_r |x_r| (smallest r on ties), then scale the column
// by conj(x_k)/|x_k| so that x_k becomes real and positive.
__global__ __launch_bounds__(256) void gauge_fix_kernel(int n, double2 *X, int ldx) {
    __shared__ double bv[256];
    __shared__ int bi[256];
    const int col = blockIdx.x, tid = threadIdx.x;
    double2 *x = X + (size_t)col * ldx;
    double best = -1.0;
    int bidx = 0x7fffffff;
    for (int r = tid; r < n; r += 256) {
        double a = zabs2(x[r]);
        if (a > best) { best = a; bidx = r; }
    }
    bv[tid] = best;
    bi[tid] = bidx;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) {
            double a = bv[tid + o];
            int ia = bi[tid + o];
            if (a > bv[tid] || (a == bv[tid] && ia < bi[tid])) { bv[tid] = a; bi[tid] = ia; }
        }
        __syncthreads();
    }
    const int k = (bi[0] < n) ? bi[0] : 0;   // (only non-finite columns leave no maximum)
    double2 piv = x[k];
    double mag = sqrt(zabs2(piv));
    double2 ph = (mag > 0.0) ? make_double2(piv.x / mag, -piv.y / mag) : make_double2(1.0, 0.0);
    __syncthreads();
    for (int r = tid; r < n; r += 256)
        if (r != k) x[r] = zmul(x[r], ph);
    if (tid == 0 && mag > 0.0) x[k] = make_double2(mag, 0.0);
}

// Per selected column i: G = xbar with the gauge term added at k_i, s_i = Re(xbar_i^H x_i).
__global__ __launch_bounds__(256) void adj_prep_kernel(int n, const double2 *X, int ldx, const double2 *Xbar,
                                                       int ldxb, double2 *G, int ldg, double *s) {
    __shared__ double bv[256];
    __shared__ int bi[256];
    __shared__ double2 red[256];
    const int col = blockIdx.x, tid = threadIdx.x;
    const double2 *x = X + (size_t)col * ldx;
    const double2 *gb = Xbar + (size_t)col * ldxb;
    double best = -1.0;
    int bidx = 0x7fffffff;
    double2 acc = make_double2(0.0, 0.0);
    for (int r = tid; r < n; r += 256) {
        double2 xv = x[r];
        double a = zabs2(xv);
        if (a > best) { best = a; bidx = r; }
        acc = zadd(acc, zcmul(gb[r], xv));
    }
    bv[tid] = best;
    bi[tid] = bidx;
    red[tid] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) {
            double a = bv[tid + o];
            int ia = bi[tid + o];
            if (a > bv[tid] || (a == bv[tid] && ia < bi[tid])) { bv[tid] = a; bi[tid] = ia; }
            red[tid] = zadd(red[tid], red[tid + o]);
        }
        __syncthreads();
    }
    const int k = (bi[0] < n) ? bi[0] : 0;
    const double2 ghx = red[0];
    const double xk = x[k].x;
    const double c = (xk != 0.0) ? ghx.y / xk : 0.0;
    double2 *g = G + (size_t)col * ldg;
    for (int r = tid; r < n; r += 256) {
        double2 v = gb[r];
        if (r == k) v.y += c;
        g[r] = v;
    }
    if (tid == 0) s[col] = ghx.x;
}

// C[j, i] <- C[j, i] / (lambda_{il-1+i} - lambda_j), zero at j = il-1+i.
__global__ void adj_fmul_kernel(int n, int m, int il, const double *lam, double2 *C, int ldc) {
    int j = blockIdx.x * 64 + (threadIdx.x & 63);
    int i = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (j >= n || i >= m) return;
    int ii = il - 1 + i;
    double2 v = C[j + (size_t)i * ldc];
    C[j + (size_t)i * ldc] = (j == ii) ? make_double2(0.0, 0.0) : zscale(1.0 / (lam[ii] - lam[j]), v);
}

// P = X diag(wbar) + Z ;  Q = X diag(wbar lambda + s/2) + Z diag(lambda)   (Z overwritten by Q)
__global__ void adj_pq_kernel(int n, int m, int il, const double *lam, const double *wbar, const double *s,
                              const double2 *X, int ldx, double2 *Z, int ldz, double2 *P, int ldp) {
    int r = blockIdx.x * 64 + (threadIdx.x & 63);
    int i = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (r >= n || i >= m) return;
    double l = lam[il - 1 + i], w = wbar[i];
    double2 x = X[r + (size_t)i * ldx], z = Z[r + (size_t)i * ldz];
    P[r + (size_t)i * ldp] = zadd(zscale(w, x), z);
    Z[r + (size_t)i * ldz] = zadd(zscale(w * l + 0.5 * s[i], x), zscale(l, z));
}

// M <- alpha (M + M^H) / 2 in place (each pair (i, j), (j, i) by one thread).
__global__ void herm_kernel(int n, double2 *M, int ldm, double alpha) {
    int i = blockIdx.x * 16 + (threadIdx.x & 15);
    int j = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (i >= n || j >= n || i < j) return;
    if (i == j) {
        M[i + (size_t)i * ldm] = make_double2(alpha * M[i + (size_t)i * ldm].x, 0.0);
        return;
    }
    double2 a = M[i + (size_t)j * ldm], b = M[j + (size_t)i * ldm];
    double2 h = zscale(0.5 * alpha, zadd(a, zconj(b)));
    M[i + (size_t)j * ldm] = h;
    M[j + (size_t)i * ldm] = zconj(h);
}

void gauge_fix_run(hgv_ctx_s *ctx, int n, int m, double2 *X, int ldx) {
    if (n <= 0 || m <= 0) return;
    hipLaunchKernelGGL(gauge_fix_kernel, dim3(m), dim3(256), 0, ctx->stream, n, X, ldx);
    HGV_LAUNCH_CHECK();
}

void adjoint_run(hgv_ctx_s *ctx, int n, int il, int iu, const double *lam, const double2 *Xall, int ldxa,
                 const double *wbar, const double2 *Xbar, int ldxb, double2 *Abar, int ldab, double2 *Bbar, int ldbb,
                 Arena &ar) {
    const int m = iu - il + 1;
    size_t wsb = zgemm_splitk_bytes(n);
    double2 *ws = ar.take<double2>(wsb / sizeof(double2));
    double2 *G = ar.take<double2>((size_t)n * m);
    double2 *C = ar.take<double2>((size_t)n * m);
    double2 *Z = ar.take<double2>((size_t)n * m);
    double2 *P = ar.take<double2>((size_t)n * m);
    double *s = ar.take<double>(m);
    if (ar.measuring() || n == 0 || m <= 0) return;
    const double2 *X = Xall + (size_t)(il - 1) * ldxa;
    hipLaunchKernelGGL(adj_prep_kernel, dim3(m), dim3(256), 0, ctx->stream, n, X, ldxa, Xbar, ldxb, G, n, s);
    HGV_LAUNCH_CHECK();
    ZGemm g;   // C = Xall^H G
    g.m = n; g.n = m; g.k = n;
    g.opa = 'C'; g.A = Xall; g.lda = ldxa;
    g.B = G; g.ldb = n;
    g.C = C; g.ldc = n;
    zgemm(ctx, g, ws, wsb);
    hipLaunchKernelGGL(adj_fmul_kernel, dim3(cdiv(n, 64), cdiv(m, 4)), dim3(256), 0, ctx->stream, n, m, il, lam, C,
                       n);
    HGV_LAUNCH_CHECK();
    g = ZGemm();   // Z = Xall C
    g.m = n; g.n = m; g.k = n;
    g.A = Xall; g.lda = ldxa;
    g.B = C; g.ldb = n;
    g.C = Z; g.ldc = n;
    zgemm(ctx, g, ws, wsb);
    hipLaunchKernelGGL(adj_pq_kernel, dim3(cdiv(n, 64), cdiv(m, 4)), dim3(256), 0, ctx->stream, n, m, il, lam, wbar,
                       s, X, ldxa, Z, n, P, n);
    HGV_LAUNCH_CHECK();
    g = ZGemm();   // Abar = P X^H
    g.m = n; g.n = n; g.k = m;
    g.A = P; g.lda = n;
    g.opb = 'C'; g.B = X; g.ldb = ldxa;
    g.C = Abar; g.ldc = ldab;
    zgemm(ctx, g, ws, wsb);
    g.A = Z;   // Bbar = Q X^H
    g.C = Bbar; g.ldc = ldbb;
    zgemm(ctx, g, ws, wsb);
    hipLaunchKernelGGL(herm_kernel, dim3(cdiv(n, 16), cdiv(n, 16)), dim3(256), 0, ctx->stream, n, Abar, ldab, 1.0);
    HGV_LAUNCH_CHECK();
    hipLaunchKernelGGL(herm_kernel, dim3(cdiv(n, 16), cdiv(n, 16)), dim3(256), 0, ctx->stream, n, Bbar, ldbb, -1.0);
    HGV_LAUNCH_CHECK();
}

}  // namespace hgv
