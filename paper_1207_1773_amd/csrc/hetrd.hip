// hetrd.hip -- one-stage reduction of the Hermitian A' (lower triangle) to a
// real symmetric tridiagonal T = Q^H A' Q by Householder reflectors, blocked by
// panels of nb columns.  This is the one-stage form of the standard eigensolve
// (Sec. 4.1), whose matrix-vector products with the trailing matrix read it
// once per column and are bound by memory bandwidth; the solver keeps it as
// the comparison path of the two-stage reduction (Sec. 4.2), which the paper
// finds about as fast when every eigenvector is wanted.
//
// Reflectors: H = I - tau v v^H with H^H x = beta e_1, beta real, v_0 = 1 (the
// convention of the band reduction), so T comes out real.  Column c of a panel
// (the j-th; N = n - c - 1 rows below the diagonal) takes four kernels:
//  (a) a[c:, c] -= V[c:, 0:j] W[c, 0:j]^H + W[c:, 0:j] V[c, 0:j]^H (the panel's
//      earlier transformations, applied to the matrix only after the panel),
//      with partial sums of ||x||^2, W^H x and V^H x over x = a[c+2:, c];
//  (b) beta, tau and the scale of v = x / (x_0 - beta), and t1 = W^H v,
//      t2 = V^H v (one workgroup);
//  (c) y = A22 v with A22 = A[c+1:, c+1:] as it stood when the panel started
//      (its lower triangle in 64 x 64 tiles, each read once: A_IJ v_J goes to
//      y_I, A_IJ^H v_I to y_J), and s = v^H A22 v;
//  (d) w = tau (y - V t1 - W t2) + alpha v with alpha = -|tau|^2 (s - 2 Re t1^H t2) / 2;
//      then H^H A H = A - v w^H - w v^H on the trailing part, and v, w become
//      column j of V and W.
// After the panel: A[k+nb:, k+nb:] -= V W^H + W V^H (MFMA her2k) and the
// panel's compact-WY factor T (as for the band reduction's panels).
// (Golub & Van Loan, Matrix Computations, Sec. 8.3; the blocked form of
// Dongarra, Sorensen and Hammarling, J. Comput. Appl. Math. 27 (1989).)
#include <algorithm>
#include <cfloat>

#include "hgv_internal.h"

namespace hgv {

namespace {

constexpr int TRD_NB = 64;    // largest panel width
constexpr int TRD_K = 8;      // tiles of one block column per workgroup of the hemv

struct ColState {
    double2 tau, scale;
    double2 t1[TRD_NB], t2[TRD_NB];
};

__device__ inline double2 zero2d() { return make_double2(0.0, 0.0); }

// (a) column update and partial sums; grid over rows c .. n-1, 256 per workgroup.
// part per workgroup: [0] = sum |x_i|^2 (x = rows c+2 ..), [1 + l] = sum conj(W[i,l]) x_i,
// [1 + nbw + l] = sum conj(V[i,l]) x_i.  V, W: row-major n x nbw.
__global__ __launch_bounds__(256) void trd_colupd_kernel(int n, int c, int j, double2 *A, int lda,
                                                         const double2 *Vp, const double2 *Wp, int nbw,
                                                         double2 *part) {
    __shared__ double2 xs[256];
    __shared__ double2 vr[TRD_NB], wr[TRD_NB];
    __shared__ double red[256];
    __shared__ double2 tr1[4][TRD_NB], tr2[4][TRD_NB];
    const int tid = threadIdx.x, base = c + blockIdx.x * 256, r = base + tid;
    if (tid < j) {
        vr[tid] = zconj(Vp[(size_t)c * nbw + tid]);
        wr[tid] = zconj(Wp[(size_t)c * nbw + tid]);
    }
    __syncthreads();
    double2 x = zero2d();
    if (r < n) {
        x = A[r + (size_t)c * lda];
        const double2 *vrow = Vp + (size_t)r * nbw, *wrow = Wp + (size_t)r * nbw;
        // four independent partial sums (fixed order), so the loads and the
        // multiply-adds of consecutive l overlap instead of forming one chain
        double2 q[4] = {zero2d(), zero2d(), zero2d(), zero2d()};
        int l = 0;
        for (; l + 4 <= j; l += 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) q[u] = zadd(q[u], zadd(zmul(vrow[l + u], wr[l + u]), zmul(wrow[l + u], vr[l + u])));
        }
        for (; l < j; ++l) q[0] = zadd(q[0], zadd(zmul(vrow[l], wr[l]), zmul(wrow[l], vr[l])));
        x = zsub(x, zadd(zadd(q[0], q[1]), zadd(q[2], q[3])));
        if (r == c) x.y = 0.0;
        A[r + (size_t)c * lda] = x;
    }
    const bool below = r >= c + 2 && r < n;
    xs[tid] = below ? x : zero2d();
    red[tid] = below ? zabs2(x) : 0.0;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) red[tid] += red[tid + o];
        __syncthreads();
    }
    const int l = tid & 63, g = tid >> 6;
    double2 a1 = zero2d(), a2 = zero2d();
    if (l < j) {
        for (int rr = g; rr < 256; rr += 4) {
            const int row = base + rr;
            if (row >= c + 2 && row < n) {
                a1 = zadd(a1, zcmul(Wp[(size_t)row * nbw + l], xs[rr]));
                a2 = zadd(a2, zcmul(Vp[(size_t)row * nbw + l], xs[rr]));
            }
        }
    }
    tr1[g][l] = a1;
    tr2[g][l] = a2;
    __syncthreads();
    double2 *out = part + (size_t)blockIdx.x * (1 + 2 * nbw);
    if (tid == 0) out[0] = make_double2(red[0], 0.0);
    if (tid < j) {
        out[1 + tid] = zadd(zadd(tr1[0][tid], tr1[1][tid]), zadd(tr1[2][tid], tr1[3][tid]));
        out[1 + nbw + tid] = zadd(zadd(tr2[0][tid], tr2[1][tid]), zadd(tr2[2][tid], tr2[3][tid]));
    }
}

// (b) reflector of column c, t1 and t2 (one workgroup).
__global__ __launch_bounds__(256) void trd_refl_kernel(int n, int c, int j, int nwg, const double2 *part, int nbw,
                                                       double2 *A, int lda, const double2 *Vp, const double2 *Wp,
                                                       double *d, double *e, double2 *taup, ColState *st) {
    __shared__ double red[256];
    __shared__ double2 sc;
    const int tid = threadIdx.x;
    const int stride = 1 + 2 * nbw;
    double nx = 0.0;
    for (int w = tid; w < nwg; w += 256) nx += part[(size_t)w * stride].x;
    red[tid] = nx;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) red[tid] += red[tid + o];
        __syncthreads();
    }
    if (tid == 0) {
        d[c] = A[c + (size_t)c * lda].x;
        double2 tau = zero2d(), scale = zero2d();
        if (c + 1 < n) {
            const double2 alpha = A[(c + 1) + (size_t)c * lda];
            const double t2 = red[0];
            double beta;
            if (t2 == 0.0 && alpha.y == 0.0) {
                beta = alpha.x;
            } else {
                const double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + t2);
                beta = -copysign(nrm, alpha.x);
                tau = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
                scale = zdiv(make_double2(1.0, 0.0), make_double2(alpha.x - beta, alpha.y));
            }
            e[c] = beta;
            A[(c + 1) + (size_t)c * lda] = make_double2(beta, 0.0);
        }
        taup[j] = tau;
        st->tau = tau;
        st->scale = scale;
        sc = scale;
    }
    __syncthreads();
    if (tid < j && c + 1 < n) {
        // t1 = W^H v, t2 = V^H v with v_0 = 1 (row c+1) and v_i = scale x_i below
        double2 u1 = zero2d(), u2 = zero2d();
        for (int w = 0; w < nwg; ++w) {
            u1 = zadd(u1, part[(size_t)w * stride + 1 + tid]);
            u2 = zadd(u2, part[(size_t)w * stride + 1 + nbw + tid]);
        }
        const double2 s = sc;
        st->t1[tid] = zadd(zconj(Wp[(size_t)(c + 1) * nbw + tid]), zmul(s, u1));
        st->t2[tid] = zadd(zconj(Vp[(size_t)(c + 1) * nbw + tid]), zmul(s, u2));
    }
}

// Workgroup id -> (block column J, chunk q) of the hemv (chunks of TRD_K tiles
// down each block column of the nbk x nbk lower block triangle).
__device__ inline void trd_tile_of(int nbk, int wg, int &J, int &q) {
    J = 0;
    for (; J < nbk; ++J) {
        const int nq = (nbk - J + TRD_K - 1) / TRD_K;
        if (wg < nq) break;
        wg -= nq;
    }
    q = wg;
}

// (c) hemv over the lower triangle of A22 (order N), v = (1, scale x_1, ...).
// Outputs: P[J * ldp + i] = (A_IJ v_J)_i for rows i of blocks I > J; Qv[wg * 64 + t]
// = this workgroup's part of y on block J (the A_IJ^H v_I of its tiles, and for
// the diagonal tile A_JJ v_J); Sv[wg] = its part of v^H A22 v.
__global__ __launch_bounds__(256) void trd_hemv_kernel(int N, const double2 *A22, int lda, const double2 *x,
                                                       const ColState *st, double2 *P, int ldp, double2 *Qv,
                                                       double *Sv) {
    __shared__ double2 vJ[64], vI[64];
    __shared__ double2 ypart[4][64];
    __shared__ double2 yown[64];
    __shared__ double sred[64];
    const int tid = threadIdx.x, lane = tid & 63, cg = tid >> 6;
    const int nbk = (N + 63) / 64;
    int J, q;
    trd_tile_of(nbk, blockIdx.x, J, q);
    const double2 scale = st->scale;
    auto vloc = [&](int i) -> double2 {
        if (i >= N) return zero2d();
        return i == 0 ? make_double2(1.0, 0.0) : zmul(scale, x[i]);
    };
    if (tid < 64) {
        vJ[tid] = vloc(J * 64 + tid);
        yown[tid] = zero2d();
    }
    double2 own[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) own[u] = zero2d();
    double sacc = 0.0;
    const int I0 = J + q * TRD_K, I1 = min(nbk, I0 + TRD_K);
    __syncthreads();
    for (int I = I0; I < I1; ++I) {
        if (tid < 64) vI[tid] = vloc(I * 64 + tid);
        const int row = I * 64 + lane;
        double2 a[16];
        if (I > J) {
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int col = J * 64 + cg * 16 + u;
                const bool in = row < N && col < N;
                const double2 t = A22[(in ? row : 0) + (size_t)(in ? col : 0) * lda];
                a[u] = zsel(in, t, zero2d());
            }
        } else {
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int col = J * 64 + cg * 16 + u;
                const bool in = row < N && col < N;
                double2 t = zero2d();
                if (in) {
                    if (row > col) t = A22[row + (size_t)col * lda];
                    else if (row == col) t = make_double2(A22[row + (size_t)col * lda].x, 0.0);
                    else t = zconj(A22[col + (size_t)row * lda]);
                }
                a[u] = t;
            }
        }
        __syncthreads();   // vI in place
        double2 yp = zero2d();
#pragma unroll
        for (int u = 0; u < 16; ++u) yp = zadd(yp, zmul(a[u], vJ[cg * 16 + u]));
        ypart[cg][lane] = yp;
        if (I > J) {
            const double2 vi = vI[lane];
#pragma unroll
            for (int u = 0; u < 16; ++u) own[u] = zadd(own[u], zcmul(a[u], vi));
        }
        __syncthreads();
        if (tid < 64) {
            const double2 y = zadd(zadd(ypart[0][tid], ypart[1][tid]), zadd(ypart[2][tid], ypart[3][tid]));
            const double sv = zcmul(vI[tid], y).x;   // Re conj(v_I) y
            if (I > J) {
                if (row < N) P[(size_t)J * ldp + row] = y;
                sacc += 2.0 * sv;
            } else {
                yown[tid] = zadd(yown[tid], y);
                sacc += sv;
            }
        }
        __syncthreads();
    }
    // the A_IJ^H v_I parts: sum over the rows (lanes) of each wave's 16 columns
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        double2 t = own[u];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            t.x += __shfl_xor(t.x, o, 64);
            t.y += __shfl_xor(t.y, o, 64);
        }
        own[u] = t;
    }
    if (lane == 0) {
#pragma unroll
        for (int u = 0; u < 16; ++u) ypart[cg][u] = own[u];
    }
    if (tid < 64) sred[tid] = sacc;
    __syncthreads();
    if (tid < 64) {
        const double2 o = ypart[tid >> 4][tid & 15];
        Qv[(size_t)blockIdx.x * 64 + tid] = zadd(yown[tid], o);
    }
    if (tid == 0) {
        double s = 0.0;
        for (int t = 0; t < 64; ++t) s += sred[t];
        Sv[blockIdx.x] = s;
    }
}

// (d) w and v of column c: rows c+1 .. n-1 (local i = 0 .. N-1), 256 per workgroup.
__global__ __launch_bounds__(256) void trd_wfin_kernel(int N, int c, int j, double2 *A, int lda, const ColState *st,
                                                       const double2 *P, int ldp, const double2 *Qv,
                                                       const double *Sv, int nwgc, double2 *Vp, double2 *Wp,
                                                       int nbw) {
    __shared__ double red[256];
    __shared__ double alpha_s;
    __shared__ int qoff[6], qcnt[6];
    const int tid = threadIdx.x;
    const int nbk = (N + 63) / 64;
    double s = 0.0;
    for (int w = tid; w < nwgc; w += 256) s += Sv[w];
    red[tid] = s;
    // first workgroup id and chunk count of the block columns this workgroup's rows fall in
    if (tid == 0) {
        const int Ib = blockIdx.x * 4;
        int off = 0;
        for (int J = 0; J < nbk && J < Ib + 4; ++J) {
            const int nq = (nbk - J + TRD_K - 1) / TRD_K;
            if (J >= Ib) {
                qoff[J - Ib] = off;
                qcnt[J - Ib] = nq;
            }
            off += nq;
        }
    }
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) red[tid] += red[tid + o];
        __syncthreads();
    }
    if (tid == 0) {
        double tt = 0.0;   // Re t1^H t2
        for (int l = 0; l < j; ++l) tt += zcmul(st->t1[l], st->t2[l]).x;
        const double2 tau = st->tau;
        alpha_s = -0.5 * zabs2(tau) * (red[0] - 2.0 * tt);
    }
    __syncthreads();
    const int i = blockIdx.x * 256 + tid;
    if (i >= N) return;
    const int I = i / 64, g = c + 1 + i;
    // y_i: the block-column partials of the product, then the panel's earlier
    // transformations; four independent partial sums each (fixed order)
    double2 yq[4] = {zero2d(), zero2d(), zero2d(), zero2d()};
    {
        int J = 0;
        for (; J + 4 <= I; J += 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) yq[u] = zadd(yq[u], P[(size_t)(J + u) * ldp + i]);
        }
        for (; J < I; ++J) yq[0] = zadd(yq[0], P[(size_t)J * ldp + i]);
    }
    const int lb = I - blockIdx.x * 4;
    for (int q = 0; q < qcnt[lb]; ++q) yq[1] = zadd(yq[1], Qv[(size_t)(qoff[lb] + q) * 64 + (i & 63)]);
    const double2 scale = st->scale, tau = st->tau;
    const double2 v = i == 0 ? make_double2(1.0, 0.0) : zmul(scale, A[g + (size_t)c * lda]);
    double2 *vrow = Vp + (size_t)g * nbw, *wrow = Wp + (size_t)g * nbw;
    double2 zq[4] = {zero2d(), zero2d(), zero2d(), zero2d()};
    {
        int l = 0;
        for (; l + 4 <= j; l += 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u)
                zq[u] = zadd(zq[u], zadd(zmul(vrow[l + u], st->t1[l + u]), zmul(wrow[l + u], st->t2[l + u])));
        }
        for (; l < j; ++l) zq[0] = zadd(zq[0], zadd(zmul(vrow[l], st->t1[l]), zmul(wrow[l], st->t2[l])));
    }
    const double2 y = zsub(zadd(zadd(yq[0], yq[1]), zadd(yq[2], yq[3])), zadd(zadd(zq[0], zq[1]), zadd(zq[2], zq[3])));
    const double2 w = zadd(zmul(tau, y), zscale(alpha_s, v));
    wrow[j] = w;
    vrow[j] = v;
    if (i >= 1) A[g + (size_t)c * lda] = v;
}

// rows r0 .. n-1, columns 0 .. jb-1 of a row-major n x nbw buffer -> column-major (n - r0) x jb
__global__ void trd_to_colmajor_kernel(int n, int r0, int jb, const double2 *R, int nbw, double2 *C) {
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int l = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (r0 + i < n && l < jb) C[i + (size_t)l * (n - r0)] = R[(size_t)(r0 + i) * nbw + l];
}

__global__ void trd_zero_kernel(double2 *p, size_t cnt) {
    size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    for (; i < cnt; i += (size_t)gridDim.x * blockDim.x) p[i] = make_double2(0.0, 0.0);
}

int hemv_groups(int N) {
    const int nbk = cdiv(std::max(N, 1), 64);
    int t = 0;
    for (int J = 0; J < nbk; ++J) t += cdiv(nbk - J, TRD_K);
    return t;
}

}  // namespace

void hetrd_run(hgv_ctx_s *ctx, int n, int nb, double2 *A, int lda, double *d, double *e, double2 *T1, Arena &ar) {
    if (nb > TRD_NB || nb < 1) throw HipFail{hipErrorInvalidValue};
    const int nn = std::max(n, 1);
    const int nbk = cdiv(nn, 64), ldp = nbk * 64;
    const int nwa = cdiv(nn, 256);
    double2 *Vp = ar.take<double2>((size_t)nn * nb);
    double2 *Wp = ar.take<double2>((size_t)nn * nb);
    double2 *part = ar.take<double2>((size_t)nwa * (1 + 2 * nb));
    ColState *st = ar.take<ColState>(1);
    double2 *taup = ar.take<double2>(TRD_NB);
    double2 *P = ar.take<double2>((size_t)nbk * ldp);
    double2 *Qv = ar.take<double2>((size_t)hemv_groups(nn) * 64);
    double *Sv = ar.take<double>(hemv_groups(nn));
    double2 *Vc = ar.take<double2>((size_t)nn * nb);
    double2 *Wc = ar.take<double2>((size_t)nn * nb);
    double2 *Gm = ar.take<double2>((size_t)nb * nb);
    const size_t wsb = zgemm_splitk_bytes(n);
    void *ws = ar.take<char>(wsb);
    if (ar.measuring() || n == 0) return;
    const int np = cdiv(n, nb);
    hipLaunchKernelGGL(trd_zero_kernel, dim3((unsigned)std::min<size_t>(cdivz((size_t)np * nb * nb, 256), 4096)),
                       dim3(256), 0, ctx->stream, T1, (size_t)np * nb * nb);
    HGV_LAUNCH_CHECK();
    for (int k = 0; k < n; k += nb) {
        const int jb = std::min(nb, n - k);
        for (int j = 0; j < jb; ++j) {
            const int c = k + j, N = n - c - 1;
            const int nw = cdiv(n - c, 256);
            hipLaunchKernelGGL(trd_colupd_kernel, dim3(nw), dim3(256), 0, ctx->stream, n, c, j, A, lda, Vp, Wp, nb,
                               part);
            HGV_LAUNCH_CHECK();
            hipLaunchKernelGGL(trd_refl_kernel, dim3(1), dim3(256), 0, ctx->stream, n, c, j, nw, part, nb, A, lda, Vp,
                               Wp, d, e, taup, st);
            HGV_LAUNCH_CHECK();
            if (N == 0) continue;
            const int ng = hemv_groups(N);
            hipLaunchKernelGGL(trd_hemv_kernel, dim3(ng), dim3(256), 0, ctx->stream, N,
                               A + (c + 1) + (size_t)(c + 1) * lda, lda, A + (c + 1) + (size_t)c * lda, st, P, ldp,
                               Qv, Sv);
            HGV_LAUNCH_CHECK();
            hipLaunchKernelGGL(trd_wfin_kernel, dim3(cdiv(N, 256)), dim3(256), 0, ctx->stream, N, c, j, A, lda, st, P,
                               ldp, Qv, Sv, ng, Vp, Wp, nb);
            HGV_LAUNCH_CHECK();
        }
        // compact-WY factor of the panel's reflectors (rows k+1 .., column k + j from row k+1+j)
        const int Nr = n - k - 1, r = std::min(Nr, jb);
        if (r > 0)
            panel_t_build(ctx, Nr, r, A + (k + 1) + (size_t)k * lda, lda, taup, Vc, Gm,
                          T1 + (size_t)(k / nb) * nb * nb, nb, ws, wsb);
        // trailing update A22 -= V W^H + W V^H (lower)
        const int r0 = k + jb, N2 = n - r0;
        if (N2 > 0) {
            dim3 gt(cdiv(N2, 64), cdiv(jb, 4));
            hipLaunchKernelGGL(trd_to_colmajor_kernel, gt, dim3(256), 0, ctx->stream, n, r0, jb, Vp, nb, Vc);
            HGV_LAUNCH_CHECK();
            hipLaunchKernelGGL(trd_to_colmajor_kernel, gt, dim3(256), 0, ctx->stream, n, r0, jb, Wp, nb, Wc);
            HGV_LAUNCH_CHECK();
            ZGemm g;
            g.m = N2; g.n = N2; g.k = jb;
            g.opa = 'N'; g.A = Vc; g.lda = N2;
            g.opb = 'C'; g.B = Wc; g.ldb = N2;
            g.opa2 = 'N'; g.A2 = Wc; g.lda2 = N2;
            g.opb2 = 'C'; g.B2 = Vc; g.ldb2 = N2;
            g.alpha = make_double2(-1.0, 0.0); g.beta = make_double2(1.0, 0.0);
            g.C = A + r0 + (size_t)r0 * lda; g.ldc = lda;
            g.lower = 1;
            zgemm(ctx, g, static_cast<double2 *>(ws), wsb);
        }
    }
}

}  // namespace hgv
