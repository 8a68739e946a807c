// chol.hip -- Cholesky factorisation B = L L^H (Alg. 1 step 1), the
// triangular solves with L, and the reduction to standard form
// A' = L^-1 A L^-H (Alg. 1 step 2, the xHEGST operation the paper runs with
// its level-3 work on the accelerator).
//
// All three are recursive: an order-n problem splits at n1 (a multiple of 64
// near n/2) into two halves joined by large MFMA GEMMs (herk / her2k / hemm /
// gemm updates with K up to n/2), so nearly all flops run in gemm.hip.  The
// leaves are 64 x 64 diagonal blocks: Cholesky and the reduction to standard
// form of a block run in one workgroup out of LDS; the triangular-solve leaves
// multiply by the inverse of the 64 x 64 diagonal block of L (an MFMA GEMM in
// place, since one tile spans the 64-wide dimension).  The block inverses come
// from the Cholesky leaves, or from a batched inversion kernel when L is given.
#include "hgv_internal.h"

namespace hgv {

constexpr int LEAF = 64;

static int split_point(int n) {
    int n1 = ((n / 2 + LEAF - 1) / LEAF) * LEAF;
    if (n1 >= n) n1 = n - LEAF;
    if (n1 <= 0) n1 = n / 2;
    return n1;
}

// Inverse of the lower-triangular sz x sz block held in S (LDS) into Inv (LDS),
// NT threads: column c (independent of the others) solves L x = e_c by
// forward substitution; the QN = NT / 64 consecutive lanes of a column share
// it and split every inner product, combined with butterfly shuffles.  The
// diagonal of L is real (a Cholesky factor), so the division is a scaling.
template <int NT>
__device__ inline void tri_inverse_lds(double2 (*S)[LEAF + 1], double2 (*Inv)[LEAF + 1], int sz, int tid) {
    constexpr int QN = NT / 64;
    const int c = tid / QN, q = tid % QN;
    for (int i = 0; i < LEAF; ++i) {
        if (i < c || i >= sz || c >= sz) {
            Inv[i][c] = make_double2(0.0, 0.0);
            continue;
        }
        double2 s = make_double2(0.0, 0.0);
        for (int k = c + q; k < i; k += QN) s = zadd(s, zmul(S[i][k], Inv[k][c]));
        // sum over the column's QN = 16 lanes (one DPP row) by lane moves: xor 1,
        // xor 2, mirror within 8, mirror within 16
        static_assert(QN == 16, "one DPP row of lanes per column");
        s.x += dpp_f64<0xB1>(s.x);
        s.y += dpp_f64<0xB1>(s.y);
        s.x += dpp_f64<0x4E>(s.x);
        s.y += dpp_f64<0x4E>(s.y);
        s.x += dpp_f64<0x141>(s.x);
        s.y += dpp_f64<0x141>(s.y);
        s.x += dpp_f64<0x140>(s.x);
        s.y += dpp_f64<0x140>(s.y);
        const double2 rhs = (i == c) ? make_double2(1.0, 0.0) : make_double2(0.0, 0.0);
        // the butterfly leaves the same sum in the QN lanes, so each lane
        // stores the (identical) value and later reads only what it stored
        Inv[i][c] = zscale(1.0 / S[i][i].x, zsub(rhs, s));
    }
}

// ---- leaf Cholesky (n <= 64), one workgroup -----------------------------------
// Right-looking unblocked Cholesky of the lower triangle held in LDS, with the
// scaling of each column deferred to the end: step j subtracts
// S[i][j] conj(S[k][j]) / S[j][j] from the trailing elements (k > j, i >= k),
// which reads column j and writes only later columns, so a step needs one
// barrier; afterwards L[k][k] = sqrt(S[k][k]) and L[i][k] = S[i][k] / L[k][k].
// A non-positive (or NaN) pivot at local column j records info = base + j + 1
// (first failure wins) and stops the factorisation of this block (the columns
// before it are returned factored).  The inverse of the factor is written to
// Linv (64 x 64, column-major).  Each of the NT = 1024 threads owns four fixed
// elements.
template <int NT, class E>
__global__ __launch_bounds__(NT) void potf2_kernel(int n, E *A, int lda, int *info, int base, E *Linv) {
    constexpr int NE = LEAF * LEAF / NT;
    __shared__ double2 S[LEAF][LEAF + 1];
    __shared__ double2 Iv[LEAF][LEAF + 1];
    __shared__ double dk[LEAF];
    const int tid = threadIdx.x;
    for (int t = tid; t < LEAF * LEAF; t += NT) {
        int i = t % LEAF, j = t / LEAF;
        S[i][j] = (i < n && j < n && i >= j) ? El<E>::to(A[i + (size_t)j * lda]) : make_double2(0.0, 0.0);
    }
    __syncthreads();
    int jfail = n;
    for (int j = 0; j < n; ++j) {
        const double piv = S[j][j].x;   // the same value in every thread
        if (!(piv > 0.0)) {
            jfail = j;
            break;
        }
        const double ip = 1.0 / piv;
#pragma unroll
        for (int q = 0; q < NE; ++q) {
            const int e = tid + NT * q, i = e % LEAF, k = e / LEAF;
            if (k > j && i >= k && i < n) {
                const double2 a = S[i][j], b = S[k][j];
                S[i][k] = zsub(S[i][k], zscale(ip, make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y)));
            }
        }
        __syncthreads();
    }
    if (jfail < n && tid == 0 && info) atomicCAS(info, 0, base + jfail + 1);
    if (tid < jfail) dk[tid] = sqrt(S[tid][tid].x);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NE; ++q) {
        const int e = tid + NT * q, i = e % LEAF, k = e / LEAF;
        if (k < jfail && i >= k && i < n) S[i][k] = i == k ? make_double2(dk[k], 0.0) : zscale(1.0 / dk[k], S[i][k]);
    }
    __syncthreads();
    for (int t = tid; t < n * n; t += NT) {
        int i = t % n, j = t / n;
        if (i >= j) A[i + (size_t)j * lda] = El<E>::from(S[i][j]);
    }
    if (Linv) {
        if (jfail < n) {   // keep the solves finite; the result is flagged through info
            __syncthreads();
            for (int t = tid; t < LEAF * LEAF; t += NT) {
                int i = t % LEAF, j = t / LEAF;
                S[i][j] = (i == j) ? make_double2(1.0, 0.0) : make_double2(0.0, 0.0);
            }
            __syncthreads();
        }
        tri_inverse_lds<NT>(S, Iv, n, tid);
        __syncthreads();
        for (int t = tid; t < LEAF * LEAF; t += NT) Linv[t] = El<E>::from(Iv[t % LEAF][t / LEAF]);
    }
}

// Inverse of every 64 x 64 diagonal block of the lower-triangular L.
template <int NT, class E>
__global__ __launch_bounds__(NT) void trtri_diag_kernel(int n, const E *L, int ldl, E *Linv) {
    __shared__ double2 S[LEAF][LEAF + 1];
    __shared__ double2 Iv[LEAF][LEAF + 1];
    const int blk = blockIdx.x, tid = threadIdx.x;
    const int o = blk * LEAF, sz = min(LEAF, n - o);
    for (int t = tid; t < LEAF * LEAF; t += NT) {
        int i = t % LEAF, j = t / LEAF;
        S[i][j] = (i < sz && j < sz && i >= j) ? El<E>::to(L[(o + i) + (size_t)(o + j) * ldl]) : make_double2(0.0, 0.0);
    }
    __syncthreads();
    tri_inverse_lds<NT>(S, Iv, sz, tid);
    __syncthreads();
    E *out = Linv + (size_t)blk * LEAF * LEAF;
    for (int t = tid; t < LEAF * LEAF; t += NT) out[t] = El<E>::from(Iv[t % LEAF][t / LEAF]);
}

// ---- leaf reduction to standard form (n <= 64), one workgroup ---------------------
// C = L^-1 A L^-H for the block with the block's inverse Li = L^-1 (64 x 64,
// column-major, zero outside the n x n triangle): W = Li A (A full Hermitian
// from its lower triangle), C = W Li^H; the lower triangle of (C + C^H)/2 is
// written.  NT threads, each owning 4096 / NT elements of the product (NT =
// 1024: four waves per SIMD overlap the dependent multiply-add chains).
template <int NT, class E>
__global__ __launch_bounds__(NT) void hegs2_kernel(int n, E *A, int lda, const E *Li) {
    constexpr int CS = NT / 64, U = LEAF / CS;   // column stride and columns per thread
    __shared__ double2 Ls[LEAF][LEAF + 1];
    __shared__ double2 As[LEAF][LEAF + 1];
    const int tid = threadIdx.x;
    for (int t = tid; t < LEAF * LEAF; t += NT) {
        int i = t % LEAF, j = t / LEAF;
        Ls[i][j] = (i < n && j < n) ? El<E>::to(Li[i + (size_t)j * LEAF]) : make_double2(0.0, 0.0);
        double2 a = make_double2(0.0, 0.0);
        if (i < n && j < n) {
            if (i > j) a = El<E>::to(A[i + (size_t)j * lda]);
            else if (i == j) a = make_double2(El<E>::to(A[i + (size_t)i * lda]).x, 0.0);
            else a = zconj(El<E>::to(A[j + (size_t)i * lda]));
        }
        As[i][j] = a;
    }
    __syncthreads();
    // thread -> row r = tid % 64, columns c = tid / 64 + CS u (u = 0 .. U-1)
    const int r = tid & 63, c0 = tid >> 6;
    double2 acc[U];
    // W = Li A  (Li lower triangular: k <= r)
#pragma unroll
    for (int u = 0; u < U; ++u) acc[u] = make_double2(0.0, 0.0);
    for (int k = 0; k <= r && k < n; ++k) {
        const double2 l = Ls[r][k];
#pragma unroll
        for (int u = 0; u < U; ++u) zfma(acc[u], l, As[k][c0 + CS * u]);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < U; ++u) As[r][c0 + CS * u] = acc[u];
    __syncthreads();
    // C = W Li^H:  C[r][c] = sum_k W[r][k] conj(Li[c][k]),  k <= c
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int c = c0 + CS * u;
        double2 s2 = make_double2(0.0, 0.0);
        for (int k = 0; k <= c && k < n; ++k) zfma(s2, As[r][k], zconj(Ls[c][k]));
        acc[u] = s2;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < U; ++u) As[r][c0 + CS * u] = acc[u];
    __syncthreads();
    for (int t = tid; t < n * n; t += NT) {
        int i = t % n, j = t / n;
        if (i > j) A[i + (size_t)j * lda] = El<E>::from(zscale(0.5, zadd(As[i][j], zconj(As[j][i]))));
        else if (i == j) A[i + (size_t)i * lda] = El<E>::from(make_double2(As[i][i].x, 0.0));
    }
}

// ---- element-wise helpers in the storage type -----------------------------------------
// A[j, i] = conj(A[i, j]) for i > j (upper triangle made the mirror of the lower)
template <class E>
__global__ void fill_upper_t_kernel(int n, E *A, int lda) {
    int i = blockIdx.x * 16 + (threadIdx.x & 15);
    int j = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (i < n && j < n && i > j) A[j + (size_t)i * lda] = El<E>::from(zconj(El<E>::to(A[i + (size_t)j * lda])));
}
template <class E>
static void fill_upper_t(hgv_ctx_s *ctx, int n, E *A, int lda) {
    if (n <= 1) return;
    hipLaunchKernelGGL(fill_upper_t_kernel<E>, dim3(cdiv(n, 16), cdiv(n, 16)), dim3(256), 0, ctx->stream, n, A, lda);
    HGV_LAUNCH_CHECK();
}
// Y -= 1/2 X (m x n)
template <class E>
__global__ void add_half_t_kernel(int m, int n, const E *X, int ldx, E *Y, int ldy) {
    int i = blockIdx.x * 64 + (threadIdx.x & 63);
    int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i < m && j < n) {
        const double2 x = El<E>::to(X[i + (size_t)j * ldx]), y = El<E>::to(Y[i + (size_t)j * ldy]);
        Y[i + (size_t)j * ldy] = El<E>::from(make_double2(y.x - 0.5 * x.x, y.y - 0.5 * x.y));
    }
}
template <class E>
static void add_half_t(hgv_ctx_s *ctx, int m, int n, const E *X, int ldx, E *Y, int ldy) {
    if (m <= 0 || n <= 0) return;
    hipLaunchKernelGGL(add_half_t_kernel<E>, dim3(cdiv(m, 64), cdiv(n, 4)), dim3(256), 0, ctx->stream, m, n, X, ldx, Y,
                       ldy);
    HGV_LAUNCH_CHECK();
}

// ---- recursive drivers -----------------------------------------------------------------
// Linv: inverses of the 64 x 64 diagonal blocks of the current L (block k at
// Linv + k * 64 * 64); the recursion keeps every split at a multiple of 64.
template <class E>
struct TriCtx {
    hgv_ctx_s *ctx;
    void *ws;
    size_t wsb;
    E *zw = nullptr;          // hegst: L21 A'11 of the current split (n2 x n1, ld n2)
    void *ws_side = nullptr;  // hegst: split-K workspace of side stream 1 (null: no side streams)
    void *ws_side0 = nullptr; // hegst: split-K workspace of side stream 0
};

template <class E>
static const E *linv_at(const E *Linv, int off) { return Linv + (size_t)(off / LEAF) * LEAF * LEAF; }

// X (m x n, n <= 64) <- X L^-H = X (L^-1)^H   (in place: one column tile)
template <class E>
static void leaf_right_lc(const TriCtx<E> &t, int m, int n, const E *Li, E *X, int ldx) {
    typename El<E>::Gemm g;
    g.m = m; g.n = n; g.k = n;
    g.opa = 'N'; g.A = X; g.lda = ldx;
    g.opb = 'C'; g.B = Li; g.ldb = LEAF;
    g.C = X; g.ldc = ldx;
    g.allow_split = 0;
    gemm_any(t.ctx, g, t.ws, t.wsb);
}
// X (n x m, n <= 64) <- L^-1 X   (in place: one row tile)
template <class E>
static void leaf_left_ln(const TriCtx<E> &t, int n, int m, const E *Li, E *X, int ldx) {
    typename El<E>::Gemm g;
    g.m = n; g.n = m; g.k = n;
    g.opa = 'N'; g.A = Li; g.lda = LEAF;
    g.opb = 'N'; g.B = X; g.ldb = ldx;
    g.C = X; g.ldc = ldx;
    g.allow_split = 0;
    gemm_any(t.ctx, g, t.ws, t.wsb);
}
// X (n x m, n <= 64) <- L^-H X = (L^-1)^H X
template <class E>
static void leaf_left_lc(const TriCtx<E> &t, int n, int m, const E *Li, E *X, int ldx) {
    typename El<E>::Gemm g;
    g.m = n; g.n = m; g.k = n;
    g.opa = 'C'; g.A = Li; g.lda = LEAF;
    g.opb = 'N'; g.B = X; g.ldb = ldx;
    g.C = X; g.ldc = ldx;
    g.allow_split = 0;
    gemm_any(t.ctx, g, t.ws, t.wsb);
}

template <class E>
static void trsm_right_lc_rec(const TriCtx<E> &t, int m, int n, const E *L, int ldl, const E *Linv,
                              E *X, int ldx) {
    if (m <= 0 || n <= 0) return;
    if (n <= LEAF) {
        leaf_right_lc(t, m, n, Linv, X, ldx);
        return;
    }
    int n1 = split_point(n), n2 = n - n1;
    trsm_right_lc_rec(t, m, n1, L, ldl, Linv, X, ldx);
    typename El<E>::Gemm g;  // X2 -= X1 L21^H
    g.m = m; g.n = n2; g.k = n1;
    g.opa = 'N'; g.A = X; g.lda = ldx;
    g.opb = 'C'; g.B = L + n1; g.ldb = ldl;
    g.alpha = El<E>::mk(-1.0, 0.0); g.beta = El<E>::mk(1.0, 0.0);
    g.C = X + (size_t)n1 * ldx; g.ldc = ldx;
    gemm_any(t.ctx, g, t.ws, t.wsb);
    trsm_right_lc_rec(t, m, n2, L + n1 + (size_t)n1 * ldl, ldl, linv_at(Linv, n1), X + (size_t)n1 * ldx, ldx);
}

template <class E>
static void trsm_left_ln_rec(const TriCtx<E> &t, int n, int m, const E *L, int ldl, const E *Linv,
                             E *X, int ldx) {
    if (m <= 0 || n <= 0) return;
    if (n <= LEAF) {
        leaf_left_ln(t, n, m, Linv, X, ldx);
        return;
    }
    int n1 = split_point(n), n2 = n - n1;
    trsm_left_ln_rec(t, n1, m, L, ldl, Linv, X, ldx);
    typename El<E>::Gemm g;  // X2 -= L21 X1
    g.m = n2; g.n = m; g.k = n1;
    g.opa = 'N'; g.A = L + n1; g.lda = ldl;
    g.opb = 'N'; g.B = X; g.ldb = ldx;
    g.alpha = El<E>::mk(-1.0, 0.0); g.beta = El<E>::mk(1.0, 0.0);
    g.C = X + n1; g.ldc = ldx;
    gemm_any(t.ctx, g, t.ws, t.wsb);
    trsm_left_ln_rec(t, n2, m, L + n1 + (size_t)n1 * ldl, ldl, linv_at(Linv, n1), X + n1, ldx);
}

template <class E>
static void trsm_left_lc_rec(const TriCtx<E> &t, int n, int m, const E *L, int ldl, const E *Linv,
                             E *X, int ldx) {
    if (m <= 0 || n <= 0) return;
    if (n <= LEAF) {
        leaf_left_lc(t, n, m, Linv, X, ldx);
        return;
    }
    int n1 = split_point(n), n2 = n - n1;
    trsm_left_lc_rec(t, n2, m, L + n1 + (size_t)n1 * ldl, ldl, linv_at(Linv, n1), X + n1, ldx);
    typename El<E>::Gemm g;  // X1 -= L21^H X2
    g.m = n1; g.n = m; g.k = n2;
    g.opa = 'C'; g.A = L + n1; g.lda = ldl;
    g.opb = 'N'; g.B = X + n1; g.ldb = ldx;
    g.alpha = El<E>::mk(-1.0, 0.0); g.beta = El<E>::mk(1.0, 0.0);
    g.C = X; g.ldc = ldx;
    gemm_any(t.ctx, g, t.ws, t.wsb);
    trsm_left_lc_rec(t, n1, m, L, ldl, Linv, X, ldx);
}

// Scratch shared by the recursive stages: split-K partials and block inverses.
template <class E>
static TriCtx<E> tri_scratch(hgv_ctx_s *ctx, Arena &ar, int n, E **Linv) {
    TriCtx<E> t;
    t.ctx = ctx;
    t.wsb = zgemm_splitk_bytes(n);
    t.ws = ar.take<char>(t.wsb);
    *Linv = ar.take<E>((size_t)cdiv(std::max(n, 1), LEAF) * LEAF * LEAF);
    return t;
}

template <class E>
static void invert_diag_blocks(hgv_ctx_s *ctx, int n, const E *L, int ldl, E *Linv) {
    if (n <= 0) return;
    hipLaunchKernelGGL((trtri_diag_kernel<1024, E>), dim3(cdiv(n, LEAF)), dim3(1024), 0, ctx->stream, n, L, ldl, Linv);
    HGV_LAUNCH_CHECK();
}

template <class E>
void trsm_right_lc_t(hgv_ctx_s *ctx, int m, int n, const E *L, int ldl, E *X, int ldx, Arena &ar) {
    E *Linv;
    TriCtx<E> t = tri_scratch<E>(ctx, ar, n, &Linv);
    if (ar.measuring()) return;
    invert_diag_blocks(ctx, n, L, ldl, Linv);
    trsm_right_lc_rec(t, m, n, L, ldl, Linv, X, ldx);
}
template <class E>
void trsm_left_ln_t(hgv_ctx_s *ctx, int n, int m, const E *L, int ldl, E *X, int ldx, Arena &ar) {
    E *Linv;
    TriCtx<E> t = tri_scratch<E>(ctx, ar, n, &Linv);
    if (ar.measuring()) return;
    invert_diag_blocks(ctx, n, L, ldl, Linv);
    trsm_left_ln_rec(t, n, m, L, ldl, Linv, X, ldx);
}
template <class E>
void trsm_left_lc_t(hgv_ctx_s *ctx, int n, int m, const E *L, int ldl, E *X, int ldx, Arena &ar) {
    E *Linv;
    TriCtx<E> t = tri_scratch<E>(ctx, ar, n, &Linv);
    if (ar.measuring()) return;
    invert_diag_blocks(ctx, n, L, ldl, Linv);
    trsm_left_lc_rec(t, n, m, L, ldl, Linv, X, ldx);
}
template <class E>
void trsm_lh_t(hgv_ctx_s *ctx, int n, int m, const E *L, int ldl, E *X, int ldx, Arena &ar) {
    trsm_left_lc_t(ctx, n, m, L, ldl, X, ldx, ar);
}

template <class E>
static void potrf_rec(const TriCtx<E> &t, int n, E *A, int lda, int *info, int base, E *Linv) {
    if (n <= 0) return;
    if (n <= LEAF) {
        hipLaunchKernelGGL((potf2_kernel<1024, E>), dim3(1), dim3(1024), 0, t.ctx->stream, n, A, lda, info, base, Linv);
        HGV_LAUNCH_CHECK();
        return;
    }
    int n1 = split_point(n), n2 = n - n1;
    potrf_rec(t, n1, A, lda, info, base, Linv);
    trsm_right_lc_rec(t, n2, n1, A, lda, Linv, A + n1, lda);  // L21 = A21 L11^-H
    typename El<E>::Gemm g;  // A22 -= L21 L21^H (lower)
    g.m = n2; g.n = n2; g.k = n1;
    g.opa = 'N'; g.A = A + n1; g.lda = lda;
    g.opb = 'C'; g.B = A + n1; g.ldb = lda;
    g.alpha = El<E>::mk(-1.0, 0.0); g.beta = El<E>::mk(1.0, 0.0);
    g.C = A + n1 + (size_t)n1 * lda; g.ldc = lda;
    g.lower = 1;
    gemm_any(t.ctx, g, t.ws, t.wsb);
    potrf_rec(t, n2, A + n1 + (size_t)n1 * lda, lda, info, base + n1, const_cast<E *>(linv_at<E>(Linv, n1)));
}

template <class E>
void potrf_t(hgv_ctx_s *ctx, int n, E *B, int ldb, Arena &ar, int *d_info, int info_offset) {
    E *Linv;
    TriCtx<E> t = tri_scratch<E>(ctx, ar, n, &Linv);
    if (ar.measuring()) return;
    potrf_rec(t, n, B, ldb, d_info, info_offset, Linv);
}

template <class E>
static void hegst_split_rest(const TriCtx<E> &t, int n, int n1, E *A, int lda, const E *L, int ldl,
                             const E *Linv, bool spine);

// spine: the block is the trailing one of every enclosing split (its area is
// never read again by an enclosing level), so its A21 solve may run on the side
// stream with a single join at the end of the reduction
template <class E>
static void hegst_rec(const TriCtx<E> &t, int n, E *A, int lda, const E *L, int ldl, const E *Linv,
                      bool spine) {
    if (n <= 0) return;
    if (n <= LEAF) {
        hipLaunchKernelGGL((hegs2_kernel<1024, E>), dim3(1), dim3(1024), 0, t.ctx->stream, n, A, lda, Linv);
        HGV_LAUNCH_CHECK();
        return;
    }
    int n1 = split_point(n), n2 = n - n1;
    E *A11 = A, *A21 = A + n1;
    const E *L11 = L;
    if (t.ws_side && spine) {
        // A21 <- A21 L11^-H reads only the original A21 and L11: on side stream 0
        // while the (non-spine, so fork-free) reduction of A11 runs; joined
        // before A21 is next used
        hgv_ctx_s *c = t.ctx;
        hipStream_t main = c->stream;
        HGV_HIP(hipEventRecord(c->la_ev[0], main));
        HGV_HIP(hipStreamWaitEvent(c->la_stream[0], c->la_ev[0], 0));
        TriCtx<E> ts = t;
        ts.ws = t.ws_side0;
        c->stream = c->la_stream[0];
        try {
            trsm_right_lc_rec(ts, n2, n1, L11, ldl, Linv, A21, lda);
        } catch (...) {
            c->stream = main;
            throw;
        }
        c->stream = main;
        HGV_HIP(hipEventRecord(c->la_ev[1], c->la_stream[0]));
        hegst_rec(t, n1, A11, lda, L11, ldl, Linv, false);
        HGV_HIP(hipStreamWaitEvent(main, c->la_ev[1], 0));
    } else {
        hegst_rec(t, n1, A11, lda, L11, ldl, Linv, false);
        trsm_right_lc_rec(t, n2, n1, L11, ldl, Linv, A21, lda);  // A21 <- A21 L11^-H
    }
    hegst_split_rest(t, n, n1, A, lda, L, ldl, Linv, spine);
}

// The rest of a split once A'11 = L11^-1 A11 L11^-H and A21 L11^-H are in place:
// the two half-updates of A21 around the her2k of A22, the left solve of A21
// with L22, and the recursion into A22.
template <class E>
static void hegst_split_rest(const TriCtx<E> &t, int n, int n1, E *A, int lda, const E *L, int ldl,
                             const E *Linv, bool spine) {
    const int n2 = n - n1;
    E *A11 = A, *A21 = A + n1, *A22 = A + n1 + (size_t)n1 * lda;
    const E *L21 = L + n1, *L22 = L + n1 + (size_t)n1 * ldl;
    fill_upper_t<E>(t.ctx, n1, A11, lda);                   // A'11 as a full matrix
    typename El<E>::Gemm h;  // Z = L21 A'11, used for both half-updates of A21 (one product instead of two)
    h.m = n2; h.n = n1; h.k = n1;
    h.opa = 'N'; h.A = L21; h.lda = ldl;
    h.opb = 'N'; h.B = A11; h.ldb = lda;
    h.C = t.zw; h.ldc = n2;
    gemm_any(t.ctx, h, t.ws, t.wsb);
    add_half_t<E>(t.ctx, n2, n1, t.zw, n2, A21, lda);         // A21 -= 1/2 Z
    typename El<E>::Gemm r;  // A22 -= A21 L21^H + L21 A21^H (lower)
    r.m = n2; r.n = n2; r.k = n1;
    r.opa = 'N'; r.A = A21; r.lda = lda;
    r.opb = 'C'; r.B = L21; r.ldb = ldl;
    r.opa2 = 'N'; r.A2 = L21; r.lda2 = ldl;
    r.opb2 = 'C'; r.B2 = A21; r.ldb2 = lda;
    r.alpha = El<E>::mk(-1.0, 0.0); r.beta = El<E>::mk(1.0, 0.0);
    r.C = A22; r.ldc = lda;
    r.lower = 1;
    gemm_any(t.ctx, r, t.ws, t.wsb);
    add_half_t<E>(t.ctx, n2, n1, t.zw, n2, A21, lda);         // A21 -= 1/2 Z
    // A21 <- L22^-1 A21 needs nothing that the reduction of A22 produces; on the
    // spine nothing reads A21 again before the reduction ends, so with a side
    // stream it runs there (the spine's solves in order), overlapping the
    // recursion, and joins at the end
    if (t.ws_side && spine) {
        hgv_ctx_s *c = t.ctx;
        hipStream_t main = c->stream;
        HGV_HIP(hipEventRecord(c->la_ev[2], main));
        HGV_HIP(hipStreamWaitEvent(c->la_stream[1], c->la_ev[2], 0));
        TriCtx<E> ts = t;
        ts.ws = t.ws_side;
        c->stream = c->la_stream[1];
        try {
            trsm_left_ln_rec(ts, n2, n1, L22, ldl, linv_at(Linv, n1), A21, lda);
        } catch (...) {
            c->stream = main;
            throw;
        }
        c->stream = main;
    } else {
        trsm_left_ln_rec(t, n2, n1, L22, ldl, linv_at(Linv, n1), A21, lda);
    }
    hegst_rec(t, n2, A22, lda, L22, ldl, linv_at(Linv, n1), spine);
}

template <class E>
void hegst_t(hgv_ctx_s *ctx, int n, E *A, int lda, const E *L, int ldl, Arena &ar) {
    E *Linv;
    TriCtx<E> t = tri_scratch<E>(ctx, ar, n, &Linv);
    // every split of the recursion has n1 n2 <= (n / 2 + 64)^2
    const size_t zh = (size_t)std::max(n, 1) / 2 + LEAF;
    t.zw = ar.take<E>(zh * zh);
    void *wss = ar.take<char>(t.wsb);
    void *wss0 = ar.take<char>(t.wsb);
    if (ar.measuring()) return;
    invert_diag_blocks(ctx, n, L, ldl, Linv);
    const bool side = !ctx->concurrent && n > LEAF;
    if (side) {
        ensure_lookahead_stream(ctx);
        t.ws_side = wss;
        t.ws_side0 = wss0;
    }
    hegst_rec(t, n, A, lda, L, ldl, Linv, true);
    if (side) {   // join the left solves
        HGV_HIP(hipEventRecord(ctx->la_ev[3], ctx->la_stream[1]));
        HGV_HIP(hipStreamWaitEvent(ctx->stream, ctx->la_ev[3], 0));
    }
}

// B = L L^H followed by A' = L^-1 A L^-H, overlapped at the top split: the
// reduction of A11 and the solve A21 L11^-H need only L11 (and its block
// inverses, which the leaf Cholesky kernels write), so they run on side stream
// 0 while the main stream factors the trailing block of B; the rest of the
// reduction follows on the main stream as in hegst_run.  The stage timer (may
// be null) marks the end of the factorisation on the main stream.
template <class E>
void potrf_hegst_t(hgv_ctx_s *ctx, int n, E *B, int ldb, E *A, int lda, Arena &ar, int *d_info,
                     int info_offset, StageTimer *tm, double potrf_flops) {
    if (ctx->concurrent || n <= LEAF) {
        const size_t mk = ar.mark();
        potrf_t(ctx, n, B, ldb, ar, d_info, info_offset);
        ar.release(mk);
        if (tm && !ar.measuring()) {
            tm->end(HGV_ST_POTRF, potrf_flops);
            tm->begin(HGV_ST_HEGST);
        }
        hegst_t(ctx, n, A, lda, B, ldb, ar);
        return;
    }
    E *Linv;
    TriCtx<E> t = tri_scratch<E>(ctx, ar, n, &Linv);
    const size_t zh = (size_t)n / 2 + LEAF;
    t.zw = ar.take<E>(zh * zh);
    void *wss = ar.take<char>(t.wsb);
    void *wss0 = ar.take<char>(t.wsb);
    if (ar.measuring()) return;
    ensure_lookahead_stream(ctx);
    const int n1 = split_point(n), n2 = n - n1;
    E *B21 = B + n1, *B22 = B + n1 + (size_t)n1 * ldb;
    potrf_rec(t, n1, B, ldb, d_info, info_offset, Linv);   // L11 and its block inverses
    hipStream_t main = ctx->stream;
    HGV_HIP(hipEventRecord(ctx->la_ev[0], main));
    HGV_HIP(hipStreamWaitEvent(ctx->la_stream[0], ctx->la_ev[0], 0));
    TriCtx<E> ts = t;   // no forks inside: the A11 block is off the spine
    ts.ws = wss0;
    ctx->stream = ctx->la_stream[0];
    try {
        hegst_rec(ts, n1, A, lda, B, ldb, Linv, false);               // A'11
        trsm_right_lc_rec(ts, n2, n1, B, ldb, Linv, A + n1, lda);     // A21 <- A21 L11^-H
    } catch (...) {
        ctx->stream = main;
        throw;
    }
    ctx->stream = main;
    HGV_HIP(hipEventRecord(ctx->la_ev[1], ctx->la_stream[0]));
    // the rest of the factorisation (the top split of potrf_rec)
    trsm_right_lc_rec(t, n2, n1, B, ldb, Linv, B21, ldb);   // L21 = B21 L11^-H
    typename El<E>::Gemm g;  // B22 -= L21 L21^H (lower)
    g.m = n2; g.n = n2; g.k = n1;
    g.opa = 'N'; g.A = B21; g.lda = ldb;
    g.opb = 'C'; g.B = B21; g.ldb = ldb;
    g.alpha = El<E>::mk(-1.0, 0.0); g.beta = El<E>::mk(1.0, 0.0);
    g.C = B22; g.ldc = ldb;
    g.lower = 1;
    gemm_any(ctx, g, t.ws, t.wsb);
    potrf_rec(t, n2, B22, ldb, d_info, info_offset + n1, Linv + (size_t)(n1 / LEAF) * LEAF * LEAF);
    if (tm) {
        tm->end(HGV_ST_POTRF, potrf_flops);
        tm->begin(HGV_ST_HEGST);
    }
    HGV_HIP(hipStreamWaitEvent(main, ctx->la_ev[1], 0));
    t.ws_side = wss;
    t.ws_side0 = wss0;
    hegst_split_rest(t, n, n1, A, lda, B, ldb, Linv, true);
    HGV_HIP(hipEventRecord(ctx->la_ev[3], ctx->la_stream[1]));   // join the left solves
    HGV_HIP(hipStreamWaitEvent(main, ctx->la_ev[3], 0));
}

// ---- entry points of the complex-double path and the complex-float instantiations ----------
void trsm_right_lc(hgv_ctx_s *ctx, int m, int n, const double2 *L, int ldl, double2 *X, int ldx, Arena &ar) {
    trsm_right_lc_t<double2>(ctx, m, n, L, ldl, X, ldx, ar);
}
void trsm_left_ln(hgv_ctx_s *ctx, int n, int m, const double2 *L, int ldl, double2 *X, int ldx, Arena &ar) {
    trsm_left_ln_t<double2>(ctx, n, m, L, ldl, X, ldx, ar);
}
void trsm_left_lc(hgv_ctx_s *ctx, int n, int m, const double2 *L, int ldl, double2 *X, int ldx, Arena &ar) {
    trsm_left_lc_t<double2>(ctx, n, m, L, ldl, X, ldx, ar);
}
void trsm_lh_run(hgv_ctx_s *ctx, int n, int m, const double2 *L, int ldl, double2 *X, int ldx, Arena &ar) {
    trsm_lh_t<double2>(ctx, n, m, L, ldl, X, ldx, ar);
}
void potrf_run(hgv_ctx_s *ctx, int n, double2 *B, int ldb, Arena &ar, int *d_info, int info_offset) {
    potrf_t<double2>(ctx, n, B, ldb, ar, d_info, info_offset);
}
void hegst_run(hgv_ctx_s *ctx, int n, double2 *A, int lda, const double2 *L, int ldl, Arena &ar) {
    hegst_t<double2>(ctx, n, A, lda, L, ldl, ar);
}
void potrf_hegst_run(hgv_ctx_s *ctx, int n, double2 *B, int ldb, double2 *A, int lda, Arena &ar, int *d_info,
                     int info_offset, StageTimer *tm, double potrf_flops) {
    potrf_hegst_t<double2>(ctx, n, B, ldb, A, lda, ar, d_info, info_offset, tm, potrf_flops);
}
template void trsm_lh_t<float2>(hgv_ctx_s *, int, int, const float2 *, int, float2 *, int, Arena &);
template void potrf_hegst_t<float2>(hgv_ctx_s *, int, float2 *, int, float2 *, int, Arena &, int *, int,
                                    StageTimer *, double);

}  // namespace hgv
