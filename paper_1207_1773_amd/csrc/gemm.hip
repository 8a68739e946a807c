// gemm.hip -- MFMA matrix-multiply tiles for gfx950.
//
// Every level-3 operation of the solver (the herk/her2k/hemm/trsm updates of
// the Cholesky and reduction to standard form, the two-sided trailing update
// of the band reduction, the block-reflector back-transformations, the
// divide-and-conquer eigenvector merges) is issued as one of these GEMMs.
//
// Design (CDNA4):
//  * workgroup = 4 wave64s arranged 2 x 2; each wave owns a (BM/2) x (BN/2)
//    sub-tile made of 16x16 MFMA blocks; registers are capped so that two
//    workgroups share a CU (two waves per SIMD hide LDS and MFMA latency);
//  * complex double: three real v_mfma_f64_16x16x4f64 per 16x16x4 complex
//    block (the 3M form: re*re, im*im and (re+im)*(re+im) accumulated
//    separately, combined in the epilogue); real double: one; complex float:
//    three v_mfma_f32_16x16x4f32 with fp32 accumulation;
//  * A and B tiles of depth 16 are staged through LDS (interleaved complex,
//    one padding element per row against bank conflicts) with the next
//    tile's global loads issued before the current tile's MFMAs;
//  * the block index is remapped so that consecutive tiles land on the same
//    XCD (workgroups are dealt round-robin over the 8 XCDs) and tiles are
//    walked in column groups of 8 row-tiles so one XCD's L2 sees the same
//    operand panels;
//  * split-K (deterministic: partial tiles summed in a fixed order by a
//    second kernel) for outputs with too few tiles to fill 256 CUs.
#include <type_traits>

#include <hip/hip_ext.h>

#include "hgv_internal.h"

namespace hgv {

// ---- device code of the tile kernel (begin) ----

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// ---- element traits -----------------------------------------------------------
struct TZ {  // complex double
    typedef double2 E;
    typedef v4d Acc;
    typedef double S;
    static constexpr bool cplx = true;
    __device__ static E zero() { return make_double2(0.0, 0.0); }
    __device__ static E conj(E a) { return make_double2(a.x, -a.y); }
    __device__ static E realpart(E a) { return make_double2(a.x, 0.0); }
    __device__ static Acc mfma(S a, S b, Acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    // output layout of v_mfma_f64_16x16x4f64: lane l, register r -> row l/16 + 4r, column l%16
    __device__ static int out_row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
struct TD {  // real double
    typedef double E;
    typedef v4d Acc;
    typedef double S;
    static constexpr bool cplx = false;
    __device__ static E zero() { return 0.0; }
    __device__ static E conj(E a) { return a; }
    __device__ static E realpart(E a) { return a; }
    __device__ static Acc mfma(S a, S b, Acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static int out_row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
struct TC {  // complex float
    typedef float2 E;
    typedef v4f Acc;
    typedef float S;
    static constexpr bool cplx = true;
    __device__ static E zero() { return make_float2(0.0f, 0.0f); }
    __device__ static E conj(E a) { return make_float2(a.x, -a.y); }
    __device__ static E realpart(E a) { return make_float2(a.x, 0.0f); }
    __device__ static Acc mfma(S a, S b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    // output layout of v_mfma_f32_16x16x4f32: lane l, register r -> row 4(l/16) + r, column l%16
    __device__ static int out_row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

template <class T>
struct GemmDev {
    typedef typename T::E E;
    int m, n, k;
    const E *A; int lda; int opa;
    const E *B; int ldb; int opb;
    const E *A2; int lda2; int opa2;
    const E *B2; int ldb2; int opb2;
    int nseg;
    E alpha, beta;
    int beta_zero;
    E *C; int ldc;
    int lower;
    int splits;        // split-K factor (gridDim.y)
    int lower_tiles;   // grid enumerates only the tiles on or below the diagonal
    E *P;              // partial tiles when splits > 1: splits x (m x n), ld m
    int tiles_m, tiles_n;
    const int *gate;   // non-null: run only if *gate == gate_val
    int gate_val;
};

// Tile shape per element type: output BM x BN per workgroup, k depth of a
// staged tile, waves per workgroup (2 x NW/2, each owning BM/2 x 2BN/NW).  The
// complex tiles use 4 waves and depth 16 (two workgroups per CU); the real
// 128 x 128 tile uses 8 waves, so that each thread holds half the accumulators
// and half the prefetched operands and a depth of 32 fits in registers: its
// chunk of MFMAs then covers the latency of the next chunk's loads.
template <class T>
struct Shape {
    static constexpr int BM = 64, BN = 64, BK = 16, NW = 4;
};
template <>
struct Shape<TD> {
    static constexpr int BM = 128, BN = 128, BK = 32, NW = 8;
};
template <class T>
struct KDepth {
    static constexpr int v = Shape<T>::BK;
};
constexpr int PAD = 1;


__device__ inline int remap_xcd(int bid, int total) {
    int full = (total / 8) * 8;
    if (bid < full) return (bid % 8) * (total / 8) + bid / 8;
    return bid;
}

// Fix-ups of a loaded element, applied when it is stored to LDS: bit 0 in
// range (else zero), bit 1 conjugate, bit 2 real part only (the diagonal of a
// Hermitian operand).  Keeping them as flag bits leaves the loads themselves
// unconditional (clamped to an in-range address), so that a thread's loads of a
// tile are all in flight together and none waits for the previous one.
template <class T>
__device__ inline typename T::E fix_elem(typename T::E v, unsigned f);
template <>
__device__ inline double2 fix_elem<TZ>(double2 v, unsigned f) {
    const bool in = f & 1u, cj = f & 2u, re = f & 4u;
    return make_double2(in ? v.x : 0.0, (in && !re) ? (cj ? -v.y : v.y) : 0.0);
}
template <>
__device__ inline float2 fix_elem<TC>(float2 v, unsigned f) {
    const bool in = f & 1u, cj = f & 2u, re = f & 4u;
    return make_float2(in ? v.x : 0.0f, (in && !re) ? (cj ? -v.y : v.y) : 0.0f);
}
template <>
__device__ inline double fix_elem<TD>(double v, unsigned f) { return (f & 1u) ? v : 0.0; }

// Load the BM x BK tile of op(A) (rows m0.., cols k0..) into registers.  The
// LDS slot of element t is ibase + t * istep (the element-to-slot map is
// affine in t for both access orders); fl receives the fix-up bits (3 per
// element, at most 21 elements).  op: 0 N, 1 T, 2 C, 3 H (Hermitian, lower
// triangle stored).
template <class T, int BM, int NT>
__device__ inline void load_a(const typename T::E *__restrict__ A, int lda, int op, int M, int K,
                              int m0, int k0, int tid, typename T::E (&r)[BM * KDepth<T>::v / NT],
                              int &ibase, int &istep, unsigned long long &fl) {
    constexpr int BK = KDepth<T>::v;
    constexpr int NE = BM * BK / NT;
    const bool mirrored = (op == 1 || op == 2) || (op == 3 && m0 + BM - 1 < k0);
    fl = 0;
    if (!mirrored) {
        const bool herm = op == 3;
        const size_t safe = m0 + (size_t)k0 * lda;
        ibase = (tid / BM) * (BM + PAD) + tid % BM;
        istep = (NT / BM) * (BM + PAD);
#pragma unroll
        for (int t = 0; t < NE; ++t) {
            const int e = tid + t * NT;
            const int mm = e % BM, kk = e / BM;
            const int gm = m0 + mm, gk = k0 + kk;
            const bool in = gm < M && gk < K;
            const bool up = herm && gm < gk;   // above the diagonal: the mirrored element, conjugated
            const size_t off = up ? gk + (size_t)gm * lda : gm + (size_t)gk * lda;
            r[t] = A[in ? off : safe];
            fl |= (unsigned long long)((in ? 1u : 0u) | (up ? 2u : 0u) | ((herm && gm == gk) ? 4u : 0u)) << (3 * t);
        }
    } else {
        const unsigned cj = (op == 2 || op == 3) ? 2u : 0u;
        const size_t safe = k0 + (size_t)m0 * lda;
        ibase = (tid % BK) * (BM + PAD) + tid / BK;
        istep = NT / BK;
#pragma unroll
        for (int t = 0; t < NE; ++t) {
            const int e = tid + t * NT;
            const int kk = e % BK, mm = e / BK;
            const int gm = m0 + mm, gk = k0 + kk;
            const bool in = gm < M && gk < K;
            r[t] = A[in ? gk + (size_t)gm * lda : safe];
            fl |= (unsigned long long)((in ? 1u : 0u) | cj) << (3 * t);
        }
    }
}

// Load the BK x BN tile of op(B) (rows k0.., cols n0..).  op: 0 N, 1 T, 2 C.
template <class T, int BN, int NT>
__device__ inline void load_b(const typename T::E *__restrict__ B, int ldb, int op, int K, int N,
                              int k0, int n0, int tid, typename T::E (&r)[BN * KDepth<T>::v / NT],
                              int &ibase, int &istep, unsigned long long &fl) {
    constexpr int BK = KDepth<T>::v;
    constexpr int NE = BN * BK / NT;
    fl = 0;
    if (op == 0) {
        const size_t safe = k0 + (size_t)n0 * ldb;
        ibase = (tid % BK) * (BN + PAD) + tid / BK;
        istep = NT / BK;
#pragma unroll
        for (int t = 0; t < NE; ++t) {
            const int e = tid + t * NT;
            const int kk = e % BK, nn = e / BK;
            const int gk = k0 + kk, gn = n0 + nn;
            const bool in = gk < K && gn < N;
            r[t] = B[in ? gk + (size_t)gn * ldb : safe];
            fl |= (unsigned long long)(in ? 1u : 0u) << (3 * t);
        }
    } else {
        const unsigned cj = (op == 2) ? 2u : 0u;
        const size_t safe = n0 + (size_t)k0 * ldb;
        ibase = (tid / BN) * (BN + PAD) + tid % BN;
        istep = (NT / BN) * (BN + PAD);
#pragma unroll
        for (int t = 0; t < NE; ++t) {
            const int e = tid + t * NT;
            const int nn = e % BN, kk = e / BN;
            const int gk = k0 + kk, gn = n0 + nn;
            const bool in = gk < K && gn < N;
            r[t] = B[in ? gn + (size_t)gk * ldb : safe];
            fl |= (unsigned long long)((in ? 1u : 0u) | cj) << (3 * t);
        }
    }
}

// One 16x16x4 block product.  Complex types use three real products per
// block (the 3M form):  P1 += Ar Br,  P2 += Ai Bi,  P3 += (Ar + Ai)(Br + Bi),
// re = P1 - P2,  im = P3 - P1 - P2  (normwise the same error bound as the
// four-product form up to a small constant; componentwise the imaginary part
// is relative to (|Ar| + |Ai|)(|Br| + |Bi|)).
template <class T>
__device__ inline void mfma_step(typename T::E a, typename T::E b, typename T::Acc &p1, typename T::Acc &p2,
                                 typename T::Acc &p3);

template <>
__device__ inline void mfma_step<TZ>(double2 a, double2 b, v4d &p1, v4d &p2, v4d &p3) {
    p1 = TZ::mfma(a.x, b.x, p1);
    p2 = TZ::mfma(a.y, b.y, p2);
    p3 = TZ::mfma(a.x + a.y, b.x + b.y, p3);
}
template <>
__device__ inline void mfma_step<TC>(float2 a, float2 b, v4f &p1, v4f &p2, v4f &p3) {
    p1 = TC::mfma(a.x, b.x, p1);
    p2 = TC::mfma(a.y, b.y, p2);
    p3 = TC::mfma(a.x + a.y, b.x + b.y, p3);
}
template <>
__device__ inline void mfma_step<TD>(double a, double b, v4d &p1, v4d &p2, v4d &p3) {
    (void)p2;
    (void)p3;
    p1 = TD::mfma(a, b, p1);
}

template <class T>
__device__ inline typename T::E make_e(typename T::S re, typename T::S im);
template <>
__device__ inline double2 make_e<TZ>(double re, double im) { return make_double2(re, im); }
template <>
__device__ inline float2 make_e<TC>(float re, float im) { return make_float2(re, im); }
template <>
__device__ inline double make_e<TD>(double re, double im) { (void)im; return re; }

__device__ inline double2 e_mul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline float2 e_mul(float2 a, float2 b) { return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline double e_mul(double a, double b) { return a * b; }
__device__ inline double2 e_add(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline float2 e_add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ inline double e_add(double a, double b) { return a + b; }

template <class T, int BM, int BN, int NW>
__global__ __launch_bounds__(NW * 64, 2) void gemm_kernel(GemmDev<T> g) {
    typedef typename T::E E;
    typedef typename T::Acc Acc;
    constexpr int NT = NW * 64;
    constexpr int WM = BM / 2, WN = BN / (NW / 2);
    constexpr int FM = WM / 16, FN = WN / 16;
    constexpr int BK = KDepth<T>::v;
    constexpr int NA = BM * BK / NT, NB = BN * BK / NT;
    __shared__ E As[2][BK * (BM + PAD)];
    __shared__ E Bs[2][BK * (BN + PAD)];

    if (g.gate && *g.gate != g.gate_val) return;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;

    // tile selection: XCD-aware remap (each XCD takes a contiguous range of
    // tile ids), then either column groups of 8 row tiles, or, for outputs
    // restricted to the lower triangle with square tiles, the lower tiles
    // only, numbered row by row (so every XCD gets the same number of tiles
    // and consecutive tiles share their row panel of A)
    int tm, tn;
    if (g.lower_tiles) {
        const int total = (int)gridDim.x;
        const int id = remap_xcd(blockIdx.x, total);
        const int K = min(g.tiles_m, g.tiles_n);
        const int T0 = K * (K + 1) / 2;
        if (id < T0) {
            int r = (int)((sqrt(8.0 * id + 1.0) - 1.0) * 0.5);
            while (r > 0 && r * (r + 1) / 2 > id) --r;
            while ((r + 1) * (r + 2) / 2 <= id) ++r;
            tm = r;
            tn = id - r * (r + 1) / 2;
        } else {
            const int q = id - T0;
            tm = K + q / g.tiles_n;
            tn = q % g.tiles_n;
        }
    } else {
        const int total = g.tiles_m * g.tiles_n;
        int id = remap_xcd(blockIdx.x, total);
        constexpr int GROUP = 8;
        int per_group = GROUP * g.tiles_n;
        int grp = id / per_group;
        int first_m = grp * GROUP;
        int gm_cnt = min(g.tiles_m - first_m, GROUP);
        int within = id % per_group;
        tm = first_m + within % gm_cnt;
        tn = within / gm_cnt;
    }
    const int m0 = tm * BM, n0 = tn * BN;
    if (g.lower && m0 + BM - 1 < n0) return;  // tile entirely above the diagonal

    // K range of this split (chunks of BK over the concatenated segments)
    const int cps = (g.k + BK - 1) / BK;  // chunks per segment
    const int nchunks = cps * g.nseg;
    const int z = blockIdx.y;
    const int per = (nchunks + g.splits - 1) / g.splits;
    const int c_beg = z * per;
    const int c_end = min(nchunks, c_beg + per);

    // P2 and P3 of the 3M form only for the complex types
    constexpr int FMI = T::cplx ? FM : 1, FNI = T::cplx ? FN : 1;
    Acc acc1[FM][FN], acc2[FMI][FNI], acc3[FMI][FNI];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc1[i][j] = Acc{0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < FMI; ++i)
#pragma unroll
        for (int j = 0; j < FNI; ++j) {
            acc2[i][j] = Acc{0, 0, 0, 0};
            acc3[i][j] = Acc{0, 0, 0, 0};
        }

    E ra[NA], rb[NB];
    int iab = 0, ias = 0, ibb = 0, ibs = 0;
    unsigned long long fa = 0, fb = 0;
    auto fetch = [&](int c) {
        int seg = c / cps;
        int k0 = (c % cps) * BK;
        if (seg == 0) {
            load_a<T, BM, NT>(g.A, g.lda, g.opa, g.m, g.k, m0, k0, tid, ra, iab, ias, fa);
            load_b<T, BN, NT>(g.B, g.ldb, g.opb, g.k, g.n, k0, n0, tid, rb, ibb, ibs, fb);
        } else {
            load_a<T, BM, NT>(g.A2, g.lda2, g.opa2, g.m, g.k, m0, k0, tid, ra, iab, ias, fa);
            load_b<T, BN, NT>(g.B2, g.ldb2, g.opb2, g.k, g.n, k0, n0, tid, rb, ibb, ibs, fb);
        }
    };

    auto stage = [&](int buf) {
#pragma unroll
        for (int t = 0; t < NA; ++t) As[buf][iab + t * ias] = fix_elem<T>(ra[t], (unsigned)(fa >> (3 * t)) & 7u);
#pragma unroll
        for (int t = 0; t < NB; ++t) Bs[buf][ibb + t * ibs] = fix_elem<T>(rb[t], (unsigned)(fb >> (3 * t)) & 7u);
    };
    auto compute = [&](int buf) {
#pragma unroll
        for (int ks = 0; ks < BK / 4; ++ks) {
            const int kl = ks * 4 + (lane >> 4);
            E af[FM], bf[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i) af[i] = As[buf][kl * (BM + PAD) + wm * WM + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < FN; ++j) bf[j] = Bs[buf][kl * (BN + PAD) + wn * WN + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    mfma_step<T>(af[i], bf[j], acc1[i][j], acc2[T::cplx ? i : 0][T::cplx ? j : 0],
                                 acc3[T::cplx ? i : 0][T::cplx ? j : 0]);
        }
    };
    // two LDS buffers, one barrier per chunk: the next chunk's global loads are
    // issued before this chunk's MFMAs and stored to the other buffer after them
    // (that buffer was last read before the previous barrier)
    if (c_beg < c_end) {
        fetch(c_beg);
        stage(0);
    }
    __syncthreads();
    for (int c = c_beg; c < c_end; ++c) {
        const int buf = (c - c_beg) & 1;
        if (c + 1 < c_end) fetch(c + 1);
        compute(buf);
        if (c + 1 < c_end) stage(buf ^ 1);
        __syncthreads();
    }

    // epilogue: each lane holds four rows (T::out_row) of column lane%16 of each
    // block; for beta != 0 the C elements of one block row are loaded together
    // (clamped addresses) before any of them is used
    const bool need_c = g.splits == 1 && !g.beta_zero;
#pragma unroll
    for (int i = 0; i < FM; ++i) {
        E cv[FN][4];
        if (need_c) {
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = m0 + wm * WM + i * 16 + T::out_row(lane, r);
                    const int col = n0 + wn * WN + j * 16 + (lane & 15);
                    const bool in = row < g.m && col < g.n;
                    cv[j][r] = g.C[in ? row + (size_t)col * g.ldc : m0 + (size_t)n0 * g.ldc];
                }
        }
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int row = m0 + wm * WM + i * 16 + T::out_row(lane, r);
                int col = n0 + wn * WN + j * 16 + (lane & 15);
                if (row >= g.m || col >= g.n) continue;
                if (g.lower && row < col) continue;
                const typename T::S p1 = acc1[i][j][r];
                const typename T::S p2 = acc2[T::cplx ? i : 0][T::cplx ? j : 0][r];
                const typename T::S p3 = acc3[T::cplx ? i : 0][T::cplx ? j : 0][r];
                E v = make_e<T>(p1 - p2, p3 - p1 - p2);
                if (g.splits > 1) {
                    g.P[(size_t)z * g.m * g.n + row + (size_t)col * g.m] = v;
                } else {
                    E o = e_mul(g.alpha, v);
                    if (need_c) o = e_add(o, e_mul(g.beta, cv[j][r]));
                    g.C[row + (size_t)col * g.ldc] = o;
                }
            }
    }
}

// ---- device code of the tile kernel (end) ----

// C = alpha * sum_z P[z] + beta * C  (fixed summation order)
template <class T>
__global__ __launch_bounds__(256) void splitk_reduce(GemmDev<T> g) {
    typedef typename T::E E;
    if (g.gate && *g.gate != g.gate_val) return;
    size_t total = (size_t)g.m * g.n;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
        int row = (int)(t % g.m), col = (int)(t / g.m);
        if (g.lower && row < col) continue;
        E s = g.P[t];
        // the same order of summation; the unrolling lets 8 of the loads be in flight
#pragma unroll 8
        for (int z = 1; z < g.splits; ++z) s = e_add(s, g.P[(size_t)z * total + t]);
        E o = e_mul(g.alpha, s);
        if (!g.beta_zero) o = e_add(o, e_mul(g.beta, g.C[row + (size_t)col * g.ldc]));
        g.C[row + (size_t)col * g.ldc] = o;
    }
}

static int op_code(char op) {
    switch (op) {
        case 'N': case 'n': return 0;
        case 'T': case 't': return 1;
        case 'C': case 'c': return 2;
        case 'H': case 'h': return 3;
    }
    return -1;
}

// Choose tile shape and split-K factor, then launch.  `ws` (bytes) holds the
// partial tiles of split-K; when it is too small the split factor is reduced.
template <class T, class G>
static void gemm_launch(hgv_ctx_s *ctx, const G &a, typename T::E *ws, size_t ws_bytes,
                        double flops) {
    typedef typename T::E E;
    if (a.m <= 0 || a.n <= 0) return;
    GemmDev<T> g;
    g.m = a.m; g.n = a.n; g.k = a.k;
    g.A = a.A; g.lda = a.lda; g.opa = op_code(a.opa);
    g.B = a.B; g.ldb = a.ldb; g.opb = op_code(a.opb);
    g.A2 = a.A2; g.lda2 = a.lda2; g.opa2 = op_code(a.opa2);
    g.B2 = a.B2; g.ldb2 = a.ldb2; g.opb2 = op_code(a.opb2);
    g.nseg = (a.A2 && a.B2) ? 2 : 1;
    g.alpha = a.alpha; g.beta = a.beta;
    g.C = a.C; g.ldc = a.ldc;
    g.lower = a.lower;
    g.gate = a.gate;
    g.gate_val = a.gate_val;
    g.P = nullptr;
    {
        const char *pb = reinterpret_cast<const char *>(&a.beta);
        bool z = true;
        for (size_t i = 0; i < sizeof(a.beta); ++i) z = z && pb[i] == 0;
        g.beta_zero = z ? 1 : 0;
    }
    if (a.k <= 0) {
        // C = beta C only (alpha * empty sum); realised as a split-free launch
        // with no chunks.
    }
    // tile shape: 64x64 (4 waves of 32x32) for the complex types; 128x128 for
    // real (one MFMA per 16x16x4 block, so the larger tile keeps the operand
    // bytes per flop as low as the complex tile's)
    constexpr int BM = Shape<T>::BM, BN = Shape<T>::BN, NW = Shape<T>::NW;
    // small complex-double products (fewer than 128 tiles of 64 x 64, K <= 512): a
    // one-tile product's 768 MFMAs per 16 of K run on one CU, so the output is cut
    // into 32 x 32 tiles instead, spreading the same MFMAs over four times the
    // CUs (each output element keeps its order of summation).  A product computed
    // in place keeps one tile across the aliased operand's other dimension:
    // 32 x 64 when C is A (n <= 64), 64 x 32 when C is B (m <= 64), so that no
    // workgroup writes rows or columns another one still reads; any other overlap
    // of C with an operand keeps the 64 x 64 tiles.
    int bm = BM, bn = BN;
    if constexpr (std::is_same<T, TZ>::value) {
        if (cdiv(a.m, 64) * cdiv(a.n, 64) < 128 && a.k <= 512) {
            const char *c0 = reinterpret_cast<const char *>(a.C);
            const char *c1 = c0 + ((size_t)a.ldc * (a.n - 1) + a.m) * sizeof(E);
            // the bytes an operand spans (rows x cols stored, leading dimension ld)
            auto overlaps = [&](const void *p, int ld, int rows, int cols) {
                if (!p || rows <= 0 || cols <= 0) return false;
                const char *p0 = static_cast<const char *>(p);
                const char *p1 = p0 + ((size_t)ld * (cols - 1) + rows) * sizeof(E);
                return p0 < c1 && c0 < p1;
            };
            const bool ta = a.opa != 'N' && a.opa != 'n', tb = a.opb != 'N' && a.opb != 'n';
            const bool ta2 = a.opa2 != 'N' && a.opa2 != 'n', tb2 = a.opb2 != 'N' && a.opb2 != 'n';
            const bool seg2 = a.A2 && a.B2;
            const bool ovA = overlaps(a.A, a.lda, ta ? a.k : a.m, ta ? a.m : a.k);
            const bool ovB = overlaps(a.B, a.ldb, tb ? a.n : a.k, tb ? a.k : a.n);
            const bool ov2 = seg2 && (overlaps(a.A2, a.lda2, ta2 ? a.k : a.m, ta2 ? a.m : a.k) ||
                                      overlaps(a.B2, a.ldb2, tb2 ? a.n : a.k, tb2 ? a.k : a.n));
            const bool sameA = static_cast<const void *>(a.C) == static_cast<const void *>(a.A) && !ta &&
                               a.lda == a.ldc;
            const bool sameB = static_cast<const void *>(a.C) == static_cast<const void *>(a.B) && !tb &&
                               a.ldb == a.ldc;
            if (!ovA && !ovB && !ov2) {
                bm = 32; bn = 32;
            } else if (sameA && !ovB && !ov2 && a.n <= 64) {
                bm = 32; bn = 64;
            } else if (sameB && !ovA && !ov2 && a.m <= 64) {
                bm = 64; bn = 32;
            }
        }
    }
    const bool small = bm != BM || bn != BN;
    g.tiles_m = cdiv(a.m, bm);
    g.tiles_n = cdiv(a.n, bn);
    int tiles = g.tiles_m * g.tiles_n;
    g.lower_tiles = 0;
    if (a.lower && bm == bn) {
        // lower tiles of row tile tm: tn = 0 .. min(tm, tiles_n - 1)
        const int K = std::min(g.tiles_m, g.tiles_n);
        tiles = K * (K + 1) / 2 + (g.tiles_m - K) * g.tiles_n;
        g.lower_tiles = 1;
    }
    int chunks = cdiv(std::max(a.k, 0), KDepth<T>::v) * g.nseg;
    int splits = 1;
    // fewer tiles than resident workgroups and a long K: split the K loop into the
    // number of parts that takes the fewest chunk steps on the critical path, the
    // waves of resident workgroups times the chunks per part, plus the reduction
    // (its launch, about two chunk steps, and its traffic, the parts written and
    // read back at ~4 TB/s against ~2.5 us per chunk step); every part keeps at
    // least 4 chunks
    const int ti = std::is_same<T, TZ>::value ? 0 : (std::is_same<T, TC>::value ? 1 : 2);
    if (ctx->gemm_slots[ti] == 0) {
        int cus = 0, per = 0;
        HGV_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
        HGV_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, gemm_kernel<T, BM, BN, NW>, NW * 64, 0));
        ctx->gemm_slots[ti] = std::max(1, cus * per);
    }
    const long slots = ctx->gemm_slots[ti];
    if (!small && a.allow_split && tiles < slots) {
        double best = chunks;
        const double out = (double)a.m * a.n * sizeof(E) * 1e-7;   // chunk steps per pass over C
        for (int s = 2; s <= 64 && chunks / s >= 4; ++s) {
            const double cost = (double)(((long)tiles * s + slots - 1) / slots * ((chunks + s - 1) / s)) + 2.0 +
                                (s + 1) * out;
            if (cost < best) {
                best = cost;
                splits = s;
            }
        }
    }
    size_t need = (size_t)splits * a.m * a.n * sizeof(E);
    while (splits > 1 && (ws == nullptr || need > ws_bytes)) {
        --splits;
        need = (size_t)splits * a.m * a.n * sizeof(E);
    }
    g.splits = splits;
    g.P = splits > 1 ? ws : nullptr;

    // optional accounting of the 64 x 64 complex-double tile kernel alone (the
    // events bracket gemm_kernel<TZ, 64, 64, 4>; the split-K reduction and the
    // small-product tiles are separate kernels)
    const bool timed = ctx->time_gemm && std::is_same<T, TZ>::value && !small;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timed) {
        if (ctx->ev_free.size() < 2) {
            hipEvent_t x, y;
            HGV_HIP(hipEventCreate(&x));
            HGV_HIP(hipEventCreate(&y));
            ctx->ev_free.push_back(x);
            ctx->ev_free.push_back(y);
        }
        e0 = ctx->ev_free.back(); ctx->ev_free.pop_back();
        e1 = ctx->ev_free.back(); ctx->ev_free.pop_back();
    }
    dim3 grid(tiles, splits);
    if (timed) {
        // the start and stop events ride on the kernel's own dispatch (no separate
        // marker packets between the launches)
        hipExtLaunchKernelGGL((gemm_kernel<T, BM, BN, NW>), grid, dim3(NW * 64), 0, ctx->stream, e0, e1, 0, g);
    } else if (small && bn == 32 && bm == 32) {
        hipLaunchKernelGGL((gemm_kernel<T, 32, 32, 4>), grid, dim3(256), 0, ctx->stream, g);
    } else if (small && bm == 32) {
        hipLaunchKernelGGL((gemm_kernel<T, 32, 64, 4>), grid, dim3(256), 0, ctx->stream, g);
    } else if (small) {
        hipLaunchKernelGGL((gemm_kernel<T, 64, 32, 4>), grid, dim3(256), 0, ctx->stream, g);
    } else {
        hipLaunchKernelGGL((gemm_kernel<T, BM, BN, NW>), grid, dim3(NW * 64), 0, ctx->stream, g);
    }
    HGV_LAUNCH_CHECK();
    if (timed) {
        ctx->ev_pending.push_back({e0, e1});
        ctx->ev_flops.push_back(flops);
    }
    if (splits > 1) {
        size_t total = (size_t)a.m * a.n;
        int blocks = (int)std::min<size_t>(cdivz(total, 256), 4096);
        hipLaunchKernelGGL((splitk_reduce<T>), dim3(blocks), dim3(256), 0, ctx->stream, g);
        HGV_LAUNCH_CHECK();
    }
}

size_t zgemm_splitk_bytes(int n) {
    // room for 16 partial tiles of a 256 x 256 output (or n x n when smaller),
    // and for 8 partial copies of an n x 64 panel product
    size_t d = (size_t)std::min(std::max(n, 64), 256);
    return std::max(16 * d * d, (size_t)8 * std::max(n, 1) * 64) * sizeof(double2);
}

void zgemm(hgv_ctx_s *ctx, const ZGemm &g, double2 *ws, size_t ws_bytes) {
    if (g.m <= 0 || g.n <= 0) return;
    double f = 8.0 * g.m * (double)g.n * g.k * ((g.A2 && g.B2) ? 2 : 1);
    if (g.lower) f *= 0.5;
    gemm_launch<TZ>(ctx, g, ws, ws_bytes, f);
}

void cgemm(hgv_ctx_s *ctx, const CGemm &g, float2 *ws, size_t ws_bytes) {
    if (g.m <= 0 || g.n <= 0) return;
    double f = 8.0 * g.m * (double)g.n * g.k * ((g.A2 && g.B2) ? 2 : 1);
    if (g.lower) f *= 0.5;
    gemm_launch<TC>(ctx, g, ws, ws_bytes, f);
}

struct DGemmArgs {
    int m, n, k;
    char opa, opb;
    const double *A; int lda;
    const double *B; int ldb;
    char opa2, opb2;
    const double *A2; int lda2;
    const double *B2; int ldb2;
    double alpha, beta;
    double *C; int ldc;
    int lower;
    int allow_split;
    const int *gate = nullptr;
    int gate_val = 0;
};

void dgemm_nn(hgv_ctx_s *ctx, int m, int n, int k, double alpha, const double *A, int lda,
              const double *B, int ldb, double beta, double *C, int ldc) {
    if (m <= 0 || n <= 0) return;
    DGemmArgs a{m, n, k, 'N', 'N', A, lda, B, ldb, 'N', 'N', nullptr, 1, nullptr, 1, alpha, beta, C, ldc, 0, 1};
    gemm_launch<TD>(ctx, a, nullptr, 0, 2.0 * m * (double)n * k);
}

}  // namespace hgv
