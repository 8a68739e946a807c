// he2hb.hip -- first stage of the two-stage tridiagonalisation (Alg. 2 step 1,
// Sec. 4.2, Fig. 1): reduction of the Hermitian A' to a band of width nb by
// block Householder transformations, and the matching back-transformation
// Y <- Q1 Y of Alg. 2 step 3.
//
// Panel p (columns k = p*nb .. k+jb-1) is factored below the band:
//   (a) panel QR of P = A[k+nb:n, k:k+jb]:  P = (H_0 ... H_{r-1}) [R; 0],
//       H_j = I - tau_j v_j v_j^H with H_j^H x = beta_j e_1, beta_j real;
//   (b) T (compact WY, forward) from tau and V^H V:  H_0...H_{r-1} = I - V T V^H;
//   (c) two-sided update of the trailing block A22 = A[k+nb:, k+nb:]:
//       X = A22 V T (hemm), W = X - 1/2 V (T^H (V^H X)),
//       A22 <- A22 - V W^H - W V^H (her2k, lower triangle only).
// (b) and (c) are MFMA GEMMs (gemm.hip).  The panel QR is a sequence of
// column steps; each step is one launch over row chunks of the panel held in
// LDS: it finishes the reduction of the previous step's partial inner
// products (fixed order, so results are reproducible), forms the reflector,
// applies it to its rows, and computes the partial inner products the next
// column needs.  Each launch boundary is the grid-wide synchronisation.
//
// Every stage is a template on the storage type E (complex128, or complex64 for
// the mixed-precision solve); the panel's inner products, norms, reflector
// scalars and the T factors are always computed in FP64.
#include <algorithm>
#include <type_traits>

#include "hgv_internal.h"

namespace hgv {

constexpr int PNB = 64;    // largest panel width supported by the column kernel
// panel rows per workgroup: 64 for complex double (67 KB of LDS, so that a
// chunk can share a CU with GEMM tiles while the next panel is factored
// during an update), 128 for complex float (75 KB)
template <class E>
constexpr int pch() {
    return sizeof(E) == 16 ? 64 : 128;
}

template <class E>
struct PanelArgs {
    E *P; int ldp;         // panel, N x jb
    int N, jb;
    double2 *part;         // [2][G][PNB] partial sums (double-buffered by step)
    double2 *rowb;         // [2][PNB] pivot row of the next column (double-buffered)
    double2 *tau;          // [jb]
    int G;
    const int *skip;       // non-null and set: the panel was factored another way
};

// Reflector of x = (alpha, x_1..) with tail = ||x_1..||^2:  H^H x = beta e_1,
// H = I - tau v v^H, v_0 = 1, v_i = scale x_i.
__device__ inline void make_reflector(double2 alpha, double tail, double &beta, double2 &tau, double2 &scale) {
    if (tail == 0.0 && alpha.y == 0.0) {
        beta = alpha.x;
        tau = make_double2(0.0, 0.0);
        scale = make_double2(0.0, 0.0);
        return;
    }
    double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + tail);
    beta = -copysign(nrm, alpha.x);
    tau = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
    scale = zdiv(make_double2(1.0, 0.0), make_double2(alpha.x - beta, alpha.y));
}

template <class E>
struct PanelShared {
    E Ps[pch<E>()][PNB + 1];
    double2 s[PNB], r0v[PNB], w[PNB];
    double2 vrow[pch<E>()];
    double2 red[4][PNB];
};

// The three parts of step j (-1: only prepare column 0) of the panel QR on row
// chunk g: load the chunk's columns c0.. into LDS, compute the step, write the
// columns back.
template <class E>
__device__ void panel_chunk_load(const PanelArgs<E> &a, PanelShared<E> &sh, int g, int c0) {
    auto &Ps = sh.Ps;
    const int tid = threadIdx.x;
    constexpr int PCH = pch<E>();
    const int row0 = g * PCH;
    const int rows = min(PCH, a.N - row0);
    // load the chunk's columns c0..jb-1 through registers: every load is issued
    // (elements outside the chunk read its in-range element (row0, c0)) before
    // the first one is waited for
    {
        constexpr int NLD = PCH * PNB / 256;
        E pv[NLD];
#pragma unroll
        for (int u = 0; u < NLD; ++u) {
            const int t = tid + 256 * u, r = t % PCH, c = c0 + t / PCH;
            const bool in = r < rows && c < a.jb;
            pv[u] = a.P[in ? row0 + r + (size_t)c * a.ldp : row0 + (size_t)c0 * a.ldp];
        }
        // unconditional stores (a conditional one would let the compiler sink its
        // load into the branch): rows past the chunk are never read, columns past
        // the panel go to the padding column PNB
#pragma unroll
        for (int u = 0; u < NLD; ++u) {
            const int t = tid + 256 * u, r = t % PCH, c = c0 + t / PCH;
            Ps[r][c < a.jb ? c : PNB] = pv[u];
        }
    }
}

template <class E>
__device__ void panel_chunk_store(const PanelArgs<E> &a, PanelShared<E> &sh, int g, int c0) {
    auto &Ps = sh.Ps;
    const int tid = threadIdx.x;
    constexpr int PCH = pch<E>();
    const int row0 = g * PCH;
    const int rows = min(PCH, a.N - row0);
    const int ncol = a.jb - c0;
    // write back the updated columns
    for (int t = tid; t < PCH * ncol; t += 256) {
        int r = t % PCH, c = c0 + t / PCH;
        if (r < rows) a.P[row0 + r + (size_t)c * a.ldp] = Ps[r][c];
    }
}

template <class E>
__device__ void panel_chunk_compute(const PanelArgs<E> &a, PanelShared<E> &sh, int j, int g) {
    auto &Ps = sh.Ps;
    auto &s = sh.s;
    auto &r0v = sh.r0v;
    auto &w = sh.w;
    auto &vrow = sh.vrow;
    auto &red = sh.red;
    const int tid = threadIdx.x;
    constexpr int PCH = pch<E>();
    const int row0 = g * PCH;
    const int rows = min(PCH, a.N - row0);
    const int c0 = max(j, 0);
    const int ncol = a.jb - c0;
    const int ib = (j + 1) & 1, ob = (j + 2) & 1;
    const double2 *part_in = a.part + (size_t)ib * a.G * PNB;
    double2 *part_out = a.part + (size_t)ob * a.G * PNB;
    const double2 *row_in = a.rowb + ib * PNB;
    double2 *row_out = a.rowb + ob * PNB;
    auto ld = [&](int r, int c) -> double2 { return El<E>::to(Ps[r][c]); };
    if (j >= 0) {
        // finish the reduction of the partial sums for column j: 4 threads per
        // column sum interleaved quarters of the G partials (loads issued
        // independently), then the quarters are added in a fixed order, so the
        // result is the same in every block and from run to run
        const int c = tid & 63, qq = tid >> 6;
        double2 acc = make_double2(0.0, 0.0);
        if (c < ncol) {
            // partials q = qq, qq + 4, ... in ascending order, PQ loads in flight (the
            // partials come from memory, so the number of dependent batches sets the time)
            constexpr int PQ = 24;
            const double2 *src = part_in + j + c;
            for (int q0 = qq; q0 < a.G; q0 += 4 * PQ) {
                double2 pq[PQ];
#pragma unroll
                for (int u = 0; u < PQ; ++u) {
                    const int q = q0 + 4 * u;
                    pq[u] = zsel(q < a.G, src[(size_t)(q < a.G ? q : qq) * PNB], make_double2(0.0, 0.0));
                }
#pragma unroll
                for (int u = 0; u < PQ; ++u) acc = zadd(acc, pq[u]);
            }
        }
        red[qq][c] = acc;
        if (tid < ncol) r0v[tid] = row_in[j + tid];
        __syncthreads();
        if (tid < ncol) s[tid] = zadd(zadd(red[0][tid], red[1][tid]), zadd(red[2][tid], red[3][tid]));
    }
    __syncthreads();
    if (j >= 0) {
        const double2 alpha = r0v[0];
        const double tail = s[0].x;
        double beta;
        double2 tau, scale;
        make_reflector(alpha, tail, beta, tau, scale);
        // w_c = conj(tau) * v^H p_c,  v^H p_c = p0_c + conj(scale) (s_c - conj(alpha) p0_c)
        if (tid < ncol && tid > 0) {
            double2 p0 = r0v[tid];
            double2 t1 = zsub(s[tid], zcmul(alpha, p0));
            double2 vhp = zadd(p0, zcmul(scale, t1));
            w[tid] = zcmul(tau, vhp);
        }
        if (tid < rows) {
            int gr = row0 + tid;
            double2 v = make_double2(0.0, 0.0);
            if (gr == j) v = make_double2(1.0, 0.0);
            else if (gr > j) v = zmul(scale, ld(tid, j));
            vrow[tid] = v;
        }
        __syncthreads();
        // apply H^H to columns j+1.., store v below the diagonal and beta on it;
        // thread -> row tid % PCH and columns cc = tid / PCH, tid / PCH + NCG, ...
        // (a fixed-count loop, so that its LDS accesses overlap)
        {
            constexpr int NCG = 256 / PCH;
            const int r = tid % PCH, gr = row0 + r;
            const bool rok = r < rows && gr >= j;
            const double2 vr = vrow[r];
#pragma unroll
            for (int u = 0; u < PNB / NCG; ++u) {
                const int cc = NCG * u + tid / PCH;
                if (cc < ncol && rok) {
                    const int c = j + cc;
                    Ps[r][c] = El<E>::from(cc == 0 ? zsel(gr == j, make_double2(beta, 0.0), vr)
                                                   : zsub(ld(r, c), zmul(vr, w[cc])));
                }
            }
        }
        if (g == 0 && tid == 0) a.tau[j] = tau;
        __syncthreads();
    }
    // partial inner products for column jn = j+1:
    //   part[c] = sum_{rows i >= jn} conj(P[i, jn]) P[i, c]   (c > jn)
    //   part[jn] = sum_{rows i > jn} |P[i, jn]|^2
    const int jn = j + 1;
    if (jn < a.jb && jn < a.N) {
        const int c = tid & (PNB - 1), grp = tid >> 6;
        double2 acc = make_double2(0.0, 0.0);
        if (c >= jn && c < a.jb) {
            // fixed count and no branches, so that the LDS reads overlap; rows
            // outside the chunk or above the diagonal contribute zero (for
            // c == jn the diagonal row too: conj(x) x is |x|^2 with a zero
            // imaginary part)
#pragma unroll 8
            for (int rr = 0; rr < PCH / 4; ++rr) {
                const int r = grp * (PCH / 4) + rr, gr = row0 + r;
                const bool ok = r < rows && (c == jn ? gr > jn : gr >= jn);
                acc = zadd(acc, zsel(ok, zcmul(ld(r, jn), ld(r, c)), make_double2(0.0, 0.0)));
            }
        }
        red[grp][c] = acc;
        __syncthreads();
        if (tid < PNB) {
            double2 t = zadd(zadd(red[0][tid], red[1][tid]), zadd(red[2][tid], red[3][tid]));
            part_out[(size_t)g * PNB + tid] = t;
            int lr = jn - row0;
            if (lr >= 0 && lr < rows && tid >= jn && tid < a.jb) row_out[tid] = ld(lr, tid);
        }
    }
}

// Step j of the panel QR; workgroup g = row chunk g.
template <class E>
__global__ __launch_bounds__(256) void panel_step_kernel(PanelArgs<E> a, int j) {
    __shared__ PanelShared<E> sh;
    if (a.skip && *a.skip) return;
    const int c0 = max(j, 0);
    panel_chunk_load<E>(a, sh, blockIdx.x, c0);
    panel_chunk_compute<E>(a, sh, j, blockIdx.x);
    panel_chunk_store<E>(a, sh, blockIdx.x, c0);
}

// Wait until flags[0 .. G-1] >= target: the lanes of wave 0 poll the flags with
// relaxed device-scope loads, then take an acquire fence; the workgroup
// barrier follows.  The wait is bounded: one that gives up sets *err, and
// every wait that sees *err set returns at once, so the launch always ends
// (with *err reporting that the result is not valid).
__device__ inline void panel_wait(const int *flags, int G, int target, int *err) {
    const int tid = threadIdx.x;
    if (tid < 64) {
        long spins = 0;
        for (;;) {
            bool ok = true;
            for (int q = tid; q < G; q += 64)
                ok = ok && __hip_atomic_load(&flags[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target;
            if (__all(ok)) break;
            if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
            __builtin_amdgcn_s_sleep(1);
            if (++spins > (1L << 20)) {
                __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

// The whole panel QR in one cooperative launch: workgroup g keeps row chunk g
// in LDS for every column step.  After step j it publishes the partial inner
// products of column j+1 (and, for the chunk holding row j+1, that row) and
// then flags[g] = gen + j + 2 with a release store; step j+1 starts once every
// chunk's flag has reached that value.  gen grows from panel to panel, so the
// flags are cleared once per reduction.
template <class E>
__global__ __launch_bounds__(256) void panel_persist_kernel(PanelArgs<E> a, int *flags, int gen, int *err) {
    __shared__ PanelShared<E> sh;
    if (a.skip && *a.skip) return;   // the same value in every workgroup: none waits
    const int g = blockIdx.x;
    const int r = min(a.N, a.jb);
    panel_chunk_load<E>(a, sh, g, 0);
    for (int j = -1; j < r; ++j) {
        if (j >= 0) panel_wait(flags, a.G, gen + j + 1, err);
        panel_chunk_compute<E>(a, sh, j, g);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (threadIdx.x == 0) __hip_atomic_store(&flags[g], gen + j + 2, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    panel_chunk_store<E>(a, sh, g, 0);
}

// Explicit V (N x r): unit diagonal, zeros above, reflector entries below.
template <class E>
__global__ void extract_v_kernel(int N, int r, const E *P, int ldp, E *V, int ldv) {
    int i = blockIdx.x * 64 + (threadIdx.x & 63);
    int c = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i >= N || c >= r) return;
    E v = (i > c) ? P[i + (size_t)c * ldp] : El<E>::mk(i == c ? 1.0 : 0.0, 0.0);
    V[i + (size_t)c * ldv] = v;
}

// T (r x r upper, ldt) from tau and G = V^H V:  T_jj = tau_j,
// T[0:j, j] = -tau_j T[0:j, 0:j] G[0:j, j].  One workgroup of NT threads,
// column by column; G is staged in LDS and the QN = NT / 64 consecutive lanes
// of row i share the row's triangular matrix-vector product (butterfly-
// combined).  The columns form a chain of short dependent steps, so NT = 1024
// (four waves per SIMD, a quarter of the chain per lane).
template <class E, int NT>
__global__ __launch_bounds__(NT) void build_t_kernel(int r, const double2 *tau, const E *G, int ldg, E *T, int ldt,
                                                    const int *skip) {
    if (skip && *skip) return;
    constexpr int QN = NT / 64;
    __shared__ double2 Ts[PNB][PNB + 1];
    __shared__ double2 Gs[PNB][PNB + 1];
    __shared__ double2 taus[PNB];
    const int tid = threadIdx.x;
    for (int t = tid; t < PNB * PNB; t += NT) {
        const int i = t % PNB, j = t / PNB;
        Ts[i][j] = make_double2(0.0, 0.0);
        Gs[i][j] = (i < r && j < r) ? El<E>::to(G[i + (size_t)j * ldg]) : make_double2(0.0, 0.0);
    }
    if (tid < PNB) taus[tid] = (tid < r) ? tau[tid] : make_double2(0.0, 0.0);
    __syncthreads();
    const int row = tid / QN, q = tid % QN;
    for (int j = 0; j < r; ++j) {
        const double2 tj = taus[j];
        if (row < j) {
            double2 acc = make_double2(0.0, 0.0);
            for (int l = row + q; l < j; l += QN) acc = zadd(acc, zmul(Ts[row][l], Gs[l][j]));
#pragma unroll
            for (int o = 1; o < QN; o <<= 1) {
                acc.x += __shfl_xor(acc.x, o, 64);
                acc.y += __shfl_xor(acc.y, o, 64);
            }
            if (q == 0) Ts[row][j] = zmul(make_double2(-tj.x, -tj.y), acc);
        }
        if (tid == 0) Ts[j][j] = tj;
        __syncthreads();
    }
    for (int t = tid; t < r * r; t += NT) T[t % r + (size_t)(t / r) * ldt] = El<E>::from(Ts[t % r][t / r]);
}

// ---- panel QR in a fixed number of launches -------------------------------------
// The panel QR of step (a) of the reduction to band (Sec. 4.2, Fig. 1): a complex
// double panel of full column rank that is not too ill-conditioned is factored
// without the column steps:
//   Cholesky QR twice: G1 = P^H P = L1 L1^H, Q1 = P L1^-H; G2 = Q1^H Q1 = L2 L2^H,
//   Q = Q1 L2^-H, so P = Q R with R = (L1 L2)^H (the second pass restores the
//   orthogonality the first loses to the rounding of G1).  G2 = I + E with E of
//   the order of cond(P)^2 eps, so its factor is taken to first order,
//   L2 = I + tril(E) with the diagonal halved and L2^-1 = I - (L2 - I): the
//   neglected terms are O(|E|^2), below rounding while max |E| <= 1e-9;
//   Householder reconstruction: the LU factorisation without pivoting
//   Q - [S; 0] = V U, with the unitary diagonal S chosen column by column as
//   S_jj = -u/|u| (u the current diagonal entry, -1 if zero) so that every pivot
//   has modulus at least 1, gives the unit lower-trapezoidal V of the block
//   reflector Q_h = I - V T V^H whose first r columns are Q S^H; hence
//   P = Q_h [S R; 0], the reflectors' scalars are tau_j = -U_jj conj(S_jj), and
//   T = -(U S^H) V1^-H (from V T V1^H = E - Q S^H, E the first r columns of I).
// (Yamamoto, Nakatsukasa, Yanagisawa and Fukaya, ETNA 44, 2015, for the two
// passes; Ballard, Demmel, Grigori, Jacquelin, Knight and Nguyen, IPDPS 2014,
// for the reconstruction, here in complex arithmetic.)  The results satisfy
// the same contract as the column steps: V below the diagonal of P, the band
// block S R on and above it (its diagonal complex), tau, T.
// A device flag decides between the two methods without a host round trip: the
// factorisation of G1 sets it when G1 is numerically positive definite with
// ||L1||_F ||L1^-1||_F <= 1e5, the reconstruction clears it unless
// max |G2 - I| <= 1e-9 (so the panels taken have condition numbers up to about
// 1e4).  It gates the reconstruction and the product that finishes V on, and
// the column-step kernels, the product V^H V and the T recurrence off.

constexpr int CQ_NW = 8;             // waves per workgroup
constexpr int CQ_T = 64 / CQ_NW;      // consecutive columns per wave
constexpr int CQ_MC = 8;              // rows of a product's operands staged in LDS at a time

__device__ inline double2 lane_z(double2 v, int l) { return make_double2(lane_f64(v.x, l), lane_f64(v.y, l)); }

// a[t] for a wave-uniform t, without indexing the register array
template <int NN>
__device__ inline double2 pick_reg(const double2 (&a)[NN], int t) {
    double2 r = a[0];
#pragma unroll
    for (int u = 1; u < NN; ++u) r = zsel(u == t, a[u], r);
    return r;
}
template <int NN>
__device__ inline void put_reg(double2 (&a)[NN], int t, double2 v) {
#pragma unroll
    for (int u = 0; u < NN; ++u) a[u] = zsel(u == t, v, a[u]);
}

// Sum (max when MAX, NaN winning) over the workgroup; the result in every thread.
template <bool MAX>
__device__ inline double cq_reduce(double v, double *sh) {
    for (int o = 32; o > 0; o >>= 1) {
        const double u = __shfl_xor(v, o);
        v = MAX ? ((u > v || u != u) ? u : v) : v + u;
    }
    const int tid = threadIdx.x;
    __syncthreads();
    if ((tid & 63) == 0) sh[tid >> 6] = v;
    __syncthreads();
    double r = sh[0];
    for (int q = 1; q < CQ_NW; ++q) r = MAX ? ((sh[q] > r || sh[q] != sh[q]) ? sh[q] : r) : r + sh[q];
    return r;
}

// Layout of the 64 x 64 matrices of the two kernels below: lane i holds row i,
// wave w the columns CQ_T w .. CQ_T w + CQ_T - 1 (r x r padded with the identity).
// C += A B for such a C, the operands staged in LDS CQ_MC rows of B (columns of A)
// at a time by sa(m0) (As[mm][i] = A[i][m0 + mm]) and sb(m0) (Bs[mm][k] =
// B[m0 + mm][k]); a wave reads B's entries of its columns as broadcasts.
template <class SA, class SB>
__device__ inline void cq_product(double2 (&c)[CQ_T], SA sa, SB sb, double2 (*As)[65], double2 (*Bs)[65], int w,
                                  int i) {
    for (int m0 = 0; m0 < 64; m0 += CQ_MC) {
        __syncthreads();
        sa(m0);
        sb(m0);
        __syncthreads();
#pragma unroll
        for (int mm = 0; mm < CQ_MC; ++mm) {
            const double2 av = As[mm][i];
#pragma unroll
            for (int t = 0; t < CQ_T; ++t) zfma(c[t], av, Bs[mm][CQ_T * w + t]);
        }
    }
}

// G = L L^H (r x r Hermitian, r <= 64, lower triangle read) and X = L^-1, one
// workgroup.  Step j eliminates column j below the diagonal (the wave holding
// it publishes it in LDS; one barrier per step) and applies the same row
// operations to an identity held beside it, which ends as the inverse of the
// unit lower factor; the pivots' square roots scale both at the end.  The
// updates are branch-free within a wave (a zero multiplier, or a zero entry of
// the triangular inverse, leaves an element unchanged), so that the chains of
// a wave's columns overlap.  Sets *ok to whether the factorisation succeeded with
// ||L||_F ||L^-1||_F <= 1e5.
__global__ __launch_bounds__(CQ_NW * 64) void cqr_chol_kernel(int r, const double2 *__restrict__ G, int ldg,
                                                              double2 *__restrict__ L, double2 *__restrict__ X,
                                                              int ldo, int *ok) {
    __shared__ double2 col[2][64];
    __shared__ double red[CQ_NW];
    const int tid = threadIdx.x, i = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    double2 a[CQ_T], x[CQ_T];
    double tr = 0.0;
#pragma unroll
    for (int t = 0; t < CQ_T; ++t) {
        const int k = CQ_T * w + t;
        const bool in = i < r && k < r;
        const double id = i == k ? 1.0 : 0.0;
        const double2 v = zsel(in, G[in ? i + (size_t)k * ldg : 0], make_double2(id, 0.0));
        a[t] = v;
        x[t] = make_double2(id, 0.0);
        if (in && i == k) tr += v.x;
    }
    double myd = 1.0;
    bool bad = false;
    for (int j = 0; j < 64; ++j) {
        const int buf = j & 1, wj = j / CQ_T;
        if (w == wj) col[buf][i] = pick_reg(a, j - CQ_T * w);
        __syncthreads();
        const double2 c = col[buf][i];
        const double d = lane_f64(c.x, j);   // the same pivot in every wave
        bad = bad || !(d > 0.0);
        if (i == j) myd = d;
        const double2 m = zsel(i > j && !bad, zscale(1.0 / d, c), make_double2(0.0, 0.0));
        if (w >= wj) {   // columns k > j: G[i][k] -= m_i conj(G[k][j])
#pragma unroll
            for (int t = 0; t < CQ_T; ++t) {
                const int k = CQ_T * w + t;
                const double2 mk = zsel(k > j, m, make_double2(0.0, 0.0));
                zfma(a[t], make_double2(-mk.x, -mk.y), zconj(lane_z(c, k)));
            }
        }
        if (w <= wj) {   // columns k <= j of the inverse (X[j][k] = 0 for k > j)
#pragma unroll
            for (int t = 0; t < CQ_T; ++t) zfma(x[t], make_double2(-m.x, -m.y), lane_z(x[t], j));
        }
    }
    const double si = bad ? 1.0 : 1.0 / sqrt(myd);
    double xs = 0.0;
#pragma unroll
    for (int t = 0; t < CQ_T; ++t) {
        const int k = CQ_T * w + t;
        const double dk = bad ? 1.0 : lane_f64(myd, k);
        const double sk = sqrt(dk);
        const double2 l = zsel(i == k, make_double2(sk, 0.0), zsel(i > k, zscale(1.0 / sk, a[t]), make_double2(0.0, 0.0)));
        const double2 xv = zscale(si, x[t]);
        if (i < r && k < r) {
            L[i + (size_t)k * ldo] = l;
            X[i + (size_t)k * ldo] = xv;
            xs += zabs2(xv);
        }
    }
    const double trs = cq_reduce<false>(tr, red);
    const double xss = cq_reduce<false>(xs, red);
    if (tid == 0) *ok = (!bad && trs * xss <= 1e10) ? 1 : 0;
}

// The second pass and the reconstruction, one workgroup in the layout above,
// when *ok (cleared here unless max |G2 - I| <= 1e-9):
//   L2 and L2^-1 to first order from E = G2 - I (lower triangle read);
//   Q_top = Q1[0:r, :] L2^-H;
//   its modified LU Q_top - S = V1 U, with V1^-1 formed beside it (V1 goes below
//   the diagonal of P's top block, tau_j = -U_jj conj(S_jj));
//   Y = U^-1;  M = L2^-H Y (so that V2 = Q1[r:, :] M, a GEMM);
//   T = -(U S^H) V1^-H, the block reflector's triangular factor
//   (the first r columns of I - V T V^H are Q S^H: V T V1^H = E - Q S^H);
//   the band block S (L1 L2)^H on and above the diagonal of P's top block.
__global__ __launch_bounds__(CQ_NW * 64) void cqr_recon_kernel(int r, const double2 *__restrict__ Q1, int ldq,
                                                               const double2 *__restrict__ L1,
                                                               const double2 *__restrict__ G2, int ldo, double2 *P,
                                                               int ldp, double2 *tau, double2 *__restrict__ T,
                                                               int ldt, double2 *M, int *ok) {
    if (*ok == 0) return;
    __shared__ double2 col[2][64];
    __shared__ double2 sv[64];
    __shared__ double2 As[CQ_MC][65], Bs[CQ_MC][65];
    __shared__ double red[CQ_NW];
    const int tid = threadIdx.x, i = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const double2 zero = make_double2(0.0, 0.0), one = make_double2(1.0, 0.0);
    constexpr int NT = CQ_NW * 64;
    {
        double dev = 0.0;
        for (int e = tid; e < r * r; e += NT) {
            const int ii = e % r, k = e / r;
            if (ii >= k) {
                const double2 v = G2[ii + (size_t)k * ldo];
                const double d = sqrt(zabs2(zsub(v, make_double2(ii == k ? 1.0 : 0.0, 0.0))));
                dev = (d > dev || d != d) ? d : dev;
            }
        }
        const double devm = cq_reduce<true>(dev, red);
        if (!(devm <= 1e-9)) {
            if (tid == 0) *ok = 0;
            return;
        }
    }
    // L2[k][m] (k >= m) = E[k][m] below the diagonal, 1 + E[k][k] / 2 on it;
    // X2 = L2^-1 = 2 I - L2 to first order
    auto l2 = [&](int k, int m) -> double2 {
        const double2 v = G2[k + (size_t)m * ldo];
        return zsel(k == m, make_double2(1.0 + 0.5 * (v.x - 1.0), 0.0), v);
    };
    auto x2 = [&](int k, int m) -> double2 {
        const double2 v = G2[k + (size_t)m * ldo];
        return zsel(k == m, make_double2(1.0 - 0.5 * (v.x - 1.0), 0.0), zsub(zero, v));
    };
    double2 a[CQ_T], vx[CQ_T];
#pragma unroll
    for (int t = 0; t < CQ_T; ++t) a[t] = zero;
    // Q_top = Q1[0:r, 0:r] X2^H
    cq_product(
        a,
        [&](int m0) {
            for (int e = tid; e < CQ_MC * 64; e += NT) {
                const int ii = e & 63, m = m0 + (e >> 6);
                const bool in = ii < r && m < r;
                As[e >> 6][ii] = zsel(in, Q1[in ? ii + (size_t)m * ldq : 0], zero);
            }
        },
        [&](int m0) {
            for (int e = tid; e < CQ_MC * 64; e += NT) {
                const int k = e & 63, m = m0 + (e >> 6);
                const bool in = k < r && m <= k;
                Bs[e >> 6][k] = zsel(in, zconj(x2(in ? k : 0, in ? m : 0)), zero);
            }
        },
        As, Bs, w, i);
#pragma unroll
    for (int t = 0; t < CQ_T; ++t) {
        const int k = CQ_T * w + t;
        if (i >= r || k >= r) a[t] = zsel(i == k, one, zero);
        vx[t] = zsel(i == k, one, zero);
    }
    // modified LU: at step j the pivot is a_jj - S_jj with S_jj = -a_jj / |a_jj|
    for (int j = 0; j < 64; ++j) {
        const int buf = j & 1, wj = j / CQ_T;
        if (w == wj) {
            const int tj = j - CQ_T * w;
            const double2 cur = pick_reg(a, tj);
            const double2 ajj = lane_z(cur, j);
            const double nrm = sqrt(zabs2(ajj));
            const double2 sj = zsel(nrm > 0.0, make_double2(-ajj.x / nrm, -ajj.y / nrm), make_double2(-1.0, 0.0));
            const double2 u = zsub(ajj, sj);
            const double2 l = zdiv(cur, u);
            put_reg(a, tj, zsel(i > j, l, zsel(i == j, u, cur)));
            col[buf][i] = zsel(i > j, l, zero);
            if (i == j) {
                sv[j] = sj;
                if (j < r) tau[j] = zsub(zero, zmul(u, zconj(sj)));
            }
        }
        __syncthreads();
        const double2 l = col[buf][i];
        if (w >= wj) {
#pragma unroll
            for (int t = 0; t < CQ_T; ++t) {
                const int k = CQ_T * w + t;
                const double2 lk = zsel(k > j, l, zero);
                zfma(a[t], make_double2(-lk.x, -lk.y), lane_z(a[t], j));
            }
        }
        if (w <= wj) {   // V1^-1: the same row operations on the identity
#pragma unroll
            for (int t = 0; t < CQ_T; ++t) zfma(vx[t], make_double2(-l.x, -l.y), lane_z(vx[t], j));
        }
    }
#pragma unroll
    for (int t = 0; t < CQ_T; ++t) {
        const int k = CQ_T * w + t;
        if (i > k && i < r && k < r) P[i + (size_t)k * ldp] = a[t];
        M[i + (size_t)k * 64] = vx[t];   // V1^-1 (64 x 64) parked in M's space until M is formed
    }
    // T = -(U S^H) V1^-H: A[i][m] = U[i][m] conj(S_m) (upper), B[m][k] = conj(V1^-1[k][m])
    double2 c[CQ_T];
#pragma unroll
    for (int t = 0; t < CQ_T; ++t) c[t] = zero;
    cq_product(
        c,
        [&](int m0) {
#pragma unroll
            for (int t = 0; t < CQ_T; ++t) {
                const int m = CQ_T * w + t;
                if (m >= m0 && m < m0 + CQ_MC) As[m - m0][i] = zsel(i <= m, zmul(a[t], zconj(sv[m])), zero);
            }
        },
        [&](int m0) {
            for (int e = tid; e < CQ_MC * 64; e += NT) {
                const int k = e & 63, m = m0 + (e >> 6);
                Bs[e >> 6][k] = zconj(M[k + (size_t)m * 64]);
            }
        },
        As, Bs, w, i);
#pragma unroll
    for (int t = 0; t < CQ_T; ++t) {
        const int k = CQ_T * w + t;
        if (i < r && k < r) T[i + (size_t)k * ldt] = zsub(zero, c[t]);
    }
    // Y = U^-1 (upper), right-looking backward substitution from Y = I
    __syncthreads();
    double2 y[CQ_T];
#pragma unroll
    for (int t = 0; t < CQ_T; ++t) y[t] = zsel(CQ_T * w + t == i, one, zero);
    for (int j = 63; j >= 0; --j) {
        const int buf = j & 1, wj = j / CQ_T;
        if (w == wj) col[buf][i] = zsel(i <= j, pick_reg(a, j - CQ_T * w), zero);
        __syncthreads();
        const double2 cj = col[buf][i];
        const double2 iu = zdiv(one, lane_z(cj, j));
        const double2 cu = zsel(i < j, cj, zero);
        if (w >= wj) {   // Y[j][k] = 0 for k < j
#pragma unroll
            for (int t = 0; t < CQ_T; ++t) {
                y[t] = zsel(i == j, zmul(y[t], iu), y[t]);
                zfma(y[t], make_double2(-cu.x, -cu.y), lane_z(y[t], j));
            }
        }
    }
    // M = X2^H Y: A[i][m] = conj(X2[m][i]), B = Y
#pragma unroll
    for (int t = 0; t < CQ_T; ++t) c[t] = zero;
    cq_product(
        c,
        [&](int m0) {
            for (int e = tid; e < CQ_MC * 64; e += NT) {
                const int ii = e & 63, m = m0 + (e >> 6);
                const bool in = m < r && ii <= m;
                As[e >> 6][ii] = zsel(in, zconj(x2(in ? m : 0, in ? ii : 0)), zero);
            }
        },
        [&](int m0) {
            if (i >= m0 && i < m0 + CQ_MC) {
#pragma unroll
                for (int t = 0; t < CQ_T; ++t) Bs[i - m0][CQ_T * w + t] = y[t];
            }
        },
        As, Bs, w, i);
#pragma unroll
    for (int t = 0; t < CQ_T; ++t) {
        const int k = CQ_T * w + t;
        if (i < r && k < r) M[i + (size_t)k * r] = c[t];
    }
    // Z = L1 L2 (lower); band block (S R)[k][i] = S_kk conj(Z[i][k]) for k <= i
#pragma unroll
    for (int t = 0; t < CQ_T; ++t) c[t] = zero;
    cq_product(
        c,
        [&](int m0) {
            for (int e = tid; e < CQ_MC * 64; e += NT) {
                const int ii = e & 63, m = m0 + (e >> 6);
                const bool in = ii < r && m <= ii;
                As[e >> 6][ii] = zsel(in, L1[in ? ii + (size_t)m * ldo : 0], zero);
            }
        },
        [&](int m0) {
            for (int e = tid; e < CQ_MC * 64; e += NT) {
                const int k = e & 63, m = m0 + (e >> 6);
                const bool in = m < r && k <= m;
                Bs[e >> 6][k] = zsel(in, l2(in ? m : 0, in ? k : 0), zero);
            }
        },
        As, Bs, w, i);
#pragma unroll
    for (int t = 0; t < CQ_T; ++t) {
        const int k = CQ_T * w + t;
        if (k < r && i >= k && i < r) P[k + (size_t)i * ldp] = zmul(sv[k], zconj(c[t]));
    }
}

struct CqrScratch {
    double2 *G, *L1, *X1, *M, *Q;   // r x r (ld r) each; Q: N x r (ld N)
    int *ok;
};

// Launches the fixed sequence for panel P (N x r, N >= r); sets up the flag
// that gates the column-step kernels launched after it.
static void cholqr_panel(hgv_ctx_s *ctx, double2 *P, int ldp, int N, int r, double2 *tau, double2 *T, int ldt,
                         const CqrScratch &c, void *ws, size_t wsb) {
    ZGemm g;   // G1 = P^H P
    g.m = r; g.n = r; g.k = N;
    g.opa = 'C'; g.A = P; g.lda = ldp;
    g.opb = 'N'; g.B = P; g.ldb = ldp;
    g.C = c.G; g.ldc = r;
    zgemm(ctx, g, static_cast<double2 *>(ws), wsb);
    hipLaunchKernelGGL(cqr_chol_kernel, dim3(1), dim3(CQ_NW * 64), 0, ctx->stream, r, c.G, r, c.L1, c.X1, r, c.ok);
    HGV_LAUNCH_CHECK();
    g = ZGemm();   // Q1 = P L1^-H
    g.m = N; g.n = r; g.k = r;
    g.opa = 'N'; g.A = P; g.lda = ldp;
    g.opb = 'C'; g.B = c.X1; g.ldb = r;
    g.C = c.Q; g.ldc = N;
    zgemm(ctx, g, static_cast<double2 *>(ws), wsb);
    g = ZGemm();   // G2 = Q1^H Q1
    g.m = r; g.n = r; g.k = N;
    g.opa = 'C'; g.A = c.Q; g.lda = N;
    g.opb = 'N'; g.B = c.Q; g.ldb = N;
    g.C = c.G; g.ldc = r;
    zgemm(ctx, g, static_cast<double2 *>(ws), wsb);
    hipLaunchKernelGGL(cqr_recon_kernel, dim3(1), dim3(CQ_NW * 64), 0, ctx->stream, r, c.Q, N, c.L1, c.G, r, P, ldp,
                       tau, T, ldt, c.M, c.ok);
    HGV_LAUNCH_CHECK();
    if (N > r) {
        g = ZGemm();   // V2 = Q1[r:, :] M, into P below the top block
        g.m = N - r; g.n = r; g.k = r;
        g.A = c.Q + r; g.lda = N;
        g.B = c.M; g.ldb = r;
        g.C = P + r; g.ldc = ldp;
        g.gate = c.ok; g.gate_val = 1;
        zgemm(ctx, g, static_cast<double2 *>(ws), wsb);
    }
}

template <class E>
__global__ void zero_kernel(E *p, size_t n) {
    size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = El<E>::mk(0.0, 0.0);
}

template <class E>
static void zero_async(hgv_ctx_s *ctx, E *p, size_t n) {
    if (n == 0) return;
    int blocks = (int)std::min<size_t>(cdivz(n, 256), 8192);
    hipLaunchKernelGGL(zero_kernel<E>, dim3(blocks), dim3(256), 0, ctx->stream, p, n);
    HGV_LAUNCH_CHECK();
}

static int num_panels(int n, int nb) { return (n - nb - 1 >= 0) ? (n - nb - 1) / nb + 1 : 0; }

// Panel QR + T for panel P (N x jb, r = min(N, jb) reflectors).  Leaves V in
// P (below the diagonal), beta on the diagonal, R above; T (r x r) in T, ldt.
// Workgroups of the persistent panel kernel that fit on the device at once.
template <class E>
static int panel_persist_capacity(hgv_ctx_s *ctx) {
    int cus = 0, per = 0;
    HGV_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
    HGV_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, panel_persist_kernel<E>, 256, 0));
    return cus * per;
}

__global__ void fill_int_kernel(int *p, int n, int v) {
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

// flags: progress flags of the persistent panel kernel (one per row chunk),
// err: its give-up flag (a slot no chunk uses), gen: this panel's flag base;
// the per-step launches are used when the chunks cannot all be resident at once
template <class E>
static void panel_qr(hgv_ctx_s *ctx, E *P, int ldp, int N, int jb, double2 *tau, double2 *part, double2 *rowb,
                     E *Vw, E *Gm, E *T, int ldt, void *ws, size_t wsb, int *flags, int *err, int gen,
                     int capacity, const CqrScratch *cq) {
    typedef typename El<E>::Gemm Gm_t;
    const int r = std::min(N, jb);
    const int G = cdiv(N, pch<E>());
    PanelArgs<E> a;
    a.P = P; a.ldp = ldp; a.N = N; a.jb = jb; a.tau = tau; a.G = G;
    a.part = part; a.rowb = rowb;
    a.skip = nullptr;
    if constexpr (std::is_same<E, double2>::value) {
        // complex double panels at least as tall as wide: the fixed-launch form
        // first, the column steps only where its flag says it did not apply
        if (cq && N >= jb && !(ctx->test_hooks & HGV_TEST_HOUSEHOLDER_PANELS)) {
            cholqr_panel(ctx, P, ldp, N, jb, tau, reinterpret_cast<double2 *>(T), ldt, *cq, ws, wsb);
            a.skip = cq->ok;
        }
    }
    if (G <= capacity && ctx->concurrent) {
        // side by side with the panels of other problems: a plain launch (the
        // share in `capacity` keeps every concurrent grid resident-able at once)
        hipLaunchKernelGGL(panel_persist_kernel<E>, dim3(G), dim3(256), 0, ctx->stream, a, flags, gen, err);
        HGV_LAUNCH_CHECK();
    } else if (G <= capacity) {
        void *args[] = {&a, &flags, &gen, &err};
        HGV_HIP(hipLaunchCooperativeKernel(reinterpret_cast<void *>(panel_persist_kernel<E>), dim3(G), dim3(256),
                                           args, 0, ctx->stream));
    } else {
        for (int j = -1; j < r; ++j) {
            hipLaunchKernelGGL(panel_step_kernel<E>, dim3(G), dim3(256), 0, ctx->stream, a, j);
            HGV_LAUNCH_CHECK();
        }
    }
    hipLaunchKernelGGL(extract_v_kernel<E>, dim3(cdiv(N, 64), cdiv(r, 4)), dim3(256), 0, ctx->stream, N, r, P, ldp,
                       Vw, N);
    HGV_LAUNCH_CHECK();
    // T from tau and G = V^H V, unless the fixed-launch form has written it
    Gm_t gg;  // G = V^H V
    gg.m = r; gg.n = r; gg.k = N;
    gg.opa = 'C'; gg.A = Vw; gg.lda = N;
    gg.opb = 'N'; gg.B = Vw; gg.ldb = N;
    gg.C = Gm; gg.ldc = r;
    gg.gate = a.skip; gg.gate_val = 0;
    gemm_any(ctx, gg, ws, wsb);
    hipLaunchKernelGGL((build_t_kernel<E, 1024>), dim3(1), dim3(1024), 0, ctx->stream, r, tau, Gm, r, T, ldt, a.skip);
    HGV_LAUNCH_CHECK();
}

template <class E>
void he2hb_t(hgv_ctx_s *ctx, int n, int nb, E *A, int lda, E *T1, Arena &ar, int *d_info) {
    typedef typename El<E>::Gemm Gm_t;
    if (nb > PNB) throw HipFail{hipErrorInvalidValue};
    const int np = num_panels(n, nb);
    const int Gmax = cdiv(std::max(n, 1), pch<E>());
    size_t wsb = zgemm_splitk_bytes(n);
    void *ws = ar.take<char>(wsb);
    double2 *part = ar.take<double2>((size_t)2 * Gmax * PNB);
    double2 *rowb = ar.take<double2>(2 * PNB);
    double2 *tau = ar.take<double2>(PNB);
    E *Vw = ar.take<E>((size_t)n * nb);
    E *Vw2 = ar.take<E>((size_t)n * nb);   // V of the next panel while this one's update runs
    void *ws2 = ar.take<char>(wsb);        // split-K workspace of the look-ahead stream
    E *Y = ar.take<E>((size_t)n * nb);
    E *X = ar.take<E>((size_t)n * nb);
    E *Gm = ar.take<E>((size_t)nb * nb);
    E *M = ar.take<E>((size_t)nb * nb);
    E *M2 = ar.take<E>((size_t)nb * nb);
    int *flags = ar.take<int>(Gmax + 1);   // Gmax progress flags, then the give-up flag
    CqrScratch cq{};
    const bool use_cq = std::is_same<E, double2>::value;
    if (use_cq) {
        double2 *b = ar.take<double2>((size_t)4 * PNB * PNB + (size_t)std::max(n, 1) * nb);
        cq.G = b; cq.L1 = b + PNB * PNB; cq.X1 = b + 2 * PNB * PNB; cq.M = b + 3 * PNB * PNB;
        cq.Q = b + 4 * PNB * PNB;
        cq.ok = ar.take<int>(1);
    }
    if (ar.measuring() || n == 0) return;
    const E one = El<E>::mk(1.0, 0.0), mone = El<E>::mk(-1.0, 0.0), mhalf = El<E>::mk(-0.5, 0.0);
    zero_async(ctx, T1, (size_t)std::max(np, 1) * nb * nb);
    hipLaunchKernelGGL(fill_int_kernel, dim3(cdiv(Gmax + 1, 256)), dim3(256), 0, ctx->stream, flags, Gmax + 1, 0);
    HGV_LAUNCH_CHECK();
    if (ctx->test_hooks & HGV_TEST_WAIT_FAIL) set_info(ctx, flags + Gmax, 1);
    // concurrent problems: the persistent panel only with a share of the device
    // that every side-by-side panel fits in (see hgv_ctx_s::panel_share)
    const int capacity = !ctx->concurrent         ? panel_persist_capacity<E>(ctx)
                         : ctx->panel_share > 0 ? panel_persist_capacity<E>(ctx) / ctx->panel_share
                                                : 0;
    // Look-ahead (the panel of step p + 1 factored while the update of step p
    // runs, as the paper overlaps its CPU panel with the GPU update): the
    // update first applies to the next panel's columns, then the next panel
    // is factored on a second stream while the main stream updates the rest of
    // the trailing matrix; the streams join before the next update, which
    // reads all of it.  Off while batched problems run side by side.
    const bool la = !ctx->concurrent && np > 1;
    hipStream_t main = ctx->stream;
    if (la) ensure_lookahead_stream(ctx);
    auto factor = [&](int p, hipStream_t st, E *Vp, void *wsp) {
        const int k = p * nb;
        const int jb = std::min(nb, n - k);
        const int N = n - k - nb;
        ctx->stream = st;
        try {
            panel_qr<E>(ctx, A + (k + nb) + (size_t)k * lda, lda, N, jb, tau, part, rowb, Vp, Gm,
                        T1 + (size_t)p * nb * nb, nb, wsp, wsb, flags, flags + Gmax, p * (PNB + 2), capacity,
                        use_cq ? &cq : nullptr);
        } catch (...) {
            ctx->stream = main;
            throw;
        }
        ctx->stream = main;
    };
    if (la) factor(0, main, Vw, ws);
    for (int p = 0; p < np; ++p) {
        const int k = p * nb;
        const int jb = std::min(nb, n - k);
        const int N = n - k - nb;
        const int r = std::min(N, jb);
        E *T = T1 + (size_t)p * nb * nb;
        E *V = (la && (p & 1)) ? Vw2 : Vw;
        if (!la) factor(p, main, Vw, ws);
        E *A22 = A + (k + nb) + (size_t)(k + nb) * lda;
        Gm_t g;
        // Y = V T
        g = Gm_t();
        g.m = N; g.n = r; g.k = r;
        g.A = V; g.lda = N; g.B = T; g.ldb = nb;
        g.C = Y; g.ldc = N;
        gemm_any(ctx, g, ws, wsb);
        // X = A22 Y  (A22 Hermitian, lower triangle stored)
        g = Gm_t();
        g.m = N; g.n = r; g.k = N;
        g.opa = 'H'; g.A = A22; g.lda = lda;
        g.B = Y; g.ldb = N;
        g.C = X; g.ldc = N;
        gemm_any(ctx, g, ws, wsb);
        // M = V^H X
        g = Gm_t();
        g.m = r; g.n = r; g.k = N;
        g.opa = 'C'; g.A = V; g.lda = N;
        g.B = X; g.ldb = N;
        g.C = M; g.ldc = r;
        gemm_any(ctx, g, ws, wsb);
        // M2 = T^H M
        g = Gm_t();
        g.m = r; g.n = r; g.k = r;
        g.opa = 'C'; g.A = T; g.lda = nb;
        g.B = M; g.ldb = r;
        g.C = M2; g.ldc = r;
        gemm_any(ctx, g, ws, wsb);
        // W = X - 1/2 V M2  (into X)
        g = Gm_t();
        g.m = N; g.n = r; g.k = r;
        g.A = V; g.lda = N; g.B = M2; g.ldb = r;
        g.alpha = mhalf; g.beta = one;
        g.C = X; g.ldc = N;
        gemm_any(ctx, g, ws, wsb);
        // A22 <- A22 - V W^H - W V^H (lower)
        auto her2k = [&](int off) {   // rows and columns off.. of A22
            g = Gm_t();
            g.m = N - off; g.n = N - off; g.k = r;
            g.opa = 'N'; g.A = V + off; g.lda = N;
            g.opb = 'C'; g.B = X + off; g.ldb = N;
            g.opa2 = 'N'; g.A2 = X + off; g.lda2 = N;
            g.opb2 = 'C'; g.B2 = V + off; g.ldb2 = N;
            g.alpha = mone; g.beta = one;
            g.C = A22 + off + (size_t)off * lda; g.ldc = lda;
            g.lower = 1;
            gemm_any(ctx, g, ws, wsb);
        };
        if (la && p + 1 < np) {
            const int nbn = std::min(nb, N);   // width of the next panel (its columns lead A22)
            g = Gm_t();   // columns 0 .. nbn-1 of A22, every row at or below the diagonal
            g.m = N; g.n = nbn; g.k = r;
            g.opa = 'N'; g.A = V; g.lda = N;
            g.opb = 'C'; g.B = X; g.ldb = N;
            g.opa2 = 'N'; g.A2 = X; g.lda2 = N;
            g.opb2 = 'C'; g.B2 = V; g.ldb2 = N;
            g.alpha = mone; g.beta = one;
            g.C = A22; g.ldc = lda;
            g.lower = 1;
            gemm_any(ctx, g, ws, wsb);
            HGV_HIP(hipEventRecord(ctx->la_ev[0], main));
            HGV_HIP(hipStreamWaitEvent(ctx->la_stream[0], ctx->la_ev[0], 0));
            factor(p + 1, ctx->la_stream[0], ((p + 1) & 1) ? Vw2 : Vw, ws2);
            HGV_HIP(hipEventRecord(ctx->la_ev[1], ctx->la_stream[0]));
            her2k(nbn);
            HGV_HIP(hipStreamWaitEvent(main, ctx->la_ev[1], 0));
        } else {
            her2k(0);
        }
    }
    if (capacity > 0) report_wait_fail(ctx, flags + Gmax, d_info, 2 * n + 2);
}

// Copy the r x r upper-triangular T (ld nb) into the diagonal block of T_big.
template <class E>
__global__ void place_t_kernel(int r, const E *T, int ldt, E *Tb, int ldb) {
    int i = blockIdx.x * 64 + (threadIdx.x & 63);
    int c = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i >= r || c >= r) return;
    Tb[i + (size_t)c * ldb] = T[i + (size_t)c * ldt];
}

// Q1 = H_0 H_1 ... (one block reflector I - V_p T_p V_p^H per panel) is applied
// in groups of Q1_MERGE consecutive panels merged into one block reflector
// I - V T V^H (V: the panels' reflectors side by side, each panel's block
// starting nb rows below the previous one; T upper triangular with the
// off-diagonal blocks T[0:c, c:c+r] = -T[0:c, 0:c] (V[:, 0:c]^H V[:, c:c+r]) T_p),
// so that every pass over Y has inner dimension merge * nb: 8 panels for many
// columns of Y, 4 for few (building the merged T costs merge^2 nb^2 (n - k)
// per group whatever the number of columns).
constexpr int Q1_MERGE = 8;   // largest merge
static int q1_merge(int m) { return m >= 2048 ? 8 : 4; }

// Y <- Q1 Y = (I - V_0 T_0 V_0^H) ... (I - V_{P-1} T_{P-1} V_{P-1}^H) Y (last
// group first), or Y <- Q1^H Y (first group first, T^H in place of T).
// voff: rows between a panel's first column and its first reflector row (nb for
// the band reduction; 1 for the one-stage tridiagonalisation, whose panel p
// holds the reflectors of columns p*nb .. p*nb+nb-1 from row p*nb + 1 on).
template <class E>
void unmtr_q1_t(hgv_ctx_s *ctx, int n, int nb, int m, const E *A, int lda, const E *T1, E *Y, int ldy, bool adj,
                Arena &ar, int voff) {
    typedef typename El<E>::Gemm Gm_t;
    if (nb > PNB) throw HipFail{hipErrorInvalidValue};
    const int vo = voff > 0 ? voff : nb;
    const int np = (n - vo - 1 >= 0) ? (n - vo - 1) / nb + 1 : 0;
    const int mg = q1_merge(m);
    const int R = mg * nb;
    size_t wsb = zgemm_splitk_bytes(n);
    void *ws = ar.take<char>(wsb);
    E *Vb = ar.take<E>((size_t)std::max(n, 1) * R);
    E *S = ar.take<E>((size_t)R * R);
    E *Tb = ar.take<E>((size_t)R * R);
    E *X = ar.take<E>((size_t)R * nb);
    E *W1 = ar.take<E>((size_t)R * std::max(m, 1));
    E *W2 = ar.take<E>((size_t)R * std::max(m, 1));
    if (ar.measuring() || n == 0 || m == 0 || np == 0) return;
    const E one = El<E>::mk(1.0, 0.0), mone = El<E>::mk(-1.0, 0.0);
    const int ngrp = cdiv(np, mg);
    for (int q = 0; q < ngrp; ++q) {
        const int gi = adj ? q : ngrp - 1 - q;
        const int p0 = gi * mg, p1 = std::min(np, p0 + mg);
        const int k0 = p0 * nb;
        const int Nb = n - k0 - vo;                    // rows of the merged V (start at row k0 + vo)
        if (Nb <= 0) continue;
        // columns of panel p: c_p .. c_p + r_p - 1
        int cols[Q1_MERGE + 1], rs[Q1_MERGE];
        cols[0] = 0;
        for (int p = p0; p < p1; ++p) {
            const int k = p * nb, jb = std::min(nb, n - k), N = n - k - vo;
            rs[p - p0] = std::max(0, std::min(N, jb));
            cols[p - p0 + 1] = cols[p - p0] + rs[p - p0];
        }
        const int Rg = cols[p1 - p0];
        if (Rg == 0) continue;
        zero_async(ctx, Vb, (size_t)Nb * Rg);
        zero_async(ctx, Tb, (size_t)Rg * Rg);
        for (int p = p0; p < p1; ++p) {
            const int k = p * nb, N = n - k - vo, r = rs[p - p0];
            if (r == 0) continue;
            const int off = (p - p0) * nb;
            hipLaunchKernelGGL(extract_v_kernel<E>, dim3(cdiv(N, 64), cdiv(r, 4)), dim3(256), 0, ctx->stream, N, r,
                               A + (k + vo) + (size_t)k * lda, lda, Vb + off + (size_t)cols[p - p0] * Nb, Nb);
            HGV_LAUNCH_CHECK();
            hipLaunchKernelGGL(place_t_kernel<E>, dim3(cdiv(r, 64), cdiv(r, 4)), dim3(256), 0, ctx->stream, r,
                               T1 + (size_t)p * nb * nb, nb, Tb + cols[p - p0] + (size_t)cols[p - p0] * Rg, Rg);
            HGV_LAUNCH_CHECK();
        }
        if (p1 - p0 > 1) {
            Gm_t g;  // S = V^H V
            g.m = Rg; g.n = Rg; g.k = Nb;
            g.opa = 'C'; g.A = Vb; g.lda = Nb;
            g.B = Vb; g.ldb = Nb;
            g.C = S; g.ldc = Rg;
            gemm_any(ctx, g, ws, wsb);
            for (int p = p0 + 1; p < p1; ++p) {
                const int c = cols[p - p0], r = rs[p - p0];
                if (r == 0) continue;
                g = Gm_t();  // X = S[0:c, c:c+r] T_p
                g.m = c; g.n = r; g.k = r;
                g.A = S + (size_t)c * Rg; g.lda = Rg;
                g.B = T1 + (size_t)p * nb * nb; g.ldb = nb;
                g.C = X; g.ldc = c;
                gemm_any(ctx, g, ws, wsb);
                g = Gm_t();  // T[0:c, c:c+r] = -T[0:c, 0:c] X
                g.m = c; g.n = r; g.k = c;
                g.A = Tb; g.lda = Rg;
                g.B = X; g.ldb = c;
                g.alpha = mone;
                g.C = Tb + (size_t)c * Rg; g.ldc = Rg;
                gemm_any(ctx, g, ws, wsb);
            }
        }
        E *Ys = Y + (k0 + vo);
        Gm_t g;  // W1 = V^H Ys
        g.m = Rg; g.n = m; g.k = Nb;
        g.opa = 'C'; g.A = Vb; g.lda = Nb;
        g.B = Ys; g.ldb = ldy;
        g.C = W1; g.ldc = Rg;
        gemm_any(ctx, g, ws, wsb);
        g = Gm_t();  // W2 = T W1  (T^H W1 for Q1^H)
        g.m = Rg; g.n = m; g.k = Rg;
        g.opa = adj ? 'C' : 'N'; g.A = Tb; g.lda = Rg; g.B = W1; g.ldb = Rg;
        g.C = W2; g.ldc = Rg;
        gemm_any(ctx, g, ws, wsb);
        g = Gm_t();  // Ys -= V W2
        g.m = Nb; g.n = m; g.k = Rg;
        g.A = Vb; g.lda = Nb; g.B = W2; g.ldb = Rg;
        g.alpha = mone; g.beta = one;
        g.C = Ys; g.ldc = ldy;
        gemm_any(ctx, g, ws, wsb);
    }
}

template void he2hb_t<double2>(hgv_ctx_s *, int, int, double2 *, int, double2 *, Arena &, int *);
template void he2hb_t<float2>(hgv_ctx_s *, int, int, float2 *, int, float2 *, Arena &, int *);
template void unmtr_q1_t<double2>(hgv_ctx_s *, int, int, int, const double2 *, int, const double2 *, double2 *, int,
                                  bool, Arena &, int);
template void unmtr_q1_t<float2>(hgv_ctx_s *, int, int, int, const float2 *, int, const float2 *, float2 *, int, bool,
                                 Arena &, int);

// T factor of a panel whose r reflectors sit in P (N x r, ldp, unit diagonal
// implicit) with scalars tau (device, double2): explicit V into Vw (N x r),
// G = V^H V into Gm (r x r), then T (ldt) by the column recurrence.
void panel_t_build(hgv_ctx_s *ctx, int N, int r, const double2 *P, int ldp, const double2 *tau, double2 *Vw,
                   double2 *Gm, double2 *T, int ldt, void *ws, size_t wsb) {
    if (N <= 0 || r <= 0) return;
    hipLaunchKernelGGL(extract_v_kernel<double2>, dim3(cdiv(N, 64), cdiv(r, 4)), dim3(256), 0, ctx->stream, N, r, P,
                       ldp, Vw, N);
    HGV_LAUNCH_CHECK();
    ZGemm gg;
    gg.m = r; gg.n = r; gg.k = N;
    gg.opa = 'C'; gg.A = Vw; gg.lda = N;
    gg.opb = 'N'; gg.B = Vw; gg.ldb = N;
    gg.C = Gm; gg.ldc = r;
    zgemm(ctx, gg, static_cast<double2 *>(ws), wsb);
    hipLaunchKernelGGL((build_t_kernel<double2, 1024>), dim3(1), dim3(1024), 0, ctx->stream, r, tau, Gm, r, T, ldt, nullptr);
    HGV_LAUNCH_CHECK();
}

}  // namespace hgv
