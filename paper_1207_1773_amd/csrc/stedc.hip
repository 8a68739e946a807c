// stedc.hip -- divide-and-conquer eigensolver for the real symmetric
// tridiagonal T (Alg. 2 step 2, Sec. 4.3), entirely on the device.
//
// Split: T is torn into leaves of S <= 64 rows; at a boundary with coupling e
// (rows q-1, q) T = diag(T1, T2) + rho v v^T with rho = |e| and
// v = e_{q-1} + sign(e) e_q, so |e| is subtracted from d_{q-1} and d_q.
// Leaves: cyclic Jacobi on the dense leaf block, one workgroup per leaf, the
// disjoint rotations of a round applied in parallel.
// Merge (the displayed identity of Sec. 4.3): with Z1, Z2 the children's
// eigenvectors, T = diag(Z1, Z2) (diag(L1, L2) + rho u u^T) diag(Z1, Z2)^T,
// u = [last row of Z1, sign(e) * first row of Z2]; the rank-one problem
// D + rho u u^T = Q L Q^T is solved here and Z = diag(Z1, Z2) Q is one GEMM
// per child (gemm.hip).  For the rank-one problem:
//   * the two sorted child spectra are merged (ranks by binary search);
//   * deflation: an entry with rho |u_i| <= tol is already an eigenpair;
//     two close entries are rotated so that one component of u vanishes and
//     that entry deflates (the rotation is kept and later applied to Q);
//   * each remaining root lies in (d_j, d_{j+1}) (the last in
//     (d_k, d_k + rho |u|^2)); it is a zero of
//     f(t) = 1 + rho sum u_i^2 / (delta_i - t) with t measured from the
//     nearer pole (delta_i = d_i - d_origin), so t keeps full relative
//     accuracy; found by a bracketed two-pole rational model iteration;
//   * the vector u is recomputed from the computed roots (Gu & Eisenstat,
//     SIAM J. Matrix Anal. Appl. 16 (1995)):
//       u_i^2 = prod_j (l_j - d_i) / (rho prod_{j != i} (d_j - d_i)),
//     which makes the eigenvectors q_j = (u_i / (d_i - l_j))_i / norm
//     numerically orthogonal;
//   * the eigenvalues (roots and deflated entries) are sorted and the columns
//     of Q built in that order; only the wanted columns are built and
//     multiplied in the last merge.
#include <algorithm>
#include <cfloat>

#include "hgv_internal.h"

namespace hgv {

constexpr int DC_LEAF_MAX = 64;   // rows of a leaf (held dense in LDS)

// Leaf size: the fewest doublings that bring the leaves to at most 64 rows,
// with n spread evenly over them, so that the merges at every level (above all
// the last one, which holds most of the flops) pair blocks of nearly equal size
// (n = 10000: leaves of 40 and a last merge of 5120 + 4880, where a fixed
// leaf of 32 rows gave 8192 + 1808).
static int dc_leaf_size(int n) {
    if (n <= DC_LEAF_MAX) return std::max(n, 1);
    int blocks = 1;
    while ((n + blocks - 1) / blocks > DC_LEAF_MAX) blocks *= 2;
    return (n + blocks - 1) / blocks;
}

// Sort key of an eigenvalue: NaN ordered above +inf, so that every ordering
// below is total and the ranks always form a permutation (the index arrays
// built from them stay in range whatever the input holds).
__host__ __device__ inline double dkey(double v) { return v != v ? __builtin_huge_val() : v; }
__host__ __device__ inline bool key_before(double a, int ia, double b, int ib) {
    const double ka = dkey(a), kb = dkey(b);
    const bool na = a != a, nb = b != b;
    return ka < kb || (ka == kb && (na == nb ? ia < ib : nb));
}

struct MergeGeom {
    int a, n1, n2, k;
};

__host__ __device__ inline MergeGeom merge_geom(int n, int L, int p) {
    MergeGeom g;
    g.a = p * 2 * L;
    g.n1 = min(L, n - g.a);
    g.n2 = max(0, min(L, n - g.a - g.n1));
    g.k = g.n1 + g.n2;
    return g;
}

struct DcArgs {
    int n, L, P;
    const double *e;
    double *D;
    const double *Zc;
    int ldz;
    double *ds, *zs;
    int *perm;
    double *dK, *zK;
    int *Kpos, *Dpos;
    int *kcnt, *nrot;
    double *rhop;
    int *rot_p, *rot_i;
    double *rot_c, *rot_s;
    int *org;
    double *tau, *zh, *ival;
    int *colitem;
    double *Q;
    int c_lo, c_hi;   // columns built at this level (last level: wanted range)
    int *info;        // device status (may be null): a secular root that did not converge
    const int *range; // last level with a device-side selection (may be null):
                      // range[0] = first wanted index (1-based), range[2] = columns built
};

__host__ __device__ inline size_t qoff(int L, int p) { return (size_t)p * 4 * (size_t)L * L; }

// ---- leaves -------------------------------------------------------------------------------
// Each leaf block (S <= 64 rows, torn off its neighbours) is diagonalised by the
// cyclic two-sided Jacobi method in one workgroup: the block is held dense in
// LDS and every round applies N/2 disjoint plane rotations at once, the pairs
// taken from a round-robin tournament (index 0 fixed, the others shifted one
// place per round), so that a sweep of N-1 rounds rotates every pair once.
// For a pair (p, q) the rotation [c s; -s c] with t = s/c the smaller root of
// t^2 + 2 tau t - 1 = 0, tau = (a_qq - a_pp) / (2 a_pq), zeroes a_pq
// (Golub & Van Loan, Matrix Computations, Sec. 8.5).  A pair is skipped when
// |a_pq| <= eps sqrt(|a_pp| |a_qq|) (the relative test of Demmel and Veselic,
// SIAM J. Matrix Anal. Appl. 13 (1992)); the sweeps stop when a whole sweep
// skips every pair.  Since the rotations of a round are disjoint, A <- J^T A J
// splits into independent 2 x 2 blocks (rows of pair a, columns of pair b),
// one thread per block, and V <- V J into independent row pairs.
constexpr int JAC_MAX_SWEEPS = 60;

__global__ __launch_bounds__(256) void dc_leaf_kernel(int n, int S, const double *d, const double *e, double *D,
                                                      double *Z, int ldz, int *info) {
    __shared__ double Am[DC_LEAF_MAX][DC_LEAF_MAX + 1];
    __shared__ double Vm[DC_LEAF_MAX][DC_LEAF_MAX + 1];
    __shared__ double rc[DC_LEAF_MAX / 2], rs[DC_LEAF_MAX / 2];
    __shared__ int rp[DC_LEAF_MAX / 2], rq[DC_LEAF_MAX / 2], rk[DC_LEAF_MAX / 2];
    __shared__ int last_rot;   // last sweep that rotated a pair
    __shared__ int rank[DC_LEAF_MAX];
    const int tid = threadIdx.x;
    const int a = blockIdx.x * S;
    const int sz = min(S, n - a);
    const int N = sz + (sz & 1);   // even number of indices; index sz is a dummy when sz is odd
    const int NP = N / 2;
    for (int t = tid; t < DC_LEAF_MAX * DC_LEAF_MAX; t += 256) {
        const int i = t % DC_LEAF_MAX, j = t / DC_LEAF_MAX;
        double v = 0.0;
        if (i < sz && j < sz) {
            if (i == j) {
                v = d[a + i];
                // the tears of the neighbouring boundaries
                if (i == 0 && a > 0) v -= fabs(e[a - 1]);
                if (i == sz - 1 && a + sz < n) v -= fabs(e[a + sz - 1]);
            } else if (i == j + 1) {
                v = e[a + j];
            } else if (j == i + 1) {
                v = e[a + i];
            }
        }
        Am[i][j] = v;
        Vm[i][j] = (i == j) ? 1.0 : 0.0;
    }
    if (tid == 0) last_rot = -1;
    __syncthreads();
    int sweep = 0;
    for (; sweep < JAC_MAX_SWEEPS; ++sweep) {
        for (int r = 0; r < N - 1; ++r) {
            // ---- rotation of every pair of this round ----
            if (tid < NP) {
                const int x = (tid == 0) ? 0 : 1 + (tid - 1 + r) % (N - 1);
                const int y = 1 + (N - 2 - tid + r) % (N - 1);
                const int p = min(x, y), q = max(x, y);
                double c = 1.0, s = 0.0;
                int rot = 0;
                if (q < sz) {
                    const double apq = Am[p][q], app = Am[p][p], aqq = Am[q][q];
                    if (fabs(apq) > DBL_EPSILON * sqrt(fabs(app)) * sqrt(fabs(aqq))) {
                        const double tau = (aqq - app) / (2.0 * apq);
                        // for |tau| so large that tau^2 would overflow, t = 1/(2 tau) to working precision
                        const double t = fabs(tau) > 1e150 ? 0.5 / tau
                                                           : copysign(1.0, tau) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + t * t);
                        s = t * c;
                        rot = 1;
                        last_rot = sweep;
                    }
                }
                rp[tid] = p;
                rq[tid] = q;
                rc[tid] = c;
                rs[tid] = s;
                rk[tid] = rot;
            }
            __syncthreads();
            // ---- A <- J^T A J by 2 x 2 blocks, V <- V J by row pairs ----
            for (int t = tid; t < NP * NP; t += 256) {
                const int ia = t % NP, ib = t / NP;
                const int pa = rp[ia], qa = rq[ia], pb = rp[ib], qb = rq[ib];
                const double ca = rc[ia], sa = rs[ia], cb = rc[ib], sb = rs[ib];
                const double m00 = Am[pa][pb], m01 = Am[pa][qb], m10 = Am[qa][pb], m11 = Am[qa][qb];
                const double t00 = ca * m00 - sa * m10, t01 = ca * m01 - sa * m11;
                const double t10 = sa * m00 + ca * m10, t11 = sa * m01 + ca * m11;
                double n00 = cb * t00 - sb * t01, n01 = sb * t00 + cb * t01;
                double n10 = cb * t10 - sb * t11, n11 = sb * t10 + cb * t11;
                if (ia == ib && rk[ia]) {
                    // the rotated pair: exact zero off the diagonal
                    const double tt = sa / ca;
                    n00 = m00 - tt * m01;
                    n11 = m11 + tt * m01;
                    n01 = 0.0;
                    n10 = 0.0;
                }
                Am[pa][pb] = n00;
                Am[pa][qb] = n01;
                Am[qa][pb] = n10;
                Am[qa][qb] = n11;
            }
            for (int t = tid; t < sz * NP; t += 256) {
                const int i = t % sz, ib = t / sz;
                const int pb = rp[ib], qb = rq[ib];
                const double cb = rc[ib], sb = rs[ib];
                const double vp = Vm[i][pb], vq = Vm[i][qb];
                Vm[i][pb] = cb * vp - sb * vq;
                Vm[i][qb] = sb * vp + cb * vq;
            }
            __syncthreads();
        }
        // no pair rotated in this sweep: converged.  (A thread that is already in
        // the next sweep can only have raised last_rot further, so the test is
        // the same in every thread.)
        if (last_rot < sweep) break;
    }
    if (sweep == JAC_MAX_SWEEPS && tid == 0 && info) atomicCAS(info, 0, a + 1);
    // ascending order (rank by counting, ties by index); D and the block of Z
    if (tid < sz) {
        const double v = Am[tid][tid];
        int r = 0;
        for (int j = 0; j < sz; ++j) r += key_before(Am[j][j], j, v, tid) ? 1 : 0;
        rank[tid] = r;
        D[a + r] = v;
    }
    __syncthreads();
    for (int t = tid; t < sz * sz; t += 256) {
        const int i = t % sz, c = t / sz;
        Z[(a + i) + (size_t)(a + rank[c]) * ldz] = Vm[i][c];
    }
}

// ---- merge steps ------------------------------------------------------------------------------
// M1: u (normalised later) and the merged order of the two sorted child spectra.
__global__ void dc_m1_kernel(DcArgs A) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= A.n) return;
    int p = g / (2 * A.L);
    MergeGeom m = merge_geom(A.n, A.L, p);
    if (m.n2 <= 0) return;
    int x = g - m.a;
    double lam = A.D[g];
    double sig = (A.e[m.a + m.n1 - 1] >= 0.0) ? 1.0 : -1.0;
    double z = (x < m.n1) ? A.Zc[(m.a + m.n1 - 1) + (size_t)g * A.ldz] : sig * A.Zc[(m.a + m.n1) + (size_t)g * A.ldz];
    // (each child is sorted by key_before; ties between the children go left first)
    int rank;
    if (x < m.n1) {   // count right entries strictly below lam
        const double *R = A.D + m.a + m.n1;
        int lo = 0, hi = m.n2;
        while (lo < hi) { int mid = (lo + hi) >> 1; if (key_before(R[mid], 1, lam, 0)) lo = mid + 1; else hi = mid; }
        rank = x + lo;
    } else {          // count left entries <= lam
        const double *Lf = A.D + m.a;
        int lo = 0, hi = m.n1;
        while (lo < hi) { int mid = (lo + hi) >> 1; if (key_before(Lf[mid], 0, lam, 1)) lo = mid + 1; else hi = mid; }
        rank = (x - m.n1) + lo;
    }
    A.ds[m.a + rank] = lam;
    A.zs[m.a + rank] = z;
    A.perm[m.a + rank] = x;
}

// M2: normalise u, deflation scan.  The norm of z and the largest |d| are
// reduced by the workgroup (a fixed-order tree, the same in every run); the
// scan itself is serial in sorted order: thread 0 walks chunks of the merge
// that the workgroup has copied into LDS (z already scaled), so that its
// loads are LDS reads and its global stores never wait for them.  The scan
// changes only the entries at `prev` and `i`; the current values of `prev`
// stay in registers, and a `prev` left behind in an earlier chunk is written
// back to global memory directly.
constexpr int M2CH = 2048;

__global__ __launch_bounds__(256) void dc_m2_kernel(DcArgs A) {
    __shared__ double sd[M2CH], sz[M2CH];
    __shared__ double rs[256], rm[256];
    const int p = blockIdx.x, tid = threadIdx.x;
    const MergeGeom m = merge_geom(A.n, A.L, p);
    if (m.n2 <= 0) return;
    double *ds = A.ds + m.a, *zs = A.zs + m.a;
    double nz2 = 0.0, dmax = 0.0;
    for (int i = tid; i < m.k; i += 256) {
        nz2 += zs[i] * zs[i];
        dmax = fmax(dmax, fabs(ds[i]));
    }
    rs[tid] = nz2;
    rm[tid] = dmax;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) {
            rs[tid] += rs[tid + o];
            rm[tid] = fmax(rm[tid], rm[tid + o]);
        }
        __syncthreads();
    }
    nz2 = rs[0];
    dmax = rm[0];
    const double rho = fabs(A.e[m.a + m.n1 - 1]);
    const double rhop = rho * nz2;
    const double inv = nz2 > 0.0 ? 1.0 / sqrt(nz2) : 0.0;
    const double tol = 8.0 * DBL_EPSILON * fmax(dmax, rhop);
    int kk = 0, nd = 0, nr = 0, prev = -1;
    double dprev = 0.0, zprev = 0.0;   // current values of entry prev (thread 0)
    for (int c0 = 0; c0 < m.k; c0 += M2CH) {
        const int cn = min(M2CH, m.k - c0);
        __syncthreads();   // the previous chunk is written back
        for (int i = tid; i < cn; i += 256) {
            sd[i] = ds[c0 + i];
            sz[i] = zs[c0 + i] * inv;
        }
        __syncthreads();
        if (tid == 0) {
            for (int il = 0; il < cn; ++il) {
                const int i = c0 + il;
                const double di = sd[il], zi = sz[il];
                if (rhop * fabs(zi) <= tol) {
                    A.Dpos[m.a + nd++] = i;
                    continue;
                }
                if (prev < 0) {
                    prev = i;
                    dprev = di;
                    zprev = zi;
                    continue;
                }
                double s = zprev, c = zi;
                const double r = hypot(c, s);
                c /= r;
                s /= r;
                const double t = di - dprev;
                if (fabs(t * c * s) <= tol) {
                    const double dp = dprev * c * c + di * s * s;
                    const double dn = dprev * s * s + di * c * c;
                    if (prev >= c0) {
                        sd[prev - c0] = dp;
                        sz[prev - c0] = 0.0;
                    } else {
                        ds[prev] = dp;
                        zs[prev] = 0.0;
                    }
                    sd[il] = dn;
                    sz[il] = r;
                    A.rot_p[m.a + nr] = prev;
                    A.rot_i[m.a + nr] = i;
                    A.rot_c[m.a + nr] = c;
                    A.rot_s[m.a + nr] = s;
                    ++nr;
                    A.Dpos[m.a + nd++] = prev;
                    prev = i;
                    dprev = dn;
                    zprev = r;
                } else {
                    A.Kpos[m.a + kk] = prev;
                    A.dK[m.a + kk] = dprev;
                    A.zK[m.a + kk] = zprev;
                    ++kk;
                    prev = i;
                    dprev = di;
                    zprev = zi;
                }
            }
        }
        __syncthreads();
        for (int i = tid; i < cn; i += 256) {
            ds[c0 + i] = sd[i];
            zs[c0 + i] = sz[i];
        }
    }
    if (tid == 0) {
        if (prev >= 0) {
            A.Kpos[m.a + kk] = prev;
            A.dK[m.a + kk] = dprev;
            A.zK[m.a + kk] = zprev;
            ++kk;
        }
        A.kcnt[p] = kk;
        A.nrot[p] = nr;
        A.rhop[p] = rhop;
    }
}

// M3: secular roots.  Root j lies in (d_j, d_{j+1}) (last root: right of d_k);
// t is measured from the nearer pole (origin).  Each iteration fits the model
//   f(x) ~ c + sL / (pL - x) + sR / (pR - x)
// to the value and the two partial derivatives of f at the iterate (sL from
// the terms at or left of the left pole, sR from the rest; pL, pR the poles of
// the interval) and takes the model's root (a quadratic) as the next iterate;
// a bracket [lo, hi] with f(lo) < 0 < f(hi) is kept, and the step falls back
// to bisection when the model root leaves it or every fourth iteration.  The
// iteration stops when |f| is below its rounding-error bound.
// A group of M3G consecutive lanes works on one root: lane `sub` of the group
// sums the terms i = sub, sub + M3G, ... (four loads in flight), and an xor
// butterfly over the group adds the partial sums.  Floating-point addition is
// commutative, so every lane of the group ends with the same sums bit for bit
// and takes the same branches of the iteration.
constexpr int M3G = 32;

__device__ inline double group_add(double x) {
#pragma unroll
    for (int o = 1; o < M3G; o <<= 1) x += __shfl_xor(x, o, M3G);
    return x;
}

__device__ inline void secular_eval(const double *dK, const double *zK, int kp, double dorg, double rho, double t,
                                    int split, int sub, double &f, double &dl, double &dr, double &err) {
    double psi = 0.0, phi = 0.0, dpsi = 0.0, dphi = 0.0;
    for (int i0 = sub; i0 < kp; i0 += 4 * M3G) {
        double dv[4], zv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = i0 + u * M3G;
            dv[u] = dK[i < kp ? i : 0];
            zv[u] = zK[i < kp ? i : 0];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = i0 + u * M3G;
            const double z = (i < kp) ? zv[u] : 0.0;
            const double del = (dv[u] - dorg) - t;
            const double q = z / del;
            const double term = z * q, dterm = q * q;
            if (i <= split) {
                psi += term;
                dpsi += dterm;
            } else {
                phi += term;
                dphi += dterm;
            }
        }
    }
    psi = group_add(psi);
    phi = group_add(phi);
    dpsi = group_add(dpsi);
    dphi = group_add(dphi);
    f = 1.0 + rho * (psi + phi);
    dl = rho * dpsi;
    dr = rho * dphi;
    err = 8.0 * DBL_EPSILON * (1.0 + rho * (fabs(psi) + fabs(phi)) + fabs(t) * (dl + dr)) * (double)(kp > 8 ? 8 : kp);
}

__global__ void dc_m3_kernel(DcArgs A) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int root = g / M3G, sub = g % M3G;
    // every exit below is taken by whole lane groups (it depends on root only)
    if (root >= A.n) return;
    int p = root / (2 * A.L);
    MergeGeom m = merge_geom(A.n, A.L, p);
    if (m.n2 <= 0) return;
    int j = root - m.a;
    int kp = A.kcnt[p];
    if (j >= kp) return;
    const double *dK = A.dK + m.a, *zK = A.zK + m.a;
    double rho = A.rhop[p];
    int org;
    double lo, hi;
    if (j < kp - 1) {
        double mid = 0.5 * (dK[j + 1] - dK[j]);
        double fs = 0.0;
        for (int i = sub; i < kp; i += M3G) fs += zK[i] * zK[i] / ((dK[i] - dK[j]) - mid);
        double f = 1.0 + rho * group_add(fs);
        if (f >= 0.0) { org = j; lo = 0.0; hi = mid; }
        else { org = j + 1; lo = -mid; hi = 0.0; }
    } else {
        double s2 = 0.0;
        for (int i = sub; i < kp; i += M3G) s2 += zK[i] * zK[i];
        org = j; lo = 0.0; hi = rho * group_add(s2);
    }
    const double dorg = dK[org];
    const bool last = (j == kp - 1);
    const double pL = dK[j] - dorg;                          // left pole (relative)
    const double pR = last ? 0.0 : dK[j + 1] - dorg;          // right pole (relative)
    double t = 0.5 * (lo + hi);
    bool conv = false;
    for (int it = 0; it < 200; ++it) {
        double f, sl, sr, err;
        secular_eval(dK, zK, kp, dorg, rho, t, j, sub, f, sl, sr, err);
        if (fabs(f) <= err) { conv = true; break; }
        if (f < 0.0) lo = t;
        else hi = t;
        if (hi - lo <= 4.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi))) { conv = true; break; }
        double tn = 0.5 * (lo + hi);   // bisection fallback
        if ((it & 3) != 3) {
            // model weights from the derivatives at t
            double aL = (pL - t), aR = (pR - t);
            double wL = aL * aL * sl;                        // >= 0
            if (last) {
                double c = f - wL / aL;                      // model: c + wL / (pL - x) = 0
                if (c > 0.0) tn = pL + wL / c;
            } else {
                double wR = aR * aR * sr;
                double c = f - wL / aL - wR / aR;
                double w = pR - pL;
                // u = x - pL solves c u^2 - (c w + wL + wR) u + wL w = 0 on (0, w)
                double qa = c, qb = -(c * w + wL + wR), qc = wL * w;
                double disc = qb * qb - 4.0 * qa * qc;
                if (disc >= 0.0) {
                    double sq = sqrt(disc);
                    double u;
                    if (qa == 0.0) u = -qc / qb;
                    else if (qb <= 0.0) {
                        double u1 = (-qb + sq) / (2.0 * qa), u2 = (2.0 * qc) / (-qb + sq);
                        u = (u2 > 0.0 && u2 < w) ? u2 : u1;
                    } else {
                        double u1 = (2.0 * qc) / (-qb - sq), u2 = (-qb - sq) / (2.0 * qa);
                        u = (u1 > 0.0 && u1 < w) ? u1 : u2;
                    }
                    tn = pL + u;
                }
            }
            if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
        }
        if (tn == t) { conv = true; break; }
        t = tn;
    }
    if (sub == 0) {
        A.org[m.a + j] = org;
        A.tau[m.a + j] = t;
        // the iteration ran out without meeting a stopping test: report the root
        // (its index in the merged block's order, 1-based) unless a failure is
        // already recorded
        if (!conv && A.info) atomicCAS(A.info, 0, m.a + j + 1);
    }
}

__device__ inline double group_mul(double x) {
#pragma unroll
    for (int o = 1; o < M3G; o <<= 1) x *= __shfl_xor(x, o, M3G);
    return x;
}

// M4: Gu-Eisenstat recomputation of u from the computed roots.
// One group of M3G lanes per element (as for the roots): lane `sub` multiplies
// the factors j = sub, sub + M3G, ..., and an xor butterfly multiplies the
// partial products (multiplication commutes, so every lane of the group ends
// with the same product).
__global__ void dc_m4_kernel(DcArgs A) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int gi = g / M3G, sub = g % M3G;
    // every exit below is taken by whole lane groups (it depends on gi only)
    if (gi >= A.n) return;
    int p = gi / (2 * A.L);
    MergeGeom m = merge_geom(A.n, A.L, p);
    if (m.n2 <= 0) return;
    int i = gi - m.a;
    int kp = A.kcnt[p];
    if (i >= kp) return;
    const double *dK = A.dK + m.a;
    const int *org = A.org + m.a;
    const double *tau = A.tau + m.a;
    double di = dK[i];
    double prod = 1.0;
    for (int j = sub; j < kp; j += M3G) {
        if (j == i) continue;
        prod *= ((dK[org[j]] - di) + tau[j]) / (dK[j] - di);
    }
    prod = group_mul(prod) * (((dK[org[i]] - di) + tau[i]) / A.rhop[p]);
    if (sub == 0) A.zh[m.a + i] = copysign(sqrt(fabs(prod)), A.zK[m.a + i]);
}

// M5: eigenvalue of every item (roots first, then deflated entries).
__global__ void dc_m5_kernel(DcArgs A) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= A.n) return;
    int p = g / (2 * A.L);
    MergeGeom m = merge_geom(A.n, A.L, p);
    if (m.n2 <= 0) return;
    int x = g - m.a;
    int kp = A.kcnt[p];
    double v = (x < kp) ? A.dK[m.a + A.org[m.a + x]] + A.tau[m.a + x] : A.ds[m.a + A.Dpos[m.a + x - kp]];
    A.ival[m.a + x] = v;
}

// M6: sort the items (rank by counting, ties by item index); new spectrum into D.
// One group of M3G lanes per element: lane `sub` counts over y = sub, sub + M3G,
// ..., and the group adds the counts (integers: the rank is exact).
__global__ void dc_m6_kernel(DcArgs A) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int gi = g / M3G, sub = g % M3G;
    // every exit below is taken by whole lane groups (it depends on gi only)
    if (gi >= A.n) return;
    int p = gi / (2 * A.L);
    MergeGeom m = merge_geom(A.n, A.L, p);
    if (m.n2 <= 0) return;
    int x = gi - m.a;
    const double *iv = A.ival + m.a;
    double v = iv[x];
    int r = 0;
    for (int y = sub; y < m.k; y += M3G) r += key_before(iv[y], y, v, x) ? 1 : 0;
#pragma unroll
    for (int o = 1; o < M3G; o <<= 1) r += __shfl_xor(r, o, M3G);
    if (sub == 0) {
        A.D[m.a + r] = v;
        A.colitem[m.a + r] = x;
    }
}

// M7: column `col` of Q (rows in the children's order).  The column is built
// in the sorted basis (in LDS when it fits), the deflation rotations are
// applied in reverse order, then rows are scattered through perm.
template <int KCAP>
__global__ __launch_bounds__(256) void dc_m7_kernel(DcArgs A, int p_fixed) {
    __shared__ double col_s[KCAP > 0 ? KCAP : 1];
    __shared__ double red[256];
    int p, col, slot;
    bool unused = false;   // a slot beyond a device-side selection: zero column
    if (p_fixed >= 0) {
        p = p_fixed;
        slot = blockIdx.x;
        if (A.range) {
            col = A.range[0] - 1 + slot;
            unused = slot >= A.range[2];
        } else {
            col = A.c_lo + slot;
        }
    } else {
        int g = blockIdx.x;
        p = g / (2 * A.L);
        col = g - p * 2 * A.L;
        slot = col;
    }
    MergeGeom m = merge_geom(A.n, A.L, p);
    if (m.n2 <= 0) return;
    const int tid = threadIdx.x;
    double *Qc = A.Q + qoff(A.L, p) + (size_t)slot * m.k;
    if (unused) {
        for (int i = tid; i < m.k; i += 256) Qc[i] = 0.0;
        return;
    }
    if (col >= m.k) return;
    const int kp = A.kcnt[p];
    const int x = A.colitem[m.a + col];
    const int *perm = A.perm + m.a;
    // sorted-basis column: KCAP > 0 -> LDS; else written straight to permuted rows
    double inv = 1.0;
    double dorg = 0.0, tx = 0.0;
    if (x < kp) {
        dorg = A.dK[m.a + A.org[m.a + x]];
        tx = A.tau[m.a + x];
        double ss = 0.0;
        for (int i = tid; i < kp; i += 256) {
            double v = A.zh[m.a + i] / ((A.dK[m.a + i] - dorg) - tx);
            ss += v * v;
        }
        red[tid] = ss;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (tid < o) red[tid] += red[tid + o];
            __syncthreads();
        }
        inv = 1.0 / sqrt(red[0]);
    }
    if (KCAP > 0) {
        for (int i = tid; i < m.k; i += 256) col_s[i] = 0.0;
        __syncthreads();
        if (x < kp) {
            for (int i = tid; i < kp; i += 256)
                col_s[A.Kpos[m.a + i]] = inv * A.zh[m.a + i] / ((A.dK[m.a + i] - dorg) - tx);
        } else if (tid == 0) {
            col_s[A.Dpos[m.a + x - kp]] = 1.0;
        }
        __syncthreads();
        if (tid == 0) {
            for (int t = A.nrot[p] - 1; t >= 0; --t) {
                int pr = A.rot_p[m.a + t], ir = A.rot_i[m.a + t];
                double c = A.rot_c[m.a + t], s = A.rot_s[m.a + t];
                double qp = col_s[pr], qi = col_s[ir];
                col_s[pr] = c * qp + s * qi;
                col_s[ir] = -s * qp + c * qi;
            }
        }
        __syncthreads();
        for (int i = tid; i < m.k; i += 256) Qc[perm[i]] = col_s[i];
    } else {
        for (int i = tid; i < m.k; i += 256) Qc[i] = 0.0;
        __syncthreads();
        if (x < kp) {
            for (int i = tid; i < kp; i += 256)
                Qc[perm[A.Kpos[m.a + i]]] = inv * A.zh[m.a + i] / ((A.dK[m.a + i] - dorg) - tx);
        } else if (tid == 0) {
            Qc[perm[A.Dpos[m.a + x - kp]]] = 1.0;
        }
        __threadfence_block();
        __syncthreads();
        if (tid == 0) {
            for (int t = A.nrot[p] - 1; t >= 0; --t) {
                int pr = perm[A.rot_p[m.a + t]], ir = perm[A.rot_i[m.a + t]];
                double c = A.rot_c[m.a + t], s = A.rot_s[m.a + t];
                double qp = Qc[pr], qi = Qc[ir];
                Qc[pr] = c * qp + s * qi;
                Qc[ir] = -s * qp + c * qi;
            }
        }
    }
}

__global__ void dcopy2d_kernel(int m, int n, const double *A, int lda, double *B, int ldb) {
    int i = blockIdx.x * 64 + (threadIdx.x & 63);
    int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i < m && j < n) B[i + (size_t)j * ldb] = A[i + (size_t)j * lda];
}

__global__ void dcopy_kernel(int n, const double *a, double *b) {
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) b[i] = a[i];
}

// Z[:, j] = Zc[:, range[0] - 1 + j] for j < range[2], zero for the other slots.
__global__ void dselect_cols_kernel(int n, int nslot, const double *Zc, int ldzc, const int *range, double *Z,
                                    int ldz) {
    int i = blockIdx.x * 64 + (threadIdx.x & 63);
    int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i >= n || j >= nslot) return;
    Z[i + (size_t)j * ldz] = j < range[2] ? Zc[i + (size_t)(range[0] - 1 + j) * ldzc] : 0.0;
}

static void dcopy2d(hgv_ctx_s *ctx, int m, int n, const double *A, int lda, double *B, int ldb) {
    if (m <= 0 || n <= 0) return;
    hipLaunchKernelGGL(dcopy2d_kernel, dim3(cdiv(m, 64), cdiv(n, 4)), dim3(256), 0, ctx->stream, m, n, A, lda, B, ldb);
    HGV_LAUNCH_CHECK();
}

void stedc_run(hgv_ctx_s *ctx, int n, const double *d, const double *e, int il, int iu, double *lambda, double *Z,
               int ldz, Arena &ar, int *d_info, const std::function<void()> &at_last_level, const int *d_range) {
    const int S = dc_leaf_size(n);
    const int m = iu - il + 1;
    // Q buffer: the largest level's sum of k^2 with offsets p * 4 L^2
    size_t qmax = 1;
    for (int L = S; L < n; L *= 2) {
        int P = cdiv(n, 2 * L);
        MergeGeom last = merge_geom(n, L, P - 1);
        size_t need = (P - 1 > 0 ? qoff(L, P - 1) : 0) + (size_t)last.k * last.k;
        qmax = std::max(qmax, need);
    }
    double *Za = ar.take<double>((size_t)n * n);
    double *Zb = ar.take<double>((size_t)n * n);
    double *Qb = ar.take<double>(qmax);
    double *D = ar.take<double>(n);
    double *ds = ar.take<double>(n), *zs = ar.take<double>(n);
    int *perm = ar.take<int>(n);
    double *dK = ar.take<double>(n), *zK = ar.take<double>(n);
    int *Kpos = ar.take<int>(n), *Dpos = ar.take<int>(n);
    int np = cdiv(std::max(n, 1), 2 * S) + 1;
    int *kcnt = ar.take<int>(np), *nrot = ar.take<int>(np);
    double *rhop = ar.take<double>(np);
    int *rot_p = ar.take<int>(n), *rot_i = ar.take<int>(n);
    double *rot_c = ar.take<double>(n), *rot_s = ar.take<double>(n);
    int *org = ar.take<int>(n);
    double *tau = ar.take<double>(n), *zh = ar.take<double>(n), *ival = ar.take<double>(n);
    int *colitem = ar.take<int>(n);
    if (ar.measuring() || n == 0) return;

    const int nleaf = cdiv(n, S);
    hipLaunchKernelGGL(dc_leaf_kernel, dim3(nleaf), dim3(256), 0, ctx->stream, n, S, d, e, D, Za, n, d_info);
    HGV_LAUNCH_CHECK();
    double *Zc = Za, *Zn = Zb;
    if (n <= S) {
        if (d_range) {
            hipLaunchKernelGGL(dselect_cols_kernel, dim3(cdiv(n, 64), cdiv(m, 4)), dim3(256), 0, ctx->stream, n, m,
                               Zc, n, d_range, Z, ldz);
            HGV_LAUNCH_CHECK();
        } else {
            dcopy2d(ctx, n, m, Zc + (size_t)(il - 1) * n, n, Z, ldz);
        }
        hipLaunchKernelGGL(dcopy_kernel, dim3(cdiv(n, 256)), dim3(256), 0, ctx->stream, n, D, lambda);
        HGV_LAUNCH_CHECK();
        return;
    }
    for (int L = S; L < n; L *= 2) {
        const int P = cdiv(n, 2 * L);
        const bool last = (2 * L >= n);
        if (last && at_last_level) at_last_level();
        DcArgs A;
        A.n = n; A.L = L; A.P = P; A.e = e; A.D = D; A.Zc = Zc; A.ldz = n;
        A.ds = ds; A.zs = zs; A.perm = perm; A.dK = dK; A.zK = zK; A.Kpos = Kpos; A.Dpos = Dpos;
        A.kcnt = kcnt; A.nrot = nrot; A.rhop = rhop;
        A.rot_p = rot_p; A.rot_i = rot_i; A.rot_c = rot_c; A.rot_s = rot_s;
        A.org = org; A.tau = tau; A.zh = zh; A.ival = ival; A.colitem = colitem; A.Q = Qb;
        A.c_lo = last ? il - 1 : 0;
        A.c_hi = last ? iu : 2 * L;
        A.info = d_info;
        A.range = last ? d_range : nullptr;
        dim3 gN(cdiv(n, 256));
        hipLaunchKernelGGL(dc_m1_kernel, gN, dim3(256), 0, ctx->stream, A);
        HGV_LAUNCH_CHECK();
        hipLaunchKernelGGL(dc_m2_kernel, dim3(P), dim3(256), 0, ctx->stream, A);
        HGV_LAUNCH_CHECK();
        hipLaunchKernelGGL(dc_m3_kernel, dim3(cdiv(n * M3G, 256)), dim3(256), 0, ctx->stream, A);
        HGV_LAUNCH_CHECK();
        hipLaunchKernelGGL(dc_m4_kernel, dim3(cdiv(n * M3G, 256)), dim3(256), 0, ctx->stream, A);
        HGV_LAUNCH_CHECK();
        hipLaunchKernelGGL(dc_m5_kernel, gN, dim3(256), 0, ctx->stream, A);
        HGV_LAUNCH_CHECK();
        hipLaunchKernelGGL(dc_m6_kernel, dim3(cdiv(n * M3G, 256)), dim3(256), 0, ctx->stream, A);
        HGV_LAUNCH_CHECK();
        const int kmax = std::min(2 * L, n);
        if (last) {
            int ncols = m;
            if (kmax <= 1024)
                hipLaunchKernelGGL((dc_m7_kernel<1024>), dim3(ncols), dim3(256), 0, ctx->stream, A, 0);
            else if (kmax <= 16384)
                hipLaunchKernelGGL((dc_m7_kernel<16384>), dim3(ncols), dim3(256), 0, ctx->stream, A, 0);
            else
                hipLaunchKernelGGL((dc_m7_kernel<0>), dim3(ncols), dim3(256), 0, ctx->stream, A, 0);
        } else {
            int ncols = P * 2 * L;
            if (kmax <= 1024)
                hipLaunchKernelGGL((dc_m7_kernel<1024>), dim3(ncols), dim3(256), 0, ctx->stream, A, -1);
            else if (kmax <= 16384)
                hipLaunchKernelGGL((dc_m7_kernel<16384>), dim3(ncols), dim3(256), 0, ctx->stream, A, -1);
            else
                hipLaunchKernelGGL((dc_m7_kernel<0>), dim3(ncols), dim3(256), 0, ctx->stream, A, -1);
        }
        HGV_LAUNCH_CHECK();
        // the products of a level are independent of each other: they are dealt
        // round-robin to the solve's stream and its two side streams (many of
        // them are small), which join before the next level
        const bool fan = !ctx->concurrent;
        hipStream_t main = ctx->stream;
        if (fan) {
            ensure_lookahead_stream(ctx);
            HGV_HIP(hipEventRecord(ctx->la_ev[0], main));
            for (hipStream_t st : ctx->la_stream) HGV_HIP(hipStreamWaitEvent(st, ctx->la_ev[0], 0));
        }
        int gi = 0;
        auto dgemm_rr = [&](int mm, int nn, int kk, const double *Am, int ldam, const double *Bm, int ldbm,
                            double *Cm, int ldcm) {
            ctx->stream = fan && gi % 3 ? ctx->la_stream[gi % 3 - 1] : main;
            ++gi;
            try {
                dgemm_nn(ctx, mm, nn, kk, 1.0, Am, ldam, Bm, ldbm, 0.0, Cm, ldcm);
            } catch (...) {
                ctx->stream = main;
                throw;
            }
            ctx->stream = main;
        };
        for (int p = 0; p < P; ++p) {
            MergeGeom g = merge_geom(n, L, p);
            if (g.n2 <= 0) {   // unpaired block: carried over unchanged
                if (!last) dcopy2d(ctx, g.n1, g.n1, Zc + g.a + (size_t)g.a * n, n, Zn + g.a + (size_t)g.a * n, n);
                continue;
            }
            const double *Qp = Qb + qoff(L, p);
            if (last) {
                // wanted columns only, straight into the output
                dgemm_rr(g.n1, m, g.n1, Zc + g.a + (size_t)g.a * n, n, Qp, g.k, Z + g.a, ldz);
                dgemm_rr(g.n2, m, g.n2, Zc + (g.a + g.n1) + (size_t)(g.a + g.n1) * n, n, Qp + g.n1, g.k,
                         Z + g.a + g.n1, ldz);
            } else {
                dgemm_rr(g.n1, g.k, g.n1, Zc + g.a + (size_t)g.a * n, n, Qp, g.k, Zn + g.a + (size_t)g.a * n, n);
                dgemm_rr(g.n2, g.k, g.n2, Zc + (g.a + g.n1) + (size_t)(g.a + g.n1) * n, n, Qp + g.n1, g.k,
                         Zn + (g.a + g.n1) + (size_t)g.a * n, n);
            }
        }
        if (fan) {
            HGV_HIP(hipEventRecord(ctx->la_ev[2], ctx->la_stream[0]));
            HGV_HIP(hipEventRecord(ctx->la_ev[3], ctx->la_stream[1]));
            HGV_HIP(hipStreamWaitEvent(main, ctx->la_ev[2], 0));
            HGV_HIP(hipStreamWaitEvent(main, ctx->la_ev[3], 0));
        }
        std::swap(Zc, Zn);
        if (last) break;
    }
    hipLaunchKernelGGL(dcopy_kernel, dim3(cdiv(n, 256)), dim3(256), 0, ctx->stream, n, D, lambda);
    HGV_LAUNCH_CHECK();
}

}  // namespace hgv
