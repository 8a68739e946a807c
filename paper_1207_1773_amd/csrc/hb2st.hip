// hb2st.hip -- second stage of the two-stage tridiagonalisation (Alg. 2
// step 1, Sec. 4.2): column-wise bulge chasing of the Hermitian band of width
// b to a real symmetric tridiagonal, and the matching back-transformation
// Y <- Q2 Y of Alg. 2 step 3 (the first of the two back-transformation steps
// the two-stage approach needs).
//
// Sweep s annihilates column s below its first subdiagonal.  Its task j acts
// on the rows I_j = [s+1+j*b, s+(j+1)*b] (clipped to n):
//   j = 0: reflector H_{s,0} from column s (rows I_0), applied on both sides
//          of the diagonal block A[I_0, I_0];
//   j > 0: the previous reflector is applied from the right to the block
//          E = A[I_j, I_{j-1}] (this creates the bulge), H_{s,j} is generated
//          from E's first column and applied from the left to E, then on both
//          sides of A[I_j, I_j].
// Every reflector H = I - tau v v^H maps its vector onto beta e_1 with beta
// real, so the resulting tridiagonal is real.  Band storage keeps the lower
// triangle with offsets 0 .. 2b-1 (the bulge reaches offset 2b-1):
// element (r, c), r >= c, at AB[(r - c) + c * 2b].
//
// Parallel schedule (one persistent workgroup per sweep at a time, sweeps
// dealt round-robin, all workgroups co-resident by a cooperative launch):
// task (s, j) touches rows/columns that overlap those of
// task (s-1, j+1) but of no later task of sweep s-1, so it starts once sweep
// s-1 has completed min(j+2, all) tasks.  Tasks that may run concurrently
// touch disjoint data, and every task's arithmetic is fixed, so the result
// equals the sequential one bit for bit.  Progress counters are published
// with release stores and read with acquire loads at device (agent) scope.
//
// Q2 back-transformation: the reflectors H_{s,j} of g = min(b, 32)
// consecutive sweeps s0 .. s0+g-1 at the same step j occupy a (g+b-1) x g
// parallelogram of rows; their product H_{s0} ... H_{s0+g-1} = I - V T V^H
// (compact WY).
// Applying Q2 = prod_s prod_j H_{s,j} to Y is the same as applying the
// groups block by block from the last block of sweeps to the first and,
// within a block, with j ascending: any two reflectors whose rows overlap
// keep their relative order.  Groups on one anti-diagonal of the (block, j)
// grid touch disjoint rows, so each anti-diagonal is one launch over
// (group, column tile) pairs.
#include <algorithm>
#include <type_traits>

#include "hgv_internal.h"

namespace hgv {

template <class E>
struct HbArgs {
    int n, b, ldb;
    E *AB;                // band storage, ldb = 2b
    E *V2;                // group-major reflectors
    E *tau2;
    int *prog;            // tasks completed per sweep
    int *err;             // set when a wait gives up
    int J;                // tasks of sweep 0 (max over sweeps)
};

__host__ __device__ inline int hb_tasks(int n, int b, int s) { return (n - 2 - s) / b + 1; }

// The problems of one grouped launch (batched solves), passed by value, sorted
// by order n descending (every n >= 2).  Item k of the launch is sweep s of the
// r-th problem, items ordered by s, then problem: with
// off(s) = sum_p min(s, n_p - 1) items of sweep index below s, s is the largest
// index with off(s) <= k and r = k - off(s) (the problems with a sweep s are the
// first ones of the sorted list).
constexpr int HB_BATCH_MAX = 32;
template <class E>
struct HbBatch {
    int np, nmax, nitems;
    HbArgs<E> p[HB_BATCH_MAX];
};

template <class E>
__device__ inline int hb_batch_off(const HbBatch<E> &bt, int s) {
    int o = 0;
    for (int i = 0; i < bt.np; ++i) o += min(s, bt.p[i].n - 1);
    return o;
}

template <class E>
__device__ inline int2 hb_batch_item(const HbBatch<E> &bt, int k) {
    int lo = 0, hi = bt.nmax - 2;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (hb_batch_off(bt, mid) <= k) lo = mid;
        else hi = mid - 1;
    }
    return make_int2(k - hb_batch_off(bt, lo), lo);
}

__device__ inline double wave_sum(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// Lane groups of TPR consecutive lanes own one row (or column) of a task's
// blocks; sums over a row reduce inside the group with shuffles.
template <int TPR>
__device__ inline double2 group_sum(double2 x) {
#pragma unroll
    for (int o = 1; o < TPR; o <<= 1) {
        x.x += __shfl_xor(x.x, o, 64);
        x.y += __shfl_xor(x.y, o, 64);
    }
    return x;
}

// One workgroup runs whole sweeps; per task (see the file comment):
//   D (the diagonal block, rows/columns I_j) lives in registers: thread
//   (row, q) owns D[row][q + TPR*u];
//   E (rows I_j, columns I_{j-1}) lives in LDS because it is used by rows (the
//   right application of the previous reflector) and then by columns (the
//   left application of the new one).
//
// BATCHED: the workgroups run the sweeps of many problems (the batched solve):
// item k is sweep s of problem r (hb_batch_item); the items are ordered by
// sweep index, then problem, and every workgroup takes its items in
// increasing order.  A sweep waits only for the previous sweep of
// its own problem, which has a smaller item index, so the smallest unfinished
// item always has its predecessor done and its workgroup working on it: with
// every workgroup resident (a cooperative launch) the grid always progresses.
template <int BM, int NT, class E, bool BATCHED>
__global__ __launch_bounds__(NT) void hb2st_kernel(HbArgs<E> a0, HbBatch<E> bt) {
    constexpr int NWV = NT / 64;    // waves
    constexpr int TPR = NT / BM;    // lanes per row
    constexpr int NU = BM / TPR;    // row elements per lane
    __shared__ double2 Es[BM][BM + 1];
    // staging of E for the LDS-direct loads: column c at Et[c][0 .. BM-1], each
    // column a contiguous 64 x 16-byte run (unused for narrower bands)
    __shared__ E Et[BM == 64 && sizeof(E) == 16 ? BM : 1][BM];
    __shared__ double2 v[BM], vp[BM], pv[BM];
    __shared__ double2 sh_tau, sh_taup;
    __shared__ double sh_beta;
    const int tid = threadIdx.x, lane = tid & 63;
    const int row = tid / TPR, q = tid % TPR;
    const double2 zero = make_double2(0.0, 0.0);
    double2 Dr[NU];
    const int total = BATCHED ? bt.nitems : a0.n - 1;

    for (int k = blockIdx.x; k < total; k += gridDim.x) {
        int2 it = make_int2(0, k);
        if constexpr (BATCHED) it = hb_batch_item(bt, k);
        const HbArgs<E> a = BATCHED ? bt.p[it.x] : a0;
        const int s = it.y;
        const int n = a.n, b = a.b, ldb = a.ldb;
        E *AB = a.AB;
        auto bld = [&](size_t idx) -> double2 { return El<E>::to(AB[idx]); };
        auto bst = [&](size_t idx, double2 v) { AB[idx] = El<E>::from(v); };
        const int nt = hb_tasks(n, b, s);
        for (int j = 0; j < nt; ++j) {
            // ---- wait for sweep s-1 ------------------------------------------------
            if (s > 0 && tid == 0) {
                // poll with relaxed loads (an acquire per poll would invalidate the
                // caches for every other workgroup), then one acquire fence.  The
                // wait is bounded: one that gives up sets *err, and every wait
                // that sees *err set returns at once, so the launch always ends
                // (the host side then reports d_info = 2n+2: the band is not valid)
                const int need = min(j + 2, hb_tasks(n, b, s - 1));
                long spins = 0;
                while (__hip_atomic_load(&a.prog[s - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
                    if (__hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
                    __builtin_amdgcn_s_sleep(1);
                    if (++spins > (1L << 27)) {
                        __hip_atomic_store(a.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        break;
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            __syncthreads();
            const int r0 = s + 1 + j * b;
            const int L = min(b, n - r0);          // rows of this task
            const int p0 = r0 - b;                 // first column of E (j > 0)
            // D row of this thread, read raw from the lower band (elements above
            // the diagonal from their mirror); bit u of the result marks Dr[u] as
            // mirrored (to be conjugated once the loads have arrived, so that no
            // load waits for the previous one)
            auto load_d = [&]() {
                unsigned up = 0;
#pragma unroll
                for (int u = 0; u < NU; ++u) {
                    const int k = q + TPR * u;
                    const bool in = row < L && k < L;
                    const int rr = r0 + (in ? row : 0), kk = r0 + (in ? k : 0);
                    const bool low = rr >= kk;
                    up |= (low ? 0u : 1u) << u;
                    Dr[u] = El<E>::to(AB[(low ? rr - kk : kk - rr) + (size_t)(low ? kk : rr) * ldb]);
                }
                return up;
            };
            unsigned upper = 0;
            // ---- D row into registers, E (or column s) into LDS --------------------
            // Every load is issued unconditionally (out-of-block elements read the
            // in-range diagonal element (r0, r0) and are zeroed afterwards), so a
            // thread's 2 * NU loads are in flight together instead of one after
            // another.
            if (j == 0) {
                if (tid < BM) Es[tid][0] = zsel(tid < L, bld(tid < L ? (r0 + tid - s) + (size_t)s * ldb : (size_t)s * ldb), zero);
            } else if constexpr (BM == 64 && sizeof(E) == 16) {
                // LDS-direct loads (no registers, all in flight at once): wave w
                // stages columns w, w + 4, ... of E, lane i taking row i (column c
                // of E is contiguous in the band storage); elements outside the
                // block read the in-range element (r0, r0) and are zeroed in the
                // copy into Es
#pragma unroll
                for (int cc = 0; cc < BM / NWV; ++cc) {
                    const int c = (tid >> 6) + NWV * cc, i = lane;
                    const bool in = i < L && c < b;
                    const size_t idx = in ? (r0 + i - p0 - c) + (size_t)(p0 + c) * ldb : (size_t)r0 * ldb;
                    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)(AB + idx),
                                                     (__attribute__((address_space(3))) void *)(&Et[c][0]), 16, 0,
                                                     0);
                }
                // the D block's loads go out while E's are in flight
                upper = load_d();
                __builtin_amdgcn_s_waitcnt(0);
                __syncthreads();
#pragma unroll
                for (int u = 0; u < BM * BM / NT; ++u) {
                    const int t = tid + NT * u, i = t % BM, c = t / BM;
                    Es[i][c] = zsel(i < L && c < b, El<E>::to(Et[c][i]), zero);
                }
            } else {
                // E through registers: all of a thread's E and D loads are issued
                // before the first one is waited for
                E ev[BM * BM / NT];
#pragma unroll
                for (int u = 0; u < BM * BM / NT; ++u) {
                    const int t = tid + NT * u, i = t % BM, c = t / BM;
                    const bool in = i < L && c < b;
                    ev[u] = AB[in ? (r0 + i - p0 - c) + (size_t)(p0 + c) * ldb : (size_t)r0 * ldb];
                }
                upper = load_d();
#pragma unroll
                for (int u = 0; u < BM * BM / NT; ++u) {
                    const int t = tid + NT * u, i = t % BM, c = t / BM;
                    Es[i][c] = zsel(i < L && c < b, El<E>::to(ev[u]), zero);
                }
            }
            if (j == 0) upper = load_d();
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const int k = q + TPR * u;
                const double2 d = Dr[u];
                Dr[u] = zsel(row < L && k < L, make_double2(d.x, ((upper >> u) & 1u) ? -d.y : d.y), zero);
            }
            __syncthreads();
            if (j > 0) {
                // E <- E - tau_p (E v_p) v_p^H   (previous reflector from the right)
                double2 acc = zero;
#pragma unroll
                for (int u = 0; u < NU; ++u) {
                    int c = q + TPR * u;
                    acc = zadd(acc, zmul(Es[row][c], vp[c]));
                }
                double2 y = zmul(sh_taup, group_sum<TPR>(acc));
                if (row < L) {
#pragma unroll
                    for (int u = 0; u < NU; ++u) {
                        int c = q + TPR * u;
                        Es[row][c] = zsub(Es[row][c], zmul(y, zconj(vp[c])));
                    }
                }
                __syncthreads();
            }
            // ---- reflector from Es[:, 0] (wave 0) -------------------------------------
            if (tid < 64) {
                double2 x = zsel(lane < L, Es[lane < BM ? lane : 0][0], zero);
                double t2 = wave_sum((lane >= 1) ? zabs2(x) : 0.0);
                double2 alpha = make_double2(__shfl(x.x, 0, 64), __shfl(x.y, 0, 64));
                double beta;
                double2 tau, scale;
                if (t2 == 0.0 && alpha.y == 0.0) {
                    beta = alpha.x;
                    tau = zero;
                    scale = zero;
                } else {
                    double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + t2);
                    beta = -copysign(nrm, alpha.x);
                    tau = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
                    scale = zdiv(make_double2(1.0, 0.0), make_double2(alpha.x - beta, alpha.y));
                }
                if (lane < BM) v[lane] = zsel(lane < L, zsel(lane == 0, make_double2(1.0, 0.0), zmul(scale, x)), zero);
                if (lane == 0) {
                    sh_beta = beta;
                    sh_tau = tau;
                }
            }
            __syncthreads();
            const double2 tau = sh_tau;
            const double beta = sh_beta;
            if (j == 0) {
                if (tid < L) bst((r0 + tid - s) + (size_t)s * ldb, zsel(tid == 0, make_double2(beta, 0.0), zero));
            } else {
                // E[:, 1:] <- E - conj(tau) v (v^H E);  E[:, 0] = beta e_1   (column owners)
                const int c = row;   // lane group -> column
                double2 acc = zero;
#pragma unroll
                for (int u = 0; u < NU; ++u) {
                    int i = q + TPR * u;
                    acc = zadd(acc, zcmul(v[i], Es[i][c]));
                }
                double2 wc = zcmul(tau, group_sum<TPR>(acc));
                if (c < b) {
#pragma unroll
                    for (int u = 0; u < NU; ++u) {
                        int i = q + TPR * u;
                        if (i < L) {
                            double2 val = zsel(c == 0, zsel(i == 0, make_double2(beta, 0.0), zero),
                                               zsub(Es[i][c], zmul(v[i], wc)));
                            bst((r0 + i - p0 - c) + (size_t)(p0 + c) * ldb, val);
                        }
                    }
                }
            }
            // ---- two-sided update of D:  D <- H^H D H -----------------------------------
            {
                double2 acc = zero;
#pragma unroll
                for (int u = 0; u < NU; ++u) acc = zadd(acc, zmul(Dr[u], v[q + TPR * u]));
                double2 prow = zmul(tau, group_sum<TPR>(acc));
                if (q == 0) pv[row] = zsel(row < L, prow, zero);
                __syncthreads();
                // w = p - 1/2 conj(tau) (v^H p) v   (the scalar is real; same order in every wave)
                double2 c1 = zsel(lane < BM, zcmul(v[lane < BM ? lane : 0], pv[lane < BM ? lane : 0]), zero);
                double vr = wave_sum(c1.x), vi = wave_sum(c1.y);
                double half = 0.5 * zcmul(tau, make_double2(vr, vi)).x;
                double2 wrow = zsub(prow, zscale(half, v[row]));
                double2 vrow = v[row];
                if (row < L) {
#pragma unroll
                    for (int u = 0; u < NU; ++u) {
                        int k = q + TPR * u;
                        if (k <= row) {
                            double2 wk = zsub(pv[k], zscale(half, v[k]));
                            double2 val = zsub(zsub(Dr[u], zmul(vrow, zconj(wk))), zmul(wrow, zconj(v[k])));
                            if (k == row) val.y = 0.0;
                            bst((row - k) + (size_t)(r0 + k) * ldb, val);
                        }
                    }
                }
            }
            // ---- store the reflector (group-major layout; not kept when only
            // eigenvalues are wanted) and keep it for task j+1 -----
            if (a.V2) {
                const int B = s / b, t = s % b;
                size_t base = ((size_t)B * a.J + j) * b + t;
                if (tid < b) a.V2[base * b + tid] = El<E>::from(v[tid]);
                if (tid == 0) a.tau2[base] = El<E>::from(tau);
            }
            __syncthreads();
            if (tid < BM) vp[tid] = v[tid];
            if (tid == 0) sh_taup = tau;
            // every thread's stores have reached the L2 before the barrier; thread
            // 0's release store then writes the L2 back once for the workgroup
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            if (tid == 0) __hip_atomic_store(&a.prog[s], j + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// ---- window-owner pipeline ---------------------------------------------------------------
// The same tasks and reflectors, scheduled by window instead of by sweep.
// Workgroup w owns, for every sweep s, the rows I_w(s) = [s+1+w*b, s+(w+1)*b]:
// the diagonal block D_w = A[I_w, I_w] (registers, thread (row, q) holding
// D[row][q + TPR*u]) and the block below it E_w = A[I_{w+1}, I_w] (LDS), both
// kept resident from sweep to sweep.  Index i sits at slot i mod b, so moving
// the window one index down (sweep s -> s+1) replaces one slot t: index
// c = s+(w+1)*b enters, c - b leaves; row c of E_w becomes the new last row of
// D_w, and the rest of column c (its diagonal element and the b elements below
// it) comes from workgroup w+1, which drops index c at the same sweep.
// Per task (s, w):
//   wait for H_{s,w} (posted by w-1) and for column c (posted by w+1 after its
//   task of sweep s-1); shift the window; E <- E H_{s,w}; H_{s,w+1} from E's
//   first column, posted to w+1; D <- H^H D H; the band column of the
//   window's first index (D's column, beta of H_{s,w+1} below it) posted to w-1;
//   E <- H_{s,w+1}^H E.
// Workgroup 0 makes H_{s,0} from column s, which it keeps from its window of
// sweep s-1, and writes d_s and e_s.  A message is one reflector or one band
// column (b + 1 values), so no block travels through memory between tasks.
// Task (s, w) waits for (s, w-1), (s-1, w+1) and follows (s-1, w) on its own
// workgroup: all three have a smaller 2s + w, so with every workgroup resident
// (cooperative launch) the smallest unfinished task can always run.  A mailbox
// is written again only after its reader has posted a message that depends on
// having read it (one buffer per mailbox would do; two are kept, by sweep
// parity).  Every task's arithmetic is fixed, so the result does not depend on
// timing.
template <class E>
struct HbOwnArgs {
    int n, b, ldb, J;
    const E *AB;
    E *V2, *tau2;
    double *d, *e;                 // the tridiagonal (written by workgroup 0)
    unsigned long long *boxH;      // per workgroup: 2 (sweep parity) x (BM + 1) values x 4 words
    unsigned long long *boxS;
    int *err;                      // set when a wait gives up
};

// Messages.  A complex value travels as four 64-bit words, each holding the
// tag of its message (the sweep it is for, plus one) in the upper half and 32
// bits of the value in the lower half, written and read as relaxed device-scope
// atomics.  Every word is one atomic location, so a reader that sees the
// expected tag in all four words has read the value that was sent with it: the
// receiver polls the data itself (no separate flag, no fences), and the sender
// does not wait for its stores.  A mailbox is zeroed before the launch (tag 0
// is never expected).
__device__ inline void msg_put(unsigned long long *p, double2 v, unsigned tag) {
    const unsigned long long t = (unsigned long long)tag << 32;
    const unsigned long long x = (unsigned long long)__double_as_longlong(v.x);
    const unsigned long long y = (unsigned long long)__double_as_longlong(v.y);
    __hip_atomic_store(p + 0, t | (x & 0xffffffffull), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(p + 1, t | (x >> 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(p + 2, t | (y & 0xffffffffull), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(p + 3, t | (y >> 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One poll of a lane: the four words of up to four message entries (e0, e1 for
// every lane; e2, e3 only used by lane 0).
struct MsgPoll {
    unsigned long long x[16];
};
__device__ inline void msg_issue(MsgPoll &P, const unsigned long long *e0, const unsigned long long *e1,
                                 const unsigned long long *e2, const unsigned long long *e3) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        P.x[k] = __hip_atomic_load(e0 + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        P.x[4 + k] = __hip_atomic_load(e1 + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        P.x[8 + k] = __hip_atomic_load(e2 + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        P.x[12 + k] = __hip_atomic_load(e3 + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}
// entry k of the poll carries the tag (or is not wanted)
__device__ inline bool msg_ok(const MsgPoll &P, unsigned tag, unsigned want) {
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 16; ++k) ok &= !((want >> (k >> 2)) & 1u) || (P.x[k] >> 32) == tag;
    return ok;
}
__device__ inline double2 msg_val(const MsgPoll &P, int k) {
    const unsigned long long *x = P.x + 4 * k;
    return make_double2(__longlong_as_double((long long)(((x[1] & 0xffffffffull) << 32) | (x[0] & 0xffffffffull))),
                        __longlong_as_double((long long)(((x[3] & 0xffffffffull) << 32) | (x[2] & 0xffffffffull))));
}

// Reductions of the pipeline kernel by DPP lane moves (no LDS round trips).  A
// double moves as its two 32-bit halves.  Each step adds a lane's value to its
// partner's under a pairing (xor 1, xor 2, mirror within 8, mirror within 16),
// so both partners form the same sum and every lane of the group ends with the
// same bits.
// sum over aligned groups of 8 lanes
__device__ inline double sum8_dpp(double x) {
    x += dpp_f64<0xB1>(x);    // quad_perm [1,0,3,2]: xor 1
    x += dpp_f64<0x4E>(x);    // quad_perm [2,3,0,1]: xor 2
    x += dpp_f64<0x141>(x);   // row_half_mirror: lane i <-> 7 - i
    return x;
}
__device__ inline double2 sum8_dpp(double2 x) { return make_double2(sum8_dpp(x.x), sum8_dpp(x.y)); }
// sum over the wave (the same value in every lane)
__device__ inline double wave_sum_dpp(double x) {
    x = sum8_dpp(x);
    x += dpp_f64<0x140>(x);   // row_mirror: lane i <-> 15 - i
    return (lane_f64(x, 0) + lane_f64(x, 16)) + (lane_f64(x, 32) + lane_f64(x, 48));
}

// Householder reflector of the slot-ordered vector x held by the lanes of one
// wave (lane = slot, alpha at slot f, lanes with valid == false hold no
// element): H^H x = beta e_f with beta real; returns v (v_f = 1) of this lane.
__device__ inline double2 hb_refl_slots(double2 x, bool valid, int f, double2 &tau, double &beta) {
    const int lane = threadIdx.x & 63;
    x = zsel(valid, x, make_double2(0.0, 0.0));
    const double t2 = wave_sum_dpp(lane != f ? zabs2(x) : 0.0);
    const double2 alpha = make_double2(lane_f64(x.x, f), lane_f64(x.y, f));
    double2 scale;
    if (t2 == 0.0 && alpha.y == 0.0) {
        beta = alpha.x;
        tau = make_double2(0.0, 0.0);
        scale = make_double2(0.0, 0.0);
    } else {
        const double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + t2);
        beta = -copysign(nrm, alpha.x);
        tau = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
        scale = zdiv(make_double2(1.0, 0.0), make_double2(alpha.x - beta, alpha.y));
    }
    return zsel(valid, zsel(lane == f, make_double2(1.0, 0.0), zmul(scale, x)), make_double2(0.0, 0.0));
}

template <int BM, int NT, class E>
__global__ __launch_bounds__(NT) void hb2st_owner_kernel(HbOwnArgs<E> a) {
    constexpr int TPR = NT / BM;    // lanes per row
    constexpr int NU = BM / TPR;    // row elements per lane
    constexpr int NWV = NT / 64;    // waves
    static_assert(BM <= 64 && NT % 64 == 0 && NWV >= 2 && TPR == 8, "one wave holds a reflector; two waves post; 8 lanes per row");
    __shared__ double2 Es[BM][BM + 1];
    __shared__ double2 vs[BM], v2s[BM], pv[BM], yv[BM], xs[BM], ms[BM + 1];
    __shared__ double2 sh_tau;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int row = tid / TPR, q = tid % TPR;
    const int w = blockIdx.x;
    const int n = a.n, b = a.b, ldb = a.ldb, J = a.J;
    const E *AB = a.AB;
    const double2 zero = make_double2(0.0, 0.0);
    double2 Dr[NU];
    const int nsw = n - 1 - w * b;   // sweeps with a nonempty window w
    for (int s = 0; s < nsw; ++s) {
        const int r0 = s + 1 + w * b;
        const int L = min(b, n - r0), Le = min(b, n - r0 - b);
        const int f = r0 % b;   // slot of the window's first index
        // window position of slot k (b for slots beyond the band width)
        auto widx = [&](int k) { return k >= b ? b : (k >= f ? k - f : k - f + b); };
        const int ir = widx(row);
        if (s == 0) {
            // ---- first window, read from the band ---------------------------------------
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const int ik = widx(q + TPR * u);
                const bool in = ir < L && ik < L;
                const int i = in ? ir : 0, k = in ? ik : 0;
                const bool low = i >= k;
                const double2 d = El<E>::to(AB[(low ? i - k : k - i) + (size_t)(r0 + (low ? k : i)) * ldb]);
                Dr[u] = zsel(in, make_double2(d.x, low ? d.y : -d.y), zero);
            }
            for (int t = tid; t < BM * BM; t += NT) {
                const int rho = t % BM, kap = t / BM;
                const int i = widx(rho), k = widx(kap);
                const bool in = i < Le && k < L;
                const double2 ev = El<E>::to(AB[in ? (b + i - k) + (size_t)(r0 + k) * ldb : (size_t)r0 * ldb]);
                Es[rho][kap] = zsel(in, ev, zero);
            }
            if (w == 0 && tid < BM) {
                const int i = widx(tid);
                xs[tid] = zsel(i < L, El<E>::to(AB[1 + (i < L ? i : 0)]), zero);
                if (tid == 0) a.d[0] = El<E>::to(AB[0]).x;
            }
        } else if (w == 0) {
            // ---- column s (index r0 - 1, slot t0) from the previous window -------------
            const int t0 = f > 0 ? f - 1 : b - 1;
            if (q == t0 % TPR) {
                double2 dv = zero;
#pragma unroll
                for (int u = 0; u < NU; ++u) dv = zsel(u == t0 / TPR, Dr[u], dv);
                if (row == t0) {
                    xs[row] = Es[t0][t0];
                    a.d[r0 - 1] = dv.x;   // d_s
                } else if (row < b) {
                    xs[row] = zsel(ir < L, dv, zero);
                }
            }
        }
        // ---- move the window (slot t: index c - b leaves, c enters), first the part
        // that uses only local data: row c of E becomes the new row (and column) c of D
        const int t = f > 0 ? f - 1 : b - 1;
        if (s > 0) {
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const int k = q + TPR * u;
                if (row == t) {
                    if (k != t) Dr[u] = Es[t][k];
                } else if (k == t) {
                    Dr[u] = zconj(Es[t][row]);
                }
            }
        }
        // ---- wave 0: receive the reflector (from w-1) and the entering column (from
        // w+1) into LDS ----------------------------------------------------------------------
        const int c = r0 - 1 + b;
        const bool shift_in = s > 0 && c <= n - 1;
        if (wave == 0) {
            const unsigned tag = (unsigned)s + 1;
            const unsigned long long *bh = a.boxH + ((size_t)w * 2 + (s & 1)) * (BM + 1) * 4;
            const unsigned long long *bs = a.boxS + ((size_t)w * 2 + (s & 1)) * (BM + 1) * 4;
            // lane i takes entry i of each message; lane 0 also the last entry (tau of the
            // reflector at BM, the element below the column at b)
            double2 h0 = zero, h1 = zero, s0 = zero, s1 = zero;
            if (w > 0 || shift_in) {
                const unsigned want = (w > 0 && lane < BM ? 1u : 0u) | (shift_in && lane <= b ? 2u : 0u) |
                                      (w > 0 && lane == 0 ? 4u : 0u) | (shift_in && lane == 0 && b == 64 ? 8u : 0u);
                const unsigned long long *e0 = bh + 4 * (lane < BM ? lane : 0);
                const unsigned long long *e1 = bs + 4 * (lane <= b ? lane : 0);
                const unsigned long long *e2 = bh + 4 * BM;
                const unsigned long long *e3 = bs + 4 * (b == 64 ? 64 : 0);
                // two polls in flight: each is checked while the next one is out, which
                // halves the time between a message landing and a poll reading it.
                // Bounded: a wait that gives up sets *err, and every wait that sees *err
                // set returns at once, so the launch always ends (the host side then
                // reports d_info = 2n+2: the band is not valid)
                MsgPoll PA, PB;
                msg_issue(PA, e0, e1, e2, e3);
                for (long spins = 0;; spins += 2) {
                    msg_issue(PB, e0, e1, e2, e3);
                    if (__all(msg_ok(PA, tag, want))) {
                        h0 = msg_val(PA, 0);
                        s0 = msg_val(PA, 1);
                        h1 = msg_val(PA, 2);
                        s1 = msg_val(PA, 3);
                        break;
                    }
                    msg_issue(PA, e0, e1, e2, e3);
                    if (__all(msg_ok(PB, tag, want))) {
                        h0 = msg_val(PB, 0);
                        s0 = msg_val(PB, 1);
                        h1 = msg_val(PB, 2);
                        s1 = msg_val(PB, 3);
                        break;
                    }
                    if (__hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
                    if (spins > (1L << 28)) {
                        __hip_atomic_store(a.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        break;
                    }
                }
            }
            if (w > 0 && lane < BM) {
                // window order -> slots
                if (lane < b) vs[(f + lane) % b] = zsel(lane < L, h0, zero);
                else vs[lane] = zero;
                if (lane == 0) sh_tau = h1;
            }
            if (s > 0) {
                if (lane <= BM) ms[lane] = zsel(shift_in && lane <= b, s0, zero);
                if (lane == 0 && BM == 64) ms[64] = zsel(shift_in && b == 64, s1, zero);
            }
        }
        __syncthreads();
        if (s > 0) {
            // ---- the rest of the move, each thread on its own elements: E's row t now
            // holds row c + b (in the band only at column c), its column t column c below
            // the diagonal, D[t][t] the diagonal element of index c
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const int k = q + TPR * u;
                if (row == t) {
                    Es[t][k] = zsel(k == t, ms[b], zero);
                    if (k == t) Dr[u] = make_double2(ms[0].x, 0.0);
                } else if (k == t) {
                    Es[row][t] = zsel(row < b, ms[row < b ? (row > t ? row - t : row - t + b) : 0], zero);
                }
            }
        }
        // ---- H_{s,0}: workgroup 0 makes it from column s ---------------------------------
        if (w == 0) {
            if (tid < 64) {
                double2 tau;
                double beta;
                const bool valid = lane < BM && widx(lane) < L;
                const double2 v = hb_refl_slots(xs[lane < BM ? lane : 0], valid, f, tau, beta);
                if (lane < BM) vs[lane] = v;
                if (lane == 0) {
                    sh_tau = tau;
                    a.e[r0 - 1] = beta;   // e_s
                }
                if (a.V2) {
                    // slot lane -> window position widx(lane)
                    const size_t base = ((size_t)(s / b) * J + 0) * b + s % b;
                    if (lane < b) a.V2[base * b + widx(lane)] = El<E>::from(v);
                    if (lane == 0) a.tau2[base] = El<E>::from(tau);
                }
            }
            __syncthreads();
        }
        const double2 tau = sh_tau;
        // ---- y = tau E v and p = tau D v, one pass over the thread's row (E is
        // updated once, after both messages are out) -----------------------------------------
        double2 vr[NU];   // v at the thread's column slots
#pragma unroll
        for (int u = 0; u < NU; ++u) vr[u] = vs[q + TPR * u];
        {
            double2 ay = zero, ap = zero;
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                zfma(ay, Es[row][q + TPR * u], vr[u]);
                zfma(ap, Dr[u], vr[u]);
            }
            const double2 y = zmul(tau, sum8_dpp(ay));
            const double2 prow = zmul(tau, sum8_dpp(ap));
            if (q == 0) {
                yv[row] = y;
                pv[row] = prow;
            }
        }
        __syncthreads();
        // ---- every wave: H_{s,w+1} from the first column of E H_{s,w} = E - y v^H, and
        // the scalars of the updates (the same operations in the same order in every wave,
        // so every wave holds the same values and none waits for another) ----------------
        const double2 vf = vs[f];
        const int l = lane < BM ? lane : 0;
        double2 v2 = zero, tau2 = zero;
        double beta2 = 0.0;
        if (Le > 0) {
            const bool valid = lane < BM && widx(lane) < Le;
            v2 = hb_refl_slots(zsub(Es[l][f], zmul(yv[l], zconj(vf))), valid, f, tau2, beta2);
            if (wave == 0) {
                // H_{s,w+1} to w+1, in the window order of window w+1: slot lane goes to
                // position widx(lane) (positions b .. BM-1 are zero)
                if (lane < BM) v2s[lane] = v2;
                unsigned long long *bx = a.boxH + ((size_t)(w + 1) * 2 + (s & 1)) * (BM + 1) * 4;
                if (lane < BM) msg_put(bx + 4 * (lane < b ? widx(lane) : lane), v2, (unsigned)s + 1);
                if (lane == 0) msg_put(bx + 4 * BM, tau2, (unsigned)s + 1);
                if (a.V2) {
                    const size_t base = ((size_t)(s / b) * J + (w + 1)) * b + s % b;
                    if (lane < b) a.V2[base * b + widx(lane)] = El<E>::from(v2);
                    if (lane == 0) a.tau2[base] = El<E>::from(tau2);
                }
            }
        }
        const double2 c1 = zsel(lane < BM, zcmul(vs[l], pv[l]), zero);
        const double half = 0.5 * zcmul(tau, make_double2(wave_sum_dpp(c1.x), wave_sum_dpp(c1.y))).x;
        // ---- D <- H^H D H  with  w = p - 1/2 conj(tau) (v^H p) v ----------------------------
        {
            const double2 vrow = vs[row];
            const double2 wrow = zsub(pv[row], zscale(half, vrow));
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const int k = q + TPR * u;
                const double2 wk = zsub(pv[k], zscale(half, vr[u]));
                double2 val = Dr[u];
                zfma(val, make_double2(-vrow.x, -vrow.y), zconj(wk));
                zfma(val, make_double2(-wrow.x, -wrow.y), zconj(vr[u]));
                if (k == row) val.y = 0.0;
                Dr[u] = val;
            }
        }
        // ---- the band column of index r0 (it leaves this window next sweep) -> w-1, for
        // its sweep s+1: positions 0 .. b-1 the column, position b the element below it;
        // each thread of column f sends its own element ----------------------------------
        if (w > 0) {
            unsigned long long *bx = a.boxS + ((size_t)(w - 1) * 2 + ((s + 1) & 1)) * (BM + 1) * 4;
            if (q == f % TPR && row < b) {
                double2 dv = zero;
#pragma unroll
                for (int u = 0; u < NU; ++u) dv = zsel(u == f / TPR, Dr[u], dv);
                msg_put(bx + 4 * ir, zsel(ir < L, dv, zero), (unsigned)s + 2);
            }
            if (tid == 0) msg_put(bx + 4 * b, zsel(Le > 0, make_double2(beta2, 0.0), zero), (unsigned)s + 2);
        }
        if (Le > 0) {
            // ---- E <- H_{s,w+1}^H (E - y v^H), first column beta e_f:  with
            // u = v2^H E and vy = v2^H y,  E[i][c] -= y_i conj(v_c) + conj(tau2) v2_i
            // (u_c - vy conj(v_c)) ----------------------------------------------------------
            const double2 c2 = zsel(lane < BM, zcmul(v2, yv[l]), zero);
            const double2 vy = make_double2(wave_sum_dpp(c2.x), wave_sum_dpp(c2.y));
            __syncthreads();   // v2s
            const int cc = row;   // lane group -> column
            const double2 vc = zconj(vs[cc]);
            double2 acc = zero;
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const int i = q + TPR * u;
                zcfma(acc, v2s[i], Es[i][cc]);
            }
            const double2 wc = zcmul(tau2, zsub(sum8_dpp(acc), zmul(vy, vc)));
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const int i = q + TPR * u;
                double2 upd = Es[i][cc];
                zfma(upd, make_double2(-yv[i].x, -yv[i].y), vc);
                zfma(upd, make_double2(-v2s[i].x, -v2s[i].y), wc);
                Es[i][cc] = zsel(cc == f, zsel(i == f, make_double2(beta2, 0.0), zero), upd);
            }
        }
        __syncthreads();
    }
    if (w == 0 && n >= 2) {
        // d_{n-1}: the last diagonal element, in the one-element window of the last sweep
        const int t = (n - 1) % b;
        if (row == t && q == t % TPR) {
            double2 dv = zero;
#pragma unroll
            for (int u = 0; u < NU; ++u) dv = zsel(u == t / TPR, Dr[u], dv);
            a.d[n - 1] = dv.x;
        }
    }
}

// Copy the lower band (offsets 0..b) of A into band storage; offsets b+1..2b-1 zero.
template <class E>
__global__ void band_copy_kernel(int n, int b, const E *A, int lda, E *AB, int ldb) {
    int off = threadIdx.x % ldb;
    int c = blockIdx.x * (256 / ldb) + threadIdx.x / ldb;
    if (threadIdx.x >= (256 / ldb) * ldb || c >= n) return;
    int r = c + off;
    E v = El<E>::mk(0.0, 0.0);
    if (off <= b && r < n) v = A[r + (size_t)c * lda];
    if (off == 0) v.y = 0;
    AB[off + (size_t)c * ldb] = v;
}

template <class E>
__global__ void tridiag_out_kernel(int n, const E *AB, int ldb, double *d, double *e) {
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) d[i] = AB[(size_t)i * ldb].x;
    if (i < n - 1) e[i] = AB[1 + (size_t)i * ldb].x;
}

template <class E>
__global__ void zero2_kernel(E *p, size_t cnt) {
    size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    for (; i < cnt; i += (size_t)gridDim.x * blockDim.x) p[i] = El<E>::mk(0.0, 0.0);
}
__global__ void zero_int_kernel(int *p, int cnt) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < cnt; i += gridDim.x * blockDim.x) p[i] = 0;
}

static int hb_J(int n, int b) { return n >= 2 ? hb_tasks(n, b, 0) : 0; }
static int hb_nblk(int n, int b) { return n >= 2 ? cdiv(n - 1, b) : 0; }

size_t v2_elems(int n, int nb) { return std::max<size_t>((size_t)hb_nblk(n, nb) * hb_J(n, nb) * nb * nb, 1); }
size_t v2_taus(int n, int nb) { return std::max<size_t>((size_t)hb_nblk(n, nb) * hb_J(n, nb) * nb, 1); }

template <class E>
static void zero2(hgv_ctx_s *ctx, E *p, size_t cnt) {
    if (!cnt) return;
    hipLaunchKernelGGL(zero2_kernel<E>, dim3((unsigned)std::min<size_t>(cdivz(cnt, 256), 16384)), dim3(256), 0,
                       ctx->stream, p, cnt);
    HGV_LAUNCH_CHECK();
}

template <int BM, int NT, class E>
static void launch_hb2st(hgv_ctx_s *ctx, HbArgs<E> &a) {
    int dev = ctx->device, cus = 0, per = 0;
    HGV_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    HGV_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, hb2st_kernel<BM, NT, E, false>, NT, 0));
    // a sweep starts two tasks behind its predecessor, so about J/2 sweeps are
    // in flight at once; more workgroups would only poll
    int G = std::max(1, std::min({cus * std::max(per, 1), a.n - 1, a.J / 2 + 4}));
    HbBatch<E> none;
    none.np = none.nmax = none.nitems = 0;
    void *args[] = {&a, &none};
    HGV_HIP(hipLaunchCooperativeKernel(reinterpret_cast<void *>(hb2st_kernel<BM, NT, E, false>), dim3(G), dim3(NT),
                                       args, 0, ctx->stream));
}

// The window-owner pipeline needs one resident workgroup per window of sweep 0;
// returns false (use the sweep-per-workgroup kernel) when they do not fit.
template <int BM, int NT, class E>
static bool launch_hb2st_owner(hgv_ctx_s *ctx, HbOwnArgs<E> &a) {
    int dev = ctx->device, cus = 0, per = 0;
    HGV_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    HGV_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, hb2st_owner_kernel<BM, NT, E>, NT, 0));
    if (a.J < 1 || a.J > cus * per) return false;
    void *args[] = {&a};
    HGV_HIP(hipLaunchCooperativeKernel(reinterpret_cast<void *>(hb2st_owner_kernel<BM, NT, E>), dim3(a.J), dim3(NT),
                                       args, 0, ctx->stream));
    return true;
}

template <class E>
void hb2st_t(hgv_ctx_s *ctx, int n, int nb, const E *A, int lda, double *d, double *e, E *V2, E *tau2, Arena &ar,
             int *d_info) {
    if (nb > 64) throw HipFail{hipErrorInvalidValue};
    const int b = nb, ldb = 2 * nb;
    const int BM = b <= 32 ? 32 : 64, J = hb_J(n, b);
    E *AB = ar.take<E>((size_t)ldb * std::max(n, 1));
    int *prog = ar.take<int>(std::max(n, 1) + 1);
    int *err = prog + std::max(n, 1);
    // mailboxes of the window-owner pipeline (both zeroed together before a launch)
    const size_t box_words = (size_t)std::max(J, 1) * 2 * (BM + 1) * 4;
    unsigned long long *boxH = ar.take<unsigned long long>(2 * box_words);
    unsigned long long *boxS = boxH + box_words;
    if (ar.measuring() || n == 0) return;
    hipLaunchKernelGGL(band_copy_kernel<E>, dim3(cdiv(n, 256 / ldb)), dim3(256), 0, ctx->stream, n, b, A, lda, AB,
                       ldb);
    HGV_LAUNCH_CHECK();
    if (V2) {   // null: eigenvalues only, the reflectors are not stored
        zero2(ctx, V2, v2_elems(n, nb));
        zero2(ctx, tau2, v2_taus(n, nb));
    }
    hipLaunchKernelGGL(zero_int_kernel, dim3(cdiv(n + 1, 256)), dim3(256), 0, ctx->stream, prog, std::max(n, 1) + 1);
    HGV_LAUNCH_CHECK();
    if (ctx->test_hooks & HGV_TEST_WAIT_FAIL) set_info(ctx, err, 1);
    if (n >= 2) {
        bool done = false;
        // (not while problems run concurrently on side streams: the pipeline's
        // workgroups must all be resident at once)
        if (!(ctx->test_hooks & HGV_TEST_HB2ST_SWEEPS) && !ctx->concurrent) {
            const int words = (int)(4 * box_words);   // as ints
            hipLaunchKernelGGL(zero_int_kernel, dim3(std::min(cdiv(words, 256), 4096)), dim3(256), 0, ctx->stream,
                               reinterpret_cast<int *>(boxH), words);
            HGV_LAUNCH_CHECK();
            HbOwnArgs<E> o{n, b, ldb, J, AB, V2, tau2, d, e, boxH, boxS, err};
            done = b <= 32 ? launch_hb2st_owner<32, 256, E>(ctx, o) : launch_hb2st_owner<64, 512, E>(ctx, o);
        }
        if (!done) {
            HbArgs<E> a{n, b, ldb, AB, V2, tau2, prog, err, J};
            // 64-wide bands: 512 threads (8 elements of a task's diagonal block per
            // thread), which shortens the arithmetic of the dependent task chain
            if (b <= 32) launch_hb2st<32, 256, E>(ctx, a);
            else launch_hb2st<64, 512, E>(ctx, a);
        }
        report_wait_fail(ctx, err, d_info, 2 * n + 2);
        if (done) return;   // the pipeline wrote d and e
    }
    hipLaunchKernelGGL(tridiag_out_kernel<E>, dim3(cdiv(n, 256)), dim3(256), 0, ctx->stream, n, AB, ldb, d, e);
    HGV_LAUNCH_CHECK();
}

// ---- grouped bulge chasing of many problems (batched solves) ----------------------------------
template <class E>
void hb2st_batch_plan(int n, int nb, Arena &ar, HbBatchProblem &pb) {
    pb.n = n;
    pb.nb = nb;
    pb.AB = ar.take<E>((size_t)2 * nb * std::max(n, 1));
    pb.prog = ar.take<int>(std::max(n, 1));
}

template <class E>
void hb2st_batch_prep(hgv_ctx_s *ctx, const HbBatchProblem &pb, const E *A, int lda) {
    const int n = pb.n, nb = pb.nb, ldb = 2 * nb;
    if (nb > 64) throw HipFail{hipErrorInvalidValue};
    if (n == 0) return;
    E *AB = static_cast<E *>(pb.AB);
    hipLaunchKernelGGL(band_copy_kernel<E>, dim3(cdiv(n, 256 / ldb)), dim3(256), 0, ctx->stream, n, nb, A, lda, AB,
                       ldb);
    HGV_LAUNCH_CHECK();
    if (pb.V2) {
        zero2(ctx, static_cast<E *>(pb.V2), v2_elems(n, nb));
        zero2(ctx, static_cast<E *>(pb.tau2), v2_taus(n, nb));
    }
    hipLaunchKernelGGL(zero_int_kernel, dim3(cdiv(n, 256)), dim3(256), 0, ctx->stream, pb.prog, n);
    HGV_LAUNCH_CHECK();
}

template <class E>
void hb2st_batch_run(hgv_ctx_s *ctx, const std::vector<HbBatchProblem> &pbs, int *err) {
    if (ctx->test_hooks & HGV_TEST_WAIT_FAIL) set_info(ctx, err, 1);
    else set_info(ctx, err, 0);
    std::vector<int> order;
    for (int i = 0; i < (int)pbs.size(); ++i)
        if (pbs[i].n >= 2) order.push_back(i);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return pbs[x].n > pbs[y].n; });
    int cus = 0, per = 0;
    HGV_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
    HGV_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, hb2st_kernel<64, 512, E, true>, 512, 0));
    // the largest problems first, HB_BATCH_MAX per launch
    for (size_t g0 = 0; g0 < order.size(); g0 += HB_BATCH_MAX) {
        HbBatch<E> bt;
        std::memset(&bt, 0, sizeof(bt));
        bt.np = (int)std::min<size_t>(HB_BATCH_MAX, order.size() - g0);
        long items = 0, inflight = 0;
        for (int i = 0; i < bt.np; ++i) {
            const HbBatchProblem &pb = pbs[order[g0 + i]];
            HbArgs<E> &a = bt.p[i];
            a.n = pb.n;
            a.b = pb.nb;
            a.ldb = 2 * pb.nb;
            a.AB = static_cast<E *>(pb.AB);
            a.V2 = static_cast<E *>(pb.V2);
            a.tau2 = static_cast<E *>(pb.tau2);
            a.prog = pb.prog;
            a.err = err;
            a.J = hb_J(pb.n, pb.nb);
            items += pb.n - 1;
            inflight += a.J / 2 + 4;
        }
        bt.nmax = bt.p[0].n;
        bt.nitems = (int)items;
        // about J/2 sweeps of each problem can be in flight at once
        const int G = (int)std::max<long>(1, std::min<long>({(long)cus * std::max(per, 1), items, inflight}));
        HbArgs<E> none{};
        void *args[] = {&none, &bt};
        HGV_HIP(hipLaunchCooperativeKernel(reinterpret_cast<void *>(hb2st_kernel<64, 512, E, true>), dim3(G), dim3(512),
                                           args, 0, ctx->stream));
    }
    for (const HbBatchProblem &pb : pbs)
        if (pb.n >= 2) report_wait_fail(ctx, err, pb.d_info, 2 * pb.n + 2);
}

template <class E>
void hb2st_batch_finish(hgv_ctx_s *ctx, const HbBatchProblem &pb, double *d, double *e) {
    if (pb.n == 0) return;
    hipLaunchKernelGGL(tridiag_out_kernel<E>, dim3(cdiv(pb.n, 256)), dim3(256), 0, ctx->stream, pb.n,
                       static_cast<const E *>(pb.AB), 2 * pb.nb, d, e);
    HGV_LAUNCH_CHECK();
}

template void hb2st_batch_plan<double2>(int, int, Arena &, HbBatchProblem &);
template void hb2st_batch_prep<double2>(hgv_ctx_s *, const HbBatchProblem &, const double2 *, int);
template void hb2st_batch_run<double2>(hgv_ctx_s *, const std::vector<HbBatchProblem> &, int *);
template void hb2st_batch_finish<double2>(hgv_ctx_s *, const HbBatchProblem &, double *, double *);
template void hb2st_batch_plan<float2>(int, int, Arena &, HbBatchProblem &);
template void hb2st_batch_prep<float2>(hgv_ctx_s *, const HbBatchProblem &, const float2 *, int);
template void hb2st_batch_run<float2>(hgv_ctx_s *, const std::vector<HbBatchProblem> &, int *);
template void hb2st_batch_finish<float2>(hgv_ctx_s *, const HbBatchProblem &, double *, double *);

template void hb2st_t<double2>(hgv_ctx_s *, int, int, const double2 *, int, double *, double *, double2 *, double2 *,
                               Arena &, int *);
template void hb2st_t<float2>(hgv_ctx_s *, int, int, const float2 *, int, double *, double *, float2 *, float2 *,
                              Arena &, int *);

// ---- Q2 back-transformation ------------------------------------------------------------------
// Groups hold g <= b consecutive sweeps at one step j (any g <= b keeps every
// pair of overlapping reflectors in order).  Reflector t of group (B, j) is
// H_{B*g + t, j}; it occupies local rows t .. t+b-1 of the group, whose first
// row is B*g + 1 + j*b.
template <class E>
__device__ inline const E *v2_ptr(const E *V2, int b, int J, int s, int j) {
    return V2 + (((size_t)(s / b) * J + j) * b + (s % b)) * b;
}
__device__ inline size_t tau2_idx(int b, int J, int s, int j) { return ((size_t)(s / b) * J + j) * b + (s % b); }

// T of every group: G[t1][t2] = sum_rows conj(V[row][t1]) V[row][t2] over the
// overlap rows [t2, t1+b-1]; T_tt = tau_t, T[0:t, t] = -tau_t T[0:t, 0:t] G[0:t, t].
// The recurrence runs in double whatever the storage type.
template <int BMAX, int GMAX, class E>
__global__ __launch_bounds__(256) void q2_tbuild_kernel(int n, int b, int g, int J, const E *V2, const E *tau2,
                                                         E *T2) {
    __shared__ double2 Vs[GMAX][BMAX + 1];
    __shared__ double2 Gs[GMAX][GMAX + 1];
    __shared__ double2 Ts[GMAX][GMAX + 1];
    __shared__ double2 taus[GMAX];
    const int grp = blockIdx.x;                 // B * J + j
    const int B = grp / J, j = grp % J;
    const int tid = threadIdx.x;
    for (int t = tid; t < g * b; t += 256) {
        int tt = t / b, i = t % b;
        int s = B * g + tt;
        Vs[tt][i] = (s <= n - 2) ? El<E>::to(v2_ptr(V2, b, J, s, j)[i]) : make_double2(0.0, 0.0);
    }
    if (tid < g) {
        int s = B * g + tid;
        taus[tid] = (s <= n - 2) ? El<E>::to(tau2[tau2_idx(b, J, s, j)]) : make_double2(0.0, 0.0);
    }
    for (int t = tid; t < GMAX * GMAX; t += 256) Ts[t / GMAX][t % GMAX] = make_double2(0.0, 0.0);
    __syncthreads();
    for (int t = tid; t < g * g; t += 256) {
        int t1 = t % g, t2 = t / g;
        if (t1 >= t2) continue;
        double2 acc = make_double2(0.0, 0.0);
        for (int rho = t2; rho <= t1 + b - 1; ++rho) acc = zadd(acc, zcmul(Vs[t1][rho - t1], Vs[t2][rho - t2]));
        Gs[t1][t2] = acc;
    }
    __syncthreads();
    for (int c = 0; c < g; ++c) {
        double2 tc = taus[c];
        if (tid < c) {
            double2 acc = make_double2(0.0, 0.0);
            for (int l = tid; l < c; ++l) acc = zadd(acc, zmul(Ts[tid][l], Gs[l][c]));
            Ts[tid][c] = zmul(make_double2(-tc.x, -tc.y), acc);
        }
        if (tid == 0) Ts[c][c] = tc;
        __syncthreads();
    }
    E *tout = T2 + (size_t)grp * g * g;
    for (int t = tid; t < g * g; t += 256) tout[t] = El<E>::from(Ts[t % g][t / g]);   // column-major g x g
}

// Y (n x m) <- Q2 Y (or Q2^H Y) on MFMA tiles.  A complex block product is
// three real MFMAs (3M form): v_mfma_f64_16x16x4f64 for double storage,
// v_mfma_f32_16x16x4f32 (fp32 accumulation) for float storage.
typedef double q2v4d __attribute__((ext_vector_type(4)));
typedef float q2v4f __attribute__((ext_vector_type(4)));

template <class E> struct Q2M;
template <> struct Q2M<double2> {
    typedef q2v4d Acc;
    __device__ static Acc mfma(double a, double b, Acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // lane l, register r of the 16x16 result -> row l/16 + 4r, column l%16
    __device__ static int orow(int lk, int r) { return lk + 4 * r; }
};
template <> struct Q2M<float2> {
    typedef q2v4f Acc;
    __device__ static Acc mfma(float a, float b, Acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // lane l, register r of the 16x16 result -> row 4(l/16) + r, column l%16
    __device__ static int orow(int lk, int r) { return 4 * lk + r; }
};

// complex block product in the 3M form (see gemm.hip): P1 += Ar Br,
// P2 += Ai Bi, P3 += (Ar + Ai)(Br + Bi); re = P1 - P2, im = P3 - P1 - P2
template <class E>
__device__ inline void q2_cmfma(E a, E b, typename Q2M<E>::Acc &p1, typename Q2M<E>::Acc &p2,
                                typename Q2M<E>::Acc &p3) {
    p1 = Q2M<E>::mfma(a.x, b.x, p1);
    p2 = Q2M<E>::mfma(a.y, b.y, p2);
    p3 = Q2M<E>::mfma(a.x + a.y, b.x + b.y, p3);
}

// Wavefront schedule.  Group (B, j) overlaps groups of later blocks only at
// j' <= j and groups of earlier blocks only at j' >= j, and (B, j') for
// |j' - j| = 1; so the groups with (ngrp - 1 - B) + j = w (one anti-diagonal
// of the (B, j) grid) touch pairwise disjoint rows, and applying the
// anti-diagonals w = 0, 1, ... in turn (every group of one of them in
// parallel) keeps every overlapping pair in the order of Q2; Q2^H runs the
// anti-diagonals in reverse.  One launch per anti-diagonal; a workgroup applies
// one group to 32 columns of Y:
//   Y_rows (g+b-1 rows) -> LDS,
//   W  = V^H Y_rows   (four 16x16 tiles, one per wave, whole k range),
//   W2 = T W          (T^H W for Q2^H; T read into registers up front),
//   Y_rows -= V W2    (twelve 16x16 tiles, three per wave, results to LDS),
//   Y_rows -> Y       (column-contiguous stores).
// V and T are read straight into MFMA operand registers from memory that the
// column tiles of the group share; the tiles of one group are given
// consecutive workgroup slots of one XCD, so they share that XCD's L2.  All
// operand loads are unconditional (clamped address, zeroed after), so a
// wave's loads are in flight together.
constexpr int Q2WF_NC = 32;

template <int BMAX, class E>
__global__ __launch_bounds__(256, 2) void q2_wf_kernel(int n, int m, int b, int g, int J, int Bt, int jlo, int ngs,
                                                        int adj, const E *V2, const E *T2, E *Y, int ldy) {
    typedef typename Q2M<E>::Acc Acc;
    constexpr int NC = Q2WF_NC, GM = 32, RM = 96;
    constexpr int K1 = (BMAX + 15 + 3) / 4;   // k-steps of a W tile
    __shared__ E Ys[RM][NC + 1];
    __shared__ E Ws[GM][NC + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int ct = (m + NC - 1) / NC;
    const int items = ngs * ct;
    // item p = (group, column tile); the 8 XCDs take contiguous ranges of p
    const int per = (items + 7) / 8;
    const int p = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (p >= items) return;
    const int j = jlo + p / ct, c0 = (p % ct) * NC;
    const int nc = min(NC, m - c0);
    const int B = Bt + j, s0 = B * g;
    const int R0 = s0 + 1 + j * b;
    const int nrows = min(g + b - 1, n - R0);
    const E *tg = T2 + ((size_t)B * J + j) * g * g;
    const E zero = El<E>::mk(0.0, 0.0);
    const int sblk = s0 / b, soff = s0 % b;
    // V(r, t): row r of the group's parallelogram, reflector t (sweep s0 + t)
    // (a ternary on the vector type would be compiled as a select of addresses
    // through scratch memory, so values are selected per component)
    auto keep = [](bool in, E v) -> E { return El<E>::mk(in ? v.x : 0.0, in ? v.y : 0.0); };
    auto vld = [&](bool ok, int r, int t) -> E {
        const int i = r - t;
        int sb = soff + t, blk = sblk;
        if (sb >= b) {
            sb -= b;
            ++blk;
        }
        const bool in = ok && t < g && i >= 0 && i < b && s0 + t <= n - 2;
        return keep(in, V2[in ? (((size_t)blk * J + j) * b + sb) * b + i : 0]);
    };
    auto tld = [&](bool ok, int row, int col) -> E {
        const bool in = ok && row < g && col < g;
        const E v = keep(in, tg[in ? (adj ? col + (size_t)row * g : row + (size_t)col * g) : 0]);
        return El<E>::mk(v.x, adj ? -v.y : v.y);
    };
    // wave -> (t tile, column tile) of W and W2
    const int t0 = 16 * (wave & 1), cc = 16 * (wave >> 1);
    // step-2 operands, loaded first
    const int lbeg = adj ? 0 : t0, lend = adj ? t0 + 16 : GM;
    E tv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) tv[u] = tld(lbeg + 4 * u < lend, t0 + lr, lbeg + 4 * u + lk);
    // step-1 operands conj(V)
    const int nks = (min(RM, t0 + 15 + b) - t0 + 3) / 4;
    E a1[K1];
#pragma unroll
    for (int q = 0; q < K1; ++q) {
        const E v = vld(q < nks, t0 + 4 * q + lk, t0 + lr);
        a1[q] = El<E>::mk(v.x, -v.y);
    }
    // Y rows -> LDS
    {
        E yv[RM * NC / 256];
#pragma unroll
        for (int u = 0; u < RM * NC / 256; ++u) {
            const int t = tid + 256 * u, r = t % RM, c = t / RM;
            const bool in = r < nrows && c < nc;
            yv[u] = keep(in, Y[in ? R0 + r + (size_t)(c0 + c) * ldy : (size_t)R0 + (size_t)c0 * ldy]);
        }
#pragma unroll
        for (int u = 0; u < RM * NC / 256; ++u) {
            const int t = tid + 256 * u;
            Ys[t % RM][t / RM] = yv[u];
        }
    }
    __syncthreads();
    // step 1: W tile (t0, cc) = V(:, t0..t0+15)^H Y_rows(:, cc..cc+15); even and odd
    // k-steps go to two sets of accumulators (six independent MFMA chains), added
    // at the end
    {
        Acc p[2][3];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int c = 0; c < 3; ++c) p[h][c] = Acc{0, 0, 0, 0};
#pragma unroll
        for (int q = 0; q < K1; ++q)
            if (q < nks) q2_cmfma<E>(a1[q], Ys[t0 + 4 * q + lk][cc + lr], p[q & 1][0], p[q & 1][1], p[q & 1][2]);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const auto p1 = p[0][0][i] + p[1][0][i], p2 = p[0][1][i] + p[1][1][i], p3 = p[0][2][i] + p[1][2][i];
            Ws[t0 + Q2M<E>::orow(lk, i)][cc + lr] = El<E>::mk(p1 - p2, p3 - p1 - p2);
        }
    }
    // step-3 operands of this wave's first row tile
    const int c3 = 16 * (wave & 1), q3 = wave >> 1;
    struct Ops8 {
        E v[8];
    };
    auto load3 = [&](int r0) {
        Ops8 a;
        const int tlo = max(0, r0 - b + 1) & ~3, thi = min(GM, r0 + 16);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int t4 = tlo + 4 * u;
            const E v = vld(t4 < thi && r0 < nrows, r0 + lr, t4 + lk);
            a.v[u] = El<E>::mk(-v.x, -v.y);
        }
        return a;
    };
    // all three row tiles' operands, loaded together
    Ops8 a3[3];
#pragma unroll
    for (int u = 0; u < 3; ++u) a3[u] = load3(16 * (q3 + 2 * u));
    __syncthreads();
    // step 2: W2 tile (t0, cc) = T(t0.., :) W(:, cc..)  (T upper triangular; T^H lower)
    {
        Acc p1 = {0, 0, 0, 0}, p2 = {0, 0, 0, 0}, p3 = {0, 0, 0, 0};
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (lbeg + 4 * u < lend) q2_cmfma<E>(tv[u], Ws[lbeg + 4 * u + lk][cc + lr], p1, p2, p3);
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 4; ++i) Ws[t0 + Q2M<E>::orow(lk, i)][cc + lr] = El<E>::mk(p1[i] - p2[i], p3[i] - p1[i] - p2[i]);
    }
    __syncthreads();
    // step 3: row tiles q3, q3 + 2, q3 + 4 of column tile c3, interleaved (nine
    // independent MFMA chains)
    {
        Acc p[3][3];
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            const int r0 = 16 * (q3 + 2 * u);
            p[u][1] = Acc{0, 0, 0, 0};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const E y = Ys[r0 + Q2M<E>::orow(lk, i)][c3 + lr];
                p[u][0][i] = y.x;
                p[u][2][i] = y.x + y.y;
            }
        }
#pragma unroll
        for (int v = 0; v < 8; ++v)
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                const int r0 = 16 * (q3 + 2 * u);
                const int tlo = max(0, r0 - b + 1) & ~3, thi = min(GM, r0 + 16);
                if (r0 < nrows && tlo + 4 * v < thi)
                    q2_cmfma<E>(a3[u].v[v], Ws[tlo + 4 * v + lk][c3 + lr], p[u][0], p[u][1], p[u][2]);
            }
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            const int r0 = 16 * (q3 + 2 * u);
            if (r0 < nrows) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const auto p1 = p[u][0][i], p2 = p[u][1][i], p3 = p[u][2][i];
                    Ys[r0 + Q2M<E>::orow(lk, i)][c3 + lr] = El<E>::mk(p1 - p2, p3 - p1 - p2);
                }
            }
        }
    }
    __syncthreads();
    for (int t = tid; t < nrows * NC; t += 256) {
        const int r = t % nrows, c = t / nrows;
        if (c < nc) Y[R0 + r + (size_t)(c0 + c) * ldy] = Ys[r][c];
    }
}

// Register-resident variant for complex double.  For v_mfma_f64_16x16x4f64
// the accumulator layout (lane (lk, lr), register i -> row lk + 4 i, column lr)
// is the B-operand layout of k-step i (row 4 i + lk, column lr), so one wave
// keeps its 16 columns of Y_rows, of W = V^H Y_rows and of W2 = T W in
// registers from one step to the next: Y_rows is the B operand of step 1 and
// the accumulator of step 3, W is the B operand of step 2, W2 that of step 3.
// The four waves of a workgroup take 64 consecutive columns and share the
// group's V (reflector-major, Vc[t * b + i] = entry i of reflector t) and T
// (column-major), copied into LDS by LDS-direct loads (no registers, all in
// flight with the Y loads); operand reads mask what lies outside the
// parallelogram.  With pitch b the two V operand patterns of a 16-lane group
// hit 16 distinct bank groups.
constexpr int Q2R_NC = 64;

template <int BMAX>
__global__ __launch_bounds__(256, 2) void q2_reg_kernel(int n, int m, int b, int g, int J, int Bt, int jlo, int ngs,
                                                         int adj, const double2 *V2, const double2 *T2, double2 *Y,
                                                         int ldy) {
    typedef q2v4d Acc;
    constexpr int GM = 32;
    constexpr int RQ = (GM + BMAX - 1 + 3) / 4;   // k-steps (4 rows each) covering the group's rows
    __shared__ double2 Vc[GM * BMAX];
    __shared__ double2 Tc[GM * GM];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int ct = (m + Q2R_NC - 1) / Q2R_NC;
    const int items = ngs * ct;
    const int per = (items + 7) / 8;
    const int p = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (p >= items) return;
    const int j = jlo + p / ct, c0 = (p % ct) * Q2R_NC;
    const int cw = c0 + 16 * wave + lr;           // this lane's column
    const bool colok = cw < m;
    const int B = Bt + j, s0 = B * g;
    const int R0 = s0 + 1 + j * b;
    const int nrows = min(g + b - 1, n - R0);
    const int tmax = min(g, n - 1 - s0);          // reflectors of the group that exist
    const double2 *tg = T2 + ((size_t)B * J + j) * g * g;
    const int sblk = s0 / b, soff = s0 % b;
    auto keep = [](bool in, double2 v) { return make_double2(in ? v.x : 0.0, in ? v.y : 0.0); };
    // V and T into LDS (element e of the copy: lane e % 64 of instruction e / 64)
#pragma unroll
    for (int u = 0; u < GM * BMAX / 256; ++u) {
        const int e = 256 * u + 64 * wave + lane, t = e / b, i = e % b;
        int sb = soff + t, blk = sblk;
        if (sb >= b) {
            sb -= b;
            ++blk;
        }
        const bool in = e < g * b && t < tmax;
        const double2 *src = V2 + (in ? (((size_t)blk * J + j) * b + sb) * b + i : 0);
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)src,
                                         (__attribute__((address_space(3))) void *)(&Vc[256 * u + 64 * wave]), 16, 0,
                                         0);
    }
#pragma unroll
    for (int u = 0; u < GM * GM / 256; ++u) {
        const int e = 256 * u + 64 * wave + lane;
        const double2 *src = tg + (e < g * g ? e : 0);
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)src,
                                         (__attribute__((address_space(3))) void *)(&Tc[256 * u + 64 * wave]), 16, 0,
                                         0);
    }
    // Y rows of this lane (B-operand layout): y[q] = Y(R0 + 4q + lk, cw)
    double2 y[RQ];
#pragma unroll
    for (int q = 0; q < RQ; ++q) {
        const int r = 4 * q + lk;
        const bool in = colok && r < nrows;
        y[q] = keep(in, Y[in ? R0 + r + (size_t)cw * ldy : (size_t)R0 + (size_t)c0 * ldy]);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    // V(r, t) (zero outside the parallelogram and past the last reflector)
    auto vget = [&](int r, int t) {
        const int i = r - t;
        const bool in = i >= 0 && i < b && t < tmax;
        return keep(in, Vc[in ? t * b + i : 0]);
    };
    // T(row, col), or T^H for Q2^H (zero outside g x g)
    auto tget = [&](int row, int col) {
        const bool in = row < g && col < g;
        const double2 v = keep(in, Tc[in ? (adj ? col + row * g : row + col * g) : 0]);
        return make_double2(v.x, adj ? -v.y : v.y);
    };
    auto combine = [](const Acc &p1, const Acc &p2, const Acc &p3, int i) {
        return make_double2(p1[i] - p2[i], p3[i] - p1[i] - p2[i]);
    };
    // step 1: W (32 x 16) = V^H Y_rows, one t tile after the other
    double2 w[2][4];
#pragma unroll
    for (int tt = 0; tt < 2; ++tt) {
        Acc p1 = {0, 0, 0, 0}, p2 = {0, 0, 0, 0}, p3 = {0, 0, 0, 0};
        constexpr int QS = (15 + BMAX + 3) / 4;   // k-steps of one t tile
#pragma unroll
        for (int q = 0; q < RQ; ++q)
            if (q >= 4 * tt && q < 4 * tt + QS) {
                const double2 v = vget(4 * q + lk, 16 * tt + lr);
                q2_cmfma<double2>(make_double2(v.x, -v.y), y[q], p1, p2, p3);
            }
#pragma unroll
        for (int i = 0; i < 4; ++i) w[tt][i] = combine(p1, p2, p3, i);
    }
    // step 2: W2 = T W (T upper triangular; T^H lower for Q2^H)
    double2 w2[2][4];
#pragma unroll
    for (int tt = 0; tt < 2; ++tt) {
        Acc p1 = {0, 0, 0, 0}, p2 = {0, 0, 0, 0}, p3 = {0, 0, 0, 0};
#pragma unroll
        for (int kq = 0; kq < 8; ++kq)
            if (adj ? kq <= 4 * tt + 3 : kq >= 4 * tt)
                q2_cmfma<double2>(tget(16 * tt + lr, 4 * kq + lk), w[kq >> 2][kq & 3], p1, p2, p3);
#pragma unroll
        for (int i = 0; i < 4; ++i) w2[tt][i] = combine(p1, p2, p3, i);
    }
    // step 3: Y_rows -= V W2, row tile rt accumulates into y[4 rt .. 4 rt + 3]
#pragma unroll
    for (int rt = 0; rt < RQ / 4; ++rt) {
        if (16 * rt >= nrows) continue;
        Acc p1, p2 = {0, 0, 0, 0}, p3;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            p1[i] = y[4 * rt + i].x;
            p3[i] = y[4 * rt + i].x + y[4 * rt + i].y;
        }
        const int tlo = max(0, 16 * rt - b + 1), thi = min(GM, 16 * rt + 16);
#pragma unroll
        for (int kq = 0; kq < 8; ++kq)
            if (4 * kq + 3 >= tlo && 4 * kq < thi) {
                const double2 v = vget(16 * rt + lr, 4 * kq + lk);
                q2_cmfma<double2>(make_double2(-v.x, -v.y), w2[kq >> 2][kq & 3], p1, p2, p3);
            }
#pragma unroll
        for (int i = 0; i < 4; ++i) y[4 * rt + i] = combine(p1, p2, p3, i);
    }
#pragma unroll
    for (int q = 0; q < RQ; ++q) {
        const int r = 4 * q + lk;
        if (colok && r < nrows) Y[R0 + r + (size_t)cw * ldy] = y[q];
    }
}

// Groups of g = 32 reflectors (band width 32 .. 64) on a pipelined schedule:
// one persistent workgroup per CU and launch takes a contiguous run of the
// launch's items (group, 64-column tile), group-major, so consecutive items
// share the group's V (copied into LDS when the group changes) and T (held in
// registers).  While item i is computed from registers, the rows of item i + 1
// are copied into an LDS buffer by LDS-direct loads: the HBM traffic of the
// next item overlaps the MFMAs of this one, and no operand read needs a mask.
// V lives in LDS as a zero-padded parallelogram, Vd[t * VP + r] = V(r, t) for
// the window rows r (zero outside rows t .. t + b - 1 and for reflectors past
// the last sweep), with an odd pitch VP so that both operand patterns of a
// 16-lane group (lanes stepping through reflectors, or through rows) hit
// distinct bank groups; the row buffer keeps column c of the tile at
// Yb[c * YP] with the same odd pitch.  The zero padding is written once per
// workgroup; each group overwrites only its parallelogram.
template <int BMAX> struct Q2F {
    static constexpr int GM = 32, WR = GM + BMAX - 1, RQ = (WR + 3) / 4, VP = 4 * RQ + 1, YP = 4 * RQ + 1;
};

template <int BMAX>
__device__ inline void q2f_zero(double2 *Vd) {
    for (int e = threadIdx.x; e < 32 * Q2F<BMAX>::VP; e += 256) Vd[e] = make_double2(0.0, 0.0);
}

// LDS-direct copy of the reflectors of group (B, j): wave w copies reflectors
// t = 8 w .. 8 w + 7 (lane i -> entry i); reflectors past the last sweep are zeroed
template <int BMAX>
__device__ inline void q2f_stage_v(double2 *Vd, const double2 *V2, int b, int J, int B, int j, int tmax) {
    constexpr int VP = Q2F<BMAX>::VP;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int t = 8 * wave + u, s = B * 32 + t;
        if (t < tmax) {
            if (lane < b)
                __builtin_amdgcn_global_load_lds(
                    (const __attribute__((address_space(1))) void *)(V2 + (((size_t)(s / b) * J + j) * b + s % b) * b +
                                                                     lane),
                    (__attribute__((address_space(3))) void *)(&Vd[t * VP + t]), 16, 0, 0);
        } else if (lane < b) {
            Vd[t * VP + t + lane] = make_double2(0.0, 0.0);
        }
    }
}

// T operands of step 2 in registers: tr[tt][kq] = T(16 tt + lr, 4 kq + lk), or
// T(4 kq + lk, 16 tt + lr) for Q2^H (conjugated in the product); T upper
// triangular.  tget(tt, kq) in q2f_apply returns the same operand.
template <int ADJ>
__device__ inline void q2f_load_t(double2 (&tr)[2][8], const double2 *T2, int J, int B, int j) {
    const int lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
    const double2 *tg = T2 + ((size_t)B * J + j) * 32 * 32;
#pragma unroll
    for (int tt = 0; tt < 2; ++tt)
#pragma unroll
        for (int kq = 0; kq < 8; ++kq)
            if (ADJ ? kq <= 4 * tt + 3 : kq >= 4 * tt)
                tr[tt][kq] = ADJ ? tg[4 * kq + lk + 32 * (16 * tt + lr)] : tg[16 * tt + lr + 32 * (4 * kq + lk)];
}

// Apply one group to the wave's 16 columns of Y_rows held in y (rows 4 q + lk
// of the window, column lr): W = V^H Y_rows, W2 = T W (T^H W for Q2^H),
// Y_rows -= V W2.  Rows at or past nrows must hold zeros.  emit(rt) is called
// as soon as rows 16 rt .. 16 rt + 15 (y[4 rt .. 4 rt + 3]) are final, so
// their stores drain while the remaining tiles are computed.
template <int BMAX, int ADJ, class TGet, class Emit>
__device__ __attribute__((always_inline)) inline void q2f_apply(double2 (&y)[Q2F<BMAX>::RQ], const double2 *Vd,
                                                                TGet &&tget, int nrows, Emit &&emit) {
    typedef q2v4d Acc;
    constexpr int GM = 32, RQ = Q2F<BMAX>::RQ, VP = Q2F<BMAX>::VP;
    constexpr int QS = (15 + BMAX + 3) / 4;   // k-steps of one 16-reflector tile in step 1
    const int lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
    const double2 *v1 = Vd + lr * VP + lk;   // V(4 q + lk, 16 tt + lr) = v1[16 tt VP + 4 q]
    const double2 *v3 = Vd + lk * VP + lr;   // V(16 rt + lr, 4 kq + lk) = v3[4 kq VP + 16 rt]
    auto mm = [](double a, double c, Acc acc) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, c, acc, 0, 0, 0); };
    // step 1: W = V^H Y_rows.  With a = V unconjugated, sum conj(a) c =
    // (P1 + P2) + i (P3 - P1 + P2) for P1 = sum ar cr, P2 = sum ai ci,
    // P3 = sum (ar - ai)(cr + ci).
    double2 w[2][4];
#pragma unroll
    for (int tt = 0; tt < 2; ++tt) {
        Acc p1 = {0, 0, 0, 0}, p2 = {0, 0, 0, 0}, p3 = {0, 0, 0, 0};
        double2 av[QS];   // the tile's V operands, read before its products
#pragma unroll
        for (int q = 4 * tt; q < 4 * tt + QS && q < RQ; ++q) av[q - 4 * tt] = v1[16 * tt * VP + 4 * q];
#pragma unroll
        for (int q = 4 * tt; q < 4 * tt + QS && q < RQ; ++q) {
            const double2 a = av[q - 4 * tt];
            p1 = mm(a.x, y[q].x, p1);
            p2 = mm(a.y, y[q].y, p2);
            p3 = mm(a.x - a.y, y[q].x + y[q].y, p3);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) w[tt][i] = make_double2(p1[i] + p2[i], p3[i] - p1[i] + p2[i]);
    }
    // step 2: W2 = T W (T upper triangular) or T^H W (lower)
    double ws[8];
#pragma unroll
    for (int kq = 0; kq < 8; ++kq) ws[kq] = w[kq >> 2][kq & 3].x + w[kq >> 2][kq & 3].y;
    double2 wn[8];   // -W2, the B operand of step 3
#pragma unroll
    for (int tt = 0; tt < 2; ++tt) {
        Acc p1 = {0, 0, 0, 0}, p2 = {0, 0, 0, 0}, p3 = {0, 0, 0, 0};
#pragma unroll
        for (int kq = 0; kq < 8; ++kq) {
            if (ADJ ? kq > 4 * tt + 3 : kq < 4 * tt) continue;
            const double2 a = tget(tt, kq);
            const double2 c = w[kq >> 2][kq & 3];
            p1 = mm(a.x, c.x, p1);
            p2 = mm(a.y, c.y, p2);
            p3 = mm(ADJ ? a.x - a.y : a.x + a.y, ws[kq], p3);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
            wn[4 * tt + i] = ADJ ? make_double2(-(p1[i] + p2[i]), -(p3[i] - p1[i] + p2[i]))
                                 : make_double2(p2[i] - p1[i], p1[i] + p2[i] - p3[i]);
    }
    double wns[8];
#pragma unroll
    for (int kq = 0; kq < 8; ++kq) wns[kq] = wn[kq].x + wn[kq].y;
    // step 3: Y_rows += V (-W2), row tile rt accumulating into y[4 rt .. 4 rt + 3]
#pragma unroll
    for (int rt = 0; rt < RQ / 4; ++rt) {
        if (16 * rt >= nrows) continue;
        // reflectors whose rows meet the tile for band width BMAX (a superset
        // for narrower bands, whose extra entries are zeros of the padding);
        // the tile's V operands are read before its products
        const int TLO = max(0, 16 * rt - BMAX + 1), THI = min(GM, 16 * rt + 16);
        double2 av[8];
#pragma unroll
        for (int kq = 0; kq < 8; ++kq)
            if (4 * kq + 3 >= TLO && 4 * kq < THI) av[kq] = v3[4 * kq * VP + 16 * rt];
        Acc p1, p2 = {0, 0, 0, 0}, p3;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            p1[i] = y[4 * rt + i].x;
            p3[i] = y[4 * rt + i].x + y[4 * rt + i].y;
        }
#pragma unroll
        for (int kq = 0; kq < 8; ++kq)
            if (4 * kq + 3 >= TLO && 4 * kq < THI) {
                const double2 a = av[kq];
                p1 = mm(a.x, wn[kq].x, p1);
                p2 = mm(a.y, wn[kq].y, p2);
                p3 = mm(a.x + a.y, wns[kq], p3);
            }
#pragma unroll
        for (int i = 0; i < 4; ++i) y[4 * rt + i] = make_double2(p1[i] - p2[i], p3[i] - p1[i] - p2[i]);
        emit(rt);
    }
}

template <int BMAX, int ADJ>
__global__ __launch_bounds__(256, 1) void q2_pipe_kernel(int n, int m, int b, int J, int Bt, int jlo, int ngs,
                                                          const double2 *V2, const double2 *T2, double2 *Y,
                                                          int ldy) {
    constexpr int RQ = Q2F<BMAX>::RQ, YP = Q2F<BMAX>::YP, VP = Q2F<BMAX>::VP;
    constexpr int YE = 64 * YP;   // elements of the row buffer (64 columns)
    __shared__ double2 Vd[32 * VP];
    __shared__ double2 Yb[YE];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int ct = (m + Q2R_NC - 1) / Q2R_NC, items = ngs * ct;
    const int G = gridDim.x;                      // a multiple of 8
    const int p = (blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);
    const int per = (items + G - 1) / G;
    const int i0 = p * per, i1 = min(items, i0 + per);
    if (i0 >= i1) return;
    q2f_zero<BMAX>(Vd);
    // rows of item it into Yb; entries outside the matrix read row R0 of
    // column c0 and are masked when the rows are taken into registers
    auto fetch = [&](int it) {
        const int j = jlo + it / ct, c0 = (it % ct) * Q2R_NC;
        const int R0 = (Bt + j) * 32 + 1 + j * b;
        const int nr = min(31 + b, n - R0);
#pragma unroll
        for (int u = 0; u < (YE + 255) / 256; ++u) {
            if (256 * u + 64 * wave >= YE) continue;   // uniform within the wave
            const int e = 256 * u + 64 * wave + lane, c = e / YP, r = e % YP;
            const bool ok = r < nr && c0 + c < m;
            const double2 *src = Y + (ok ? R0 + r + (size_t)(c0 + c) * ldy : R0 + (size_t)c0 * ldy);
            __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)src,
                                             (__attribute__((address_space(3))) void *)(&Yb[256 * u + 64 * wave]),
                                             16, 0, 0);
        }
    };
    double2 tr[2][8];
    int cur = -1;
    fetch(i0);
    for (int it = i0; it < i1; ++it) {
        const int j = jlo + it / ct, c0 = (it % ct) * Q2R_NC;
        const int B = Bt + j, s0 = B * 32;
        const int R0 = s0 + 1 + j * b;
        const int nrows = min(31 + b, n - R0);
        if (j != cur) {
            __syncthreads();   // the previous group's V is no longer read (first time: zero fill done)
            q2f_stage_v<BMAX>(Vd, V2, b, J, B, j, min(32, n - 1 - s0));
            q2f_load_t<ADJ>(tr, T2, J, B, j);
            cur = j;
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        const int cw = c0 + 16 * wave + lr;
        const bool colok = cw < m;
        double2 y[RQ];
#pragma unroll
        for (int q = 0; q < RQ; ++q) {
            const double2 v = Yb[(16 * wave + lr) * YP + 4 * q + lk];
            const bool in = colok && 4 * q + lk < nrows;
            y[q] = make_double2(in ? v.x : 0.0, in ? v.y : 0.0);
        }
        __syncthreads();   // every wave holds its rows: the buffer may be refilled
        if (it + 1 < i1) fetch(it + 1);
        double2 *ycol = Y + (size_t)(colok ? cw : c0) * ldy + R0;
        q2f_apply<BMAX, ADJ>(y, Vd, [&](int tt, int kq) { return tr[tt][kq]; }, nrows, [&](int rt) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = 16 * rt + 4 * i + lk;
                if (colok && r < nrows) ycol[r] = y[4 * rt + i];
            }
        });
    }
}

// reflectors per group (sweeps s0 .. s0 + g - 1 at one step j)
static int q2_group(int b) { return std::min(b, 32); }

size_t q2_t_elems(int n, int nb) {
    const int g = q2_group(nb);
    const int ngrp = n >= 2 ? cdiv(n - 1, g) : 0;
    return std::max<size_t>((size_t)ngrp * hb_J(n, nb) * g * g, 1);
}

template <class E>
void q2_build_t(hgv_ctx_s *ctx, int n, int nb, const E *V2, const E *tau2, E *T2) {
    if (nb > 64) throw HipFail{hipErrorInvalidValue};
    if (n < 2) return;
    const int b = nb, g = q2_group(b);
    const int J = hb_J(n, b), ngrp = cdiv(n - 1, g);
    if (b <= 32)
        hipLaunchKernelGGL((q2_tbuild_kernel<32, 32, E>), dim3(ngrp * J), dim3(256), 0, ctx->stream, n, b, g, J, V2,
                           tau2, T2);
    else
        hipLaunchKernelGGL((q2_tbuild_kernel<64, 32, E>), dim3(ngrp * J), dim3(256), 0, ctx->stream, n, b, g, J, V2,
                           tau2, T2);
    HGV_LAUNCH_CHECK();
}

template <class E>
void q2_apply_t(hgv_ctx_s *ctx, int n, int nb, int m, const E *V2, const E *T2, E *Y, int ldy, bool adj) {
    if (nb > 64) throw HipFail{hipErrorInvalidValue};
    if (n < 2 || m == 0) return;
    const int b = nb, g = q2_group(b);
    const int J = hb_J(n, b), ngrp = cdiv(n - 1, g);
    // anti-diagonal w holds the groups B = ngrp - 1 - w + j with j in
    // [max(0, w - ngrp + 1), min(w, J - 1)] and j < jn(B); the valid j form a prefix
    const int nw = ngrp + J - 1, ct = cdiv(m, Q2WF_NC);
    int pipe_grid = 0;   // one workgroup per CU (a multiple of 8) for the pipelined kernel
    if (std::is_same<E, double2>::value && g == 32) {
        HGV_HIP(hipDeviceGetAttribute(&pipe_grid, hipDeviceAttributeMultiprocessorCount, ctx->device));
        pipe_grid = std::max(8, pipe_grid / 8 * 8);
    }
    for (int wi = 0; wi < nw; ++wi) {
        const int w = adj ? nw - 1 - wi : wi;
        const int Bt = ngrp - 1 - w;
        const int jlo = std::max(0, -Bt);
        int jhi = std::min(w, J - 1);
        while (jhi >= jlo) {
            const int s0 = (Bt + jhi) * g;
            if (s0 <= n - 2 && jhi <= (n - 2 - s0) / b) break;
            --jhi;
        }
        if (jhi < jlo) continue;
        const int ngs = jhi - jlo + 1;
        if constexpr (std::is_same<E, double2>::value) {
            const int grid = 8 * cdiv(ngs * cdiv(m, Q2R_NC), 8);
            if (g == 32) {
                int n_ = n, m_ = m, b_ = b, J_ = J, Bt_ = Bt, jlo_ = jlo, ngs_ = ngs, ldy_ = ldy;
                const double2 *V2_ = V2, *T2_ = T2;
                double2 *Y_ = Y;
                void *args[] = {&n_, &m_, &b_, &J_, &Bt_, &jlo_, &ngs_, &V2_, &T2_, &Y_, &ldy_};
                void *kern = b <= 32 ? (adj ? reinterpret_cast<void *>(q2_pipe_kernel<32, 1>)
                                            : reinterpret_cast<void *>(q2_pipe_kernel<32, 0>))
                                     : (adj ? reinterpret_cast<void *>(q2_pipe_kernel<64, 1>)
                                            : reinterpret_cast<void *>(q2_pipe_kernel<64, 0>));
                HGV_HIP(hipLaunchKernel(kern, dim3(pipe_grid), dim3(256), args, 0, ctx->stream));
            } else {
                hipLaunchKernelGGL((q2_reg_kernel<32>), dim3(grid), dim3(256), 0, ctx->stream, n, m, b, g, J, Bt,
                                   jlo, ngs, (int)adj, V2, T2, Y, ldy);
            }
        } else {
            const int grid = 8 * cdiv(ngs * ct, 8);
            if (b <= 32)
                hipLaunchKernelGGL((q2_wf_kernel<32, E>), dim3(grid), dim3(256), 0, ctx->stream, n, m, b, g, J, Bt,
                                   jlo, ngs, (int)adj, V2, T2, Y, ldy);
            else
                hipLaunchKernelGGL((q2_wf_kernel<64, E>), dim3(grid), dim3(256), 0, ctx->stream, n, m, b, g, J, Bt,
                                   jlo, ngs, (int)adj, V2, T2, Y, ldy);
        }
        HGV_LAUNCH_CHECK();
    }
}

template <class E>
void unmtr_q2_t(hgv_ctx_s *ctx, int n, int nb, int m, const E *V2, const E *tau2, E *Y, int ldy, bool adj,
                Arena &ar) {
    if (nb > 64) throw HipFail{hipErrorInvalidValue};
    E *T2 = ar.take<E>(q2_t_elems(n, nb));
    if (ar.measuring() || n < 2 || m == 0) return;
    q2_build_t<E>(ctx, n, nb, V2, tau2, T2);
    q2_apply_t<E>(ctx, n, nb, m, V2, T2, Y, ldy, adj);
}

template void unmtr_q2_t<double2>(hgv_ctx_s *, int, int, int, const double2 *, const double2 *, double2 *, int, bool,
                                  Arena &);
template void unmtr_q2_t<float2>(hgv_ctx_s *, int, int, int, const float2 *, const float2 *, float2 *, int, bool,
                                 Arena &);
template void q2_build_t<float2>(hgv_ctx_s *, int, int, const float2 *, const float2 *, float2 *);
template void q2_build_t<double2>(hgv_ctx_s *, int, int, const double2 *, const double2 *, double2 *);
template void q2_apply_t<double2>(hgv_ctx_s *, int, int, int, const double2 *, const double2 *, double2 *, int,
                                  bool);
template void q2_apply_t<float2>(hgv_ctx_s *, int, int, int, const float2 *, const float2 *, float2 *, int, bool);

}  // namespace hgv
