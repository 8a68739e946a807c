// stebz.hip -- eigenvalues of the real symmetric tridiagonal T = (d, e) by
// Sturm counts: the eigenvalues-only path of the solver (Alg. 2 step 2 when no
// eigenvectors are wanted; Sec. 1: a fraction of the spectrum) and the
// selection of eigenpairs by a value range (vl, vu].
//
// Sturm count.  For a shift x the LDL^T factorisation of T - xI has pivots
//   q_0 = d_0 - x,   q_i = (d_i - x) - e_{i-1}^2 / q_{i-1},
// and by Sylvester's law of inertia the number of negative pivots is the number
// of eigenvalues below x.  A pivot smaller in modulus than pivmin is replaced by
// -pivmin (so the recurrence never divides by zero); the count computed in
// floating point is then the exact count of a matrix whose entries differ from
// T's by a few ulps (Kahan; Demmel, Dhillon and Ren, Parallel Computing 21
// (1995)), so an eigenvalue located by counts is accurate to O(eps ||T||).
//
// Multisection.  A group of MSG lanes owns one wanted eigenvalue k.  Its
// interval [lo, hi] keeps count(lo) < k <= count(hi); each round the lanes
// evaluate the counts at MSG interior points that split it into MSG + 1 equal
// parts, and the group keeps the part whose ends still bracket the k-th
// eigenvalue (a ballot over the group finds the first point with count >= k).
// One round shrinks the interval 17-fold, so about 14 rounds reach eps ||T||
// from the Gershgorin interval, where bisection needs 53.
#include <cfloat>
#include <mutex>
#include <vector>

#include "hgv_internal.h"

namespace hgv {

constexpr int MSG = 16;   // lanes (evaluation points) per eigenvalue

struct TriBounds {
    double lo, hi;     // Gershgorin interval, widened
    double tnorm;      // max(|gl|, |gu|)
    double pivmin;     // smallest admissible pivot modulus
};

// e2 = e^2 and the Gershgorin bounds (one workgroup; fixed-order reductions).
__global__ __launch_bounds__(256) void tri_prep_kernel(int n, const double *d, const double *e, double *e2,
                                                       TriBounds *tb) {
    __shared__ double smin[256], smax[256], se2[256];
    const int tid = threadIdx.x;
    double gl = __builtin_huge_val(), gu = -__builtin_huge_val(), m2 = 0.0;
    for (int i = tid; i < n; i += 256) {
        const double el = i > 0 ? fabs(e[i - 1]) : 0.0, er = i < n - 1 ? fabs(e[i]) : 0.0;
        gl = fmin(gl, d[i] - el - er);
        gu = fmax(gu, d[i] + el + er);
        if (i < n - 1) {
            const double s = e[i] * e[i];
            e2[i] = s;
            m2 = fmax(m2, s);
        }
    }
    smin[tid] = gl;
    smax[tid] = gu;
    se2[tid] = m2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) {
            smin[tid] = fmin(smin[tid], smin[tid + w]);
            smax[tid] = fmax(smax[tid], smax[tid + w]);
            se2[tid] = fmax(se2[tid], se2[tid + w]);
        }
        __syncthreads();
    }
    if (tid == 0) {
        const double l = smin[0], u = smax[0];
        const double tn = fmax(fabs(l), fabs(u));
        const double pivmin = DBL_MIN * fmax(1.0, se2[0]);
        const double pad = 2.0 * DBL_EPSILON * tn * n + 2.0 * pivmin;
        tb->lo = l - pad;
        tb->hi = u + pad;
        tb->tnorm = tn;
        tb->pivmin = pivmin;
    }
}

__device__ inline int sturm_count(int n, const double *d, const double *e2, double x, double pivmin) {
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    int c = q < 0.0 ? 1 : 0;
    for (int i = 1; i < n; ++i) {
        q = (d[i] - x) - e2[i - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        c += q < 0.0 ? 1 : 0;
    }
    return c;
}

// Index range of the eigenvalues in (vl, vu]: range[0] = il (1-based),
// range[1] = m (their number), range[2] = min(m, mmax) (the number returned).
__global__ __launch_bounds__(64) void sturm_range_kernel(int n, const double *d, const double *e2,
                                                         const TriBounds *tb, double vl, double vu, int mmax,
                                                         int *range) {
    __shared__ int cnt[2];
    const int lane = threadIdx.x;
    if (lane < 2) {
        // counts of the eigenvalues <= vl and <= vu: the count below the next
        // representable number above each end
        const double x = lane == 0 ? vl : vu;
        cnt[lane] = sturm_count(n, d, e2, nextafter(x, __builtin_huge_val()), tb->pivmin);
    }
    __syncthreads();
    if (lane == 0) {
        const int m = max(cnt[1] - cnt[0], 0);
        range[0] = cnt[0] + 1;
        range[1] = m;
        range[2] = min(m, mmax);
    }
}

// Eigenvalues il + s (s = 0, 1, ..., nslot - 1) into W[s].  With a device range
// (range != null) il = range[0] and only s < range[2] are computed; the other
// slots get 0.
__global__ __launch_bounds__(256) void multisect_kernel(int n, const double *d, const double *e2,
                                                        const TriBounds *tb, int il, int nslot, const int *range,
                                                        double *W) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int slot = g / MSG, j = g % MSG;
    const int glane = threadIdx.x & 63, gbase = glane & ~(MSG - 1);
    // every exit below is taken by whole lane groups (it depends on slot only)
    if (slot >= nslot) return;
    int first = il, valid = nslot;
    if (range) {
        first = range[0];
        valid = range[2];
    }
    if (slot >= valid) {
        if (j == 0) W[slot] = 0.0;
        return;
    }
    const int k = first + slot;   // 1-based index of the wanted eigenvalue
    double lo = tb->lo, hi = tb->hi;
    const double atol = DBL_EPSILON * tb->tnorm, pivmin = tb->pivmin;
    for (int round = 0; round < 64; ++round) {
        if (hi - lo <= 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + atol) break;
        const double h = (hi - lo) / (MSG + 1);
        const double x = lo + h * (j + 1);
        const int c = sturm_count(n, d, e2, x, pivmin);
        const unsigned long long bal = __ballot(c >= k);
        const unsigned grp = (unsigned)((bal >> gbase) & ((1ull << MSG) - 1));
        const int js = grp ? __builtin_ctz(grp) : MSG;   // first point with count >= k
        const double nlo = js == 0 ? lo : lo + h * js;
        const double nhi = js == MSG ? hi : lo + h * (js + 1);
        if (nlo == lo && nhi == hi) break;   // no representable progress
        lo = nlo;
        hi = nhi;
    }
    if (j == 0) W[slot] = 0.5 * (lo + hi);
}

void stebz_plan(int n, Arena &ar, double **e2, TriBounds **tb) {
    *e2 = ar.take<double>(std::max(n, 1));
    *tb = ar.take<TriBounds>(1);
}

void tri_prep(hgv_ctx_s *ctx, int n, const double *d, const double *e, double *e2, TriBounds *tb) {
    hipLaunchKernelGGL(tri_prep_kernel, dim3(1), dim3(256), 0, ctx->stream, n, d, e, e2, tb);
    HGV_LAUNCH_CHECK();
}

static void stebz_launch(hgv_ctx_s *ctx, int n, const double *d, const double *e, int il, int nslot,
                         const int *d_range, double *W, double *e2, TriBounds *tb) {
    if (n == 0 || nslot <= 0) return;
    tri_prep(ctx, n, d, e, e2, tb);
    hipLaunchKernelGGL(multisect_kernel, dim3(cdiv(nslot * MSG, 256)), dim3(256), 0, ctx->stream, n, d, e2, tb, il,
                       nslot, d_range, W);
    HGV_LAUNCH_CHECK();
}

void stebz_run(hgv_ctx_s *ctx, int n, const double *d, const double *e, int il, int nslot, const int *d_range,
               double *W, Arena &ar) {
    double *e2;
    TriBounds *tb;
    stebz_plan(n, ar, &e2, &tb);
    if (ar.measuring()) return;
    stebz_launch(ctx, n, d, e, il, nslot, d_range, W, e2, tb);
}

// ---- the allocation-free form -------------------------------------------------------------
// The scratch of the multisection (e^2 and the bounds) in a file-scope device
// array, so that a caller that cannot allocate (graph capture, serving loops)
// passes only its inputs and outputs.  Each device holds its own copy; its
// address is looked up once per device (stebz_scratch_init, from hgv_create
// with the device current) and only that address is ever handed to kernels.
// Every call on a device shares its copy: calls that overlap on one device
// race (the array keeps whatever the last call left; tri_prep rewrites all of
// it that a call reads).
static __device__ __align__(256) double scratch[STEBZ_NOALLOC_MAX + 64];

namespace {
std::mutex scratch_mu;
std::vector<double *> scratch_ptr;   // per device, null until looked up
}  // namespace

void stebz_scratch_init(int device) {
    std::lock_guard<std::mutex> lk(scratch_mu);
    if ((int)scratch_ptr.size() <= device) scratch_ptr.resize(device + 1, nullptr);
    if (scratch_ptr[device]) return;
    void *p = nullptr;
    HGV_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    scratch_ptr[device] = static_cast<double *>(p);
}

void stebz_noalloc_run(hgv_ctx_s *ctx, int n, const double *d, const double *e, int il, int nslot, double *W) {
    stebz_scratch_init(ctx->device);   // no-op after hgv_create
    double *base;
    {
        std::lock_guard<std::mutex> lk(scratch_mu);
        base = scratch_ptr[ctx->device];
    }
    // e^2 at the start, the bounds 256-byte aligned after STEBZ_NOALLOC_MAX doubles
    TriBounds *tb = reinterpret_cast<TriBounds *>(base + STEBZ_NOALLOC_MAX);
    stebz_launch(ctx, n, d, e, il, nslot, nullptr, W, base, tb);
}

void sturm_range_run(hgv_ctx_s *ctx, int n, const double *d, const double *e, double vl, double vu, int mmax,
                     int *d_range, Arena &ar) {
    double *e2;
    TriBounds *tb;
    stebz_plan(n, ar, &e2, &tb);
    if (ar.measuring() || n == 0) return;
    tri_prep(ctx, n, d, e, e2, tb);
    hipLaunchKernelGGL(sturm_range_kernel, dim3(1), dim3(64), 0, ctx->stream, n, d, e2, tb, vl, vu, mmax, d_range);
    HGV_LAUNCH_CHECK();
}

}  // namespace hgv
