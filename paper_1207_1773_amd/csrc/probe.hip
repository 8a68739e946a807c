// Device peak probes: the FP64 MFMA rate and the HBM copy bandwidth that
// kernels written like the solver's reach on this device.  They are the
// measured denominators of the roofline fractions, reported next to the
// published MI355X figures (78.6 TFLOP/s FP64 MFMA, 8 TB/s HBM3E).

#include <hip/hip_runtime.h>

#include <algorithm>

#include "hgv_internal.h"

namespace hgv {
namespace {

typedef double peak_v4d __attribute__((ext_vector_type(4)));

// Every wave runs 8 independent accumulator chains of v_mfma_f64_16x16x4f64
// (2048 flops each) for `iters` rounds with no memory traffic in the loop;
// the accumulators are folded into one store per lane so that the work is kept.
// (Two workgroups per CU in the launch bounds keep the accumulators in
// ordinary registers; without it the compiler moved them to accumulation
// registers and back on every round.)
__global__ __launch_bounds__(256, 2) void mfma_peak_kernel(int iters, double *out) {
    const int lane = threadIdx.x & 63;
    const double a = 1.0 + 1e-9 * lane, b = 1.0 - 1e-9 * lane;
    peak_v4d acc[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = peak_v4d{0.0, 0.0, 0.0, 0.0};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < 8; ++i) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[i], 0, 0, 0);
    }
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < 8; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
    out[(size_t)blockIdx.x * 256 + threadIdx.x] = s;
}

// Grid-stride copy with 16-byte loads and stores, eight in flight per thread.
__global__ __launch_bounds__(256) void copy_peak_kernel(const double2 *src, double2 *dst, size_t n) {
    const size_t stride = (size_t)gridDim.x * 256;
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    for (; i + 7 * stride < n; i += 8 * stride) {
        double2 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = src[i + u * stride];
#pragma unroll
        for (int u = 0; u < 8; ++u) dst[i + u * stride] = v[u];
    }
    for (; i < n; i += stride) dst[i] = src[i];
}

// Milliseconds of one launch (after one untimed launch of the same work).
template <class Launch>
double time_launch(hipStream_t st, Launch &&launch) {
    hipEvent_t e0, e1;
    HGV_HIP(hipEventCreate(&e0));
    HGV_HIP(hipEventCreate(&e1));
    launch();
    HGV_HIP(hipEventRecord(e0, st));
    launch();
    HGV_HIP(hipEventRecord(e1, st));
    HGV_HIP(hipEventSynchronize(e1));
    float ms = 0.0f;
    HGV_HIP(hipEventElapsedTime(&ms, e0, e1));
    HGV_HIP(hipEventDestroy(e0));
    HGV_HIP(hipEventDestroy(e1));
    return ms;
}

}  // namespace

void device_peaks(hgv_ctx_s *ctx, void *work, size_t work_bytes, double *tflops, double *gbs) {
    int cus = 0;
    HGV_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
    const int grid = 4 * std::max(cus, 1);   // 16 waves per CU
    const size_t out_bytes = (size_t)grid * 256 * sizeof(double);
    if (work_bytes < out_bytes + (2u << 20)) throw WorkspaceShort{out_bytes + (2u << 20)};
    double *out = static_cast<double *>(work);
    const int iters = 4096;
    const double ms_m = time_launch(ctx->stream, [&]() {
        hipLaunchKernelGGL(mfma_peak_kernel, dim3(grid), dim3(256), 0, ctx->stream, iters, out);
        HGV_LAUNCH_CHECK();
    });
    const double flops = (double)grid * 4 * iters * 8 * 2048.0;
    *tflops = flops / (ms_m * 1e-3) / 1e12;
    // the copy uses the rest of the buffer, 256-byte aligned halves
    const size_t off = (out_bytes + 255) / 256 * 256;
    const size_t half = (work_bytes - off) / 2 / 256 * 256;
    const size_t n = half / sizeof(double2);
    const double2 *src = reinterpret_cast<const double2 *>(static_cast<char *>(work) + off);
    double2 *dst = reinterpret_cast<double2 *>(static_cast<char *>(work) + off + half);
    const int cgrid = 8 * std::max(cus, 1) * 4;
    const double ms_c = time_launch(ctx->stream, [&]() {
        hipLaunchKernelGGL(copy_peak_kernel, dim3(cgrid), dim3(256), 0, ctx->stream, src, dst, n);
        HGV_LAUNCH_CHECK();
    });
    *gbs = 2.0 * (double)n * sizeof(double2) / (ms_c * 1e-3) / 1e9;
}

}  // namespace hgv
