// Machine micro-benchmarks (ttsvd_machine_bench): the measured counterparts
// of the hardware limits the roofline report uses -- HBM bandwidth for a pure
// load, a pure store, a copy and a triad stream, and the FP64 FMA rate -- in
// the spirit of the machine characterisation of Sec. 5 (Table 1).  Not part
// of the method.
#include "common.h"

namespace ttsvd {
namespace {

constexpr int kMbThreads = 256;
constexpr int kMbBlocksPerCu = 8;

// Grid-stride loops over 16-byte vectors; every kernel is a plain stream.
__global__ __launch_bounds__(kMbThreads) void mb_load(const double2 *__restrict__ a, int64_t n,
                                                      double *__restrict__ sink) {
    double s0 = 0.0, s1 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kMbThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kMbThreads) {
        const double2 v = a[i];
        s0 += v.x;
        s1 += v.y;
    }
    // never true for finite inputs of the caller's buffer (zeros): keeps the loads
    if (s0 + s1 == -1.0) sink[0] = s0;
}

__global__ __launch_bounds__(kMbThreads) void mb_store(double2 *__restrict__ a, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kMbThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kMbThreads)
        a[i] = make_double2(0.0, 0.0);
}

__global__ __launch_bounds__(kMbThreads) void mb_copy(const double2 *__restrict__ a,
                                                      double2 *__restrict__ b, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kMbThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kMbThreads)
        b[i] = a[i];
}

__global__ __launch_bounds__(kMbThreads) void mb_triad(double2 *__restrict__ a,
                                                       const double2 *__restrict__ b,
                                                       const double2 *__restrict__ c, double s,
                                                       int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kMbThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kMbThreads) {
        const double2 x = b[i], y = c[i];
        a[i] = make_double2(fma(s, y.x, x.x), fma(s, y.y, x.y));
    }
}

// FP64 FMA rate: 16 independent chains per thread, kFmaIters iterations.
constexpr int kFmaChains = 16;
constexpr int kFmaIters = 4096;

__global__ __launch_bounds__(kMbThreads) void mb_fma(double *__restrict__ sink, double x0) {
    double acc[kFmaChains];
#pragma unroll
    for (int c = 0; c < kFmaChains; ++c) acc[c] = x0 + c * 1e-3 + threadIdx.x * 1e-9;
    const double a = 0.999999, b = 1e-7;
    for (int it = 0; it < kFmaIters; ++it) {
#pragma unroll
        for (int c = 0; c < kFmaChains; ++c) acc[c] = fma(acc[c], a, b);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < kFmaChains; ++c) s += acc[c];
    if (s == -1.0) sink[0] = s;
}

}  // namespace
}  // namespace ttsvd

using namespace ttsvd;

extern "C" {

int ttsvd_machine_bench(int kind, void *buf, size_t bytes, int reps, hipStream_t stream,
                        double *out) {
    clear_error();
    if (!buf || !out || reps < 1) return set_error(TTSVD_EINVAL, "machine_bench: arguments");
    if (kind < TTSVD_MB_LOAD || kind > TTSVD_MB_FMA)
        return set_error(TTSVD_EINVAL, "machine_bench: kind %d", kind);
    const int narr = kind == TTSVD_MB_COPY ? 2 : kind == TTSVD_MB_TRIAD ? 3 : 1;
    const int64_t nvec = (kind == TTSVD_MB_FMA) ? 0 : (int64_t)(bytes / 16 / narr);
    if (kind != TTSVD_MB_FMA && nvec < 1)
        return set_error(TTSVD_EINVAL, "machine_bench: %zu bytes", bytes);
    int dev = 0, ncu = 0;
    TTSVD_HIP_TRY(hipGetDevice(&dev));
    TTSVD_HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    const dim3 grid((unsigned)(ncu * kMbBlocksPerCu)), block(kMbThreads);
    double2 *v = (double2 *)buf;
    auto launch = [&]() {
        switch (kind) {
            case TTSVD_MB_LOAD:
                hipLaunchKernelGGL(mb_load, grid, block, 0, stream, v, nvec, (double *)buf);
                break;
            case TTSVD_MB_STORE:
                hipLaunchKernelGGL(mb_store, grid, block, 0, stream, v, nvec);
                break;
            case TTSVD_MB_COPY:
                hipLaunchKernelGGL(mb_copy, grid, block, 0, stream, v, v + nvec, nvec);
                break;
            case TTSVD_MB_TRIAD:
                hipLaunchKernelGGL(mb_triad, grid, block, 0, stream, v, v + nvec, v + 2 * nvec, 0.5,
                                   nvec);
                break;
            default:
                hipLaunchKernelGGL(mb_fma, grid, block, 0, stream, (double *)buf, 1.0);
                break;
        }
    };
    hipEvent_t e0, e1;
    TTSVD_HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return set_error(TTSVD_EHIP, "machine_bench: event");
    }
    launch();  // warm-up
    int rc = TTSVD_OK;
    float ms = 0.f;
    if (hipEventRecord(e0, stream) != hipSuccess) rc = TTSVD_EHIP;
    for (int r = 0; r < reps && rc == TTSVD_OK; ++r) launch();
    if (rc == TTSVD_OK && (hipGetLastError() != hipSuccess || hipEventRecord(e1, stream) != hipSuccess ||
                           hipEventSynchronize(e1) != hipSuccess ||
                           hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        rc = TTSVD_EHIP;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != TTSVD_OK) return set_error(rc, "machine_bench: launch or timing failed");
    out[0] = (double)ms / reps;
    if (kind == TTSVD_MB_FMA)
        out[1] = 2.0 * kFmaChains * (double)kFmaIters * grid.x * (double)kMbThreads;
    else
        out[1] = (double)nvec * 16.0 * (kind == TTSVD_MB_COPY ? 2 : kind == TTSVD_MB_TRIAD ? 3 : 1);
    return TTSVD_OK;
}

}  // extern "C"
