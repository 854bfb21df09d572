// Fused tall-skinny matrix product and reshape (Sec. 4.1.2 of arXiv
// 2102.00104, "TSMM"): kernel and launcher; the device body and the data
// layout are described in tsmm_dev.h.
#include <stdio.h>

#include "common.h"
#include "kernels.h"
#include "profile.h"
#include "tsmm_dev.h"

namespace ttsvd {

// Single-tensor kernel: one workgroup per (blockIdx.x, blockIdx.y).
template <int KB, int RPT, typename Tin, typename Tout>
__global__ __launch_bounds__(kTsmmThreads) void tsmm_kernel(
    const Tin *__restrict__ W, int64_t rows, int m, int64_t ld,
    const double *__restrict__ V, int64_t svc, int64_t sva, int k,
    int64_t rows_next, int64_t n_next, Tout *__restrict__ Y, int64_t ld_y) {
    __shared__ __attribute__((aligned(16))) char smem[tsmm_smem<KB, RPT, Tin>()];
    tsmm_body<KB, RPT, Tin, Tout>(W, rows, m, ld, V, svc, sva, k, rows_next, n_next, Y, ld_y,
                                  blockIdx.x, blockIdx.y, smem);
}

template <typename T> struct ElemName;
template <> struct ElemName<double> { static const char *get() { return "double"; } };
template <> struct ElemName<float> { static const char *get() { return "float"; } };
template <> struct ElemName<bf16> { static const char *get() { return "ttsvd::bf16"; } };

template <typename Tin, typename Tout>
static int tsmm_dispatch(const Tin *W, int64_t rows, int64_t m, int64_t ld, const double *V,
                         int64_t svc, int64_t sva, int64_t k, int64_t n_next, Tout *Y,
                         int64_t ld_y, hipStream_t s) {
    const int64_t rows_next = rows / n_next;
    int KB = (int)cpow2((int)std::min<int64_t>(k, 64));
    const int ky = (int)ceil_div(k, KB);
#define TTSVD_TSMM_CASE(KK, RR)                                                            \
    case KK: {                                                                             \
        dim3 grid((unsigned)ceil_div(rows, (int64_t)kTsmmThreads * RR), (unsigned)ky);     \
        char name[96];                                                                     \
        snprintf(name, sizeof(name), "tsmm_kernel<%d, %d, %s, %s>", KK, RR,               \
                 ElemName<Tin>::get(), ElemName<Tout>::get());                            \
        prof_begin(s, name, (double)rows * m * sizeof(Tin) + (double)rows * k * sizeof(Tout), \
                   2.0 * (double)rows * m * k);                                            \
        hipLaunchKernelGGL((tsmm_kernel<KK, RR, Tin, Tout>), grid, dim3(kTsmmThreads), 0,  \
                           s, W, rows, (int)m, ld, V, svc, sva, (int)k, rows_next, n_next, \
                           Y, ld_y);                                                       \
        prof_end(s);                                                                       \
        break;                                                                             \
    }
    switch (KB) {
        TTSVD_TSMM_CASE(1, 8)
        TTSVD_TSMM_CASE(2, 8)
        TTSVD_TSMM_CASE(4, 8)
        TTSVD_TSMM_CASE(8, 4)
        TTSVD_TSMM_CASE(16, 4)
        TTSVD_TSMM_CASE(32, 2)
        TTSVD_TSMM_CASE(64, 1)
        default:
            return set_error(TTSVD_EUNSUPPORTED, "tsmm: k bucket %d", KB);
    }
#undef TTSVD_TSMM_CASE
    TTSVD_HIP_TRY(hipGetLastError());
    return TTSVD_OK;
}

int tsmm_launch(const void *W, int dtype, int64_t rows, int64_t m, int64_t ld, const double *V,
                int64_t svc, int64_t sva, int64_t k, int64_t n_next, void *Y, int ydtype,
                int64_t ld_y, hipStream_t s) {
    if (ydtype == TTSVD_F64) {
        switch (dtype) {
            case TTSVD_F64:
                return tsmm_dispatch((const double *)W, rows, m, ld, V, svc, sva, k, n_next, (double *)Y, ld_y, s);
            case TTSVD_F32:
                return tsmm_dispatch((const float *)W, rows, m, ld, V, svc, sva, k, n_next, (double *)Y, ld_y, s);
            case TTSVD_BF16:
                return tsmm_dispatch((const bf16 *)W, rows, m, ld, V, svc, sva, k, n_next, (double *)Y, ld_y, s);
        }
    } else if (ydtype == dtype) {
        switch (dtype) {
            case TTSVD_F32:
                return tsmm_dispatch((const float *)W, rows, m, ld, V, svc, sva, k, n_next, (float *)Y, ld_y, s);
            case TTSVD_BF16:
                return tsmm_dispatch((const bf16 *)W, rows, m, ld, V, svc, sva, k, n_next, (bf16 *)Y, ld_y, s);
        }
    }
    return set_error(TTSVD_EUNSUPPORTED, "tsmm: dtype %d -> %d", dtype, ydtype);
}

}  // namespace ttsvd
