// Fused tall-skinny matrix product and reshape (Sec. 4.1.2 of arXiv
// 2102.00104, "TSMM"):  Y <- reshape(W V, (rows/n_next, n_next k)), the
// step W^(i-1) <- reshape(W^(i) V_{:,1:r}, ...) of Algorithm 2.
//
// W (rows x m, column-major) is streamed once from HBM with coalesced loads:
// thread t of a block owns rows base + t + 256 i (i < RPT), so every wave load
// instruction reads 64 consecutive rows of one column.  The m x k block of V
// is staged through LDS in chunks of columns and read as wave-uniform
// (broadcast) values.  Each block computes up to KB output columns; larger k
// uses several blocks in grid.y (W is then read once per KB columns).
// The reshape is pure index arithmetic on the store: element (i, a) of W V
// goes to Y[(i mod rows') + ld_y (i div rows' + n_next a)], rows' = rows/n_next.
#include <stdio.h>

#include "common.h"
#include "kernels.h"
#include "profile.h"

namespace ttsvd {

constexpr int kTsmmThreads = 256;
constexpr int kTsmmChunk = 32;  // columns of V staged per LDS round

template <int KB, int RPT, typename Tin, typename Tout>
__global__ __launch_bounds__(kTsmmThreads) void tsmm_kernel(
    const Tin *__restrict__ W, int64_t rows, int m, int64_t ld,
    const double *__restrict__ V, int64_t svc, int64_t sva, int k,
    int64_t rows_next, int64_t n_next, Tout *__restrict__ Y, int64_t ld_y) {
    using T = typename Elem<Tin>::acc;
    __shared__ T vs[kTsmmChunk][KB];
    const int tid = threadIdx.x;
    const int a0 = blockIdx.y * KB;
    const int64_t base = (int64_t)blockIdx.x * kTsmmThreads * RPT + tid;

    int64_t row[RPT];
    bool ok[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        row[i] = base + (int64_t)kTsmmThreads * i;
        ok[i] = row[i] < rows;
    }
    T acc[RPT][KB];
#pragma unroll
    for (int i = 0; i < RPT; ++i)
#pragma unroll
        for (int a = 0; a < KB; ++a) acc[i][a] = T(0);

    for (int c0 = 0; c0 < m; c0 += kTsmmChunk) {
        __syncthreads();
        for (int idx = tid; idx < kTsmmChunk * KB; idx += kTsmmThreads) {
            const int cc = idx / KB, a = idx % KB;
            const int c = c0 + cc, ga = a0 + a;
            vs[cc][a] = (c < m && ga < k) ? (T)V[(int64_t)c * svc + (int64_t)ga * sva] : T(0);
        }
        __syncthreads();
        const int nc = min(kTsmmChunk, m - c0);
        int cc = 0;
        for (; cc + 4 <= nc; cc += 4) {
            T w[4][RPT];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int i = 0; i < RPT; ++i)
                    w[u][i] = ok[i] ? Elem<Tin>::load(W + row[i] + ld * (c0 + cc + u)) : T(0);
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int a = 0; a < KB; ++a) {
                    const T vv = vs[cc + u][a];
#pragma unroll
                    for (int i = 0; i < RPT; ++i) acc[i][a] = fma(w[u][i], vv, acc[i][a]);
                }
        }
        for (; cc < nc; ++cc) {
            T w[RPT];
#pragma unroll
            for (int i = 0; i < RPT; ++i)
                w[i] = ok[i] ? Elem<Tin>::load(W + row[i] + ld * (c0 + cc)) : T(0);
#pragma unroll
            for (int a = 0; a < KB; ++a) {
                const T vv = vs[cc][a];
#pragma unroll
                for (int i = 0; i < RPT; ++i) acc[i][a] = fma(w[i], vv, acc[i][a]);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        if (!ok[i]) continue;
        const int64_t q = row[i] / rows_next;
        const int64_t r = row[i] - q * rows_next;
#pragma unroll
        for (int a = 0; a < KB; ++a) {
            const int ga = a0 + a;
            if (ga < k) Elem<Tout>::store(Y + r + ld_y * (q + n_next * ga), (typename Elem<Tout>::acc)acc[i][a]);
        }
    }
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
