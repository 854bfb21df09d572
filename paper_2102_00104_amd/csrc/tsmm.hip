// Fused tall-skinny matrix product and reshape (Sec. 4.1.2 of arXiv
// 2102.00104, "TSMM"): kernel and launcher; the device body and the data
// layout are described in tsmm_dev.h.
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>

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

// ----------------------------------------------------------------------------
// FP64 MFMA form for m <= 64 columns and 16 < k <= 32 output columns, where the
// VALU kernel is limited by its FMA issue rate (I_c = 2 m k / 8 (m + k) is up
// to ~5 flop/B).  It computes Y^T = V^T W^T with v_mfma_f64_16x16x4f64, block
// by block of 16 rows: A = V^T (16 output columns x 4 inner), B = W^T (4 inner
// x 16 rows), so lane l loads W(r0 + l%16, c + l/16) (16 consecutive rows of
// 4 columns) and holds the results Y(r0 + l%16, a0 + l/16 + 4 v), v < 4
// (stores of 16 consecutive rows per column).  All of V sits in registers;
// W is read once.  Each wave takes 32-row blocks in a grid-stride loop.
// ----------------------------------------------------------------------------
typedef double tsmm_double4 __attribute__((ext_vector_type(4)));
constexpr int kMfmaMaxM = 64;
constexpr int kMfmaRowsPerWave = 32;

template <int NT>  // 16-column output tiles (k <= 16 NT)
__global__ __launch_bounds__(256) void tsmm_mfma_kernel(
    const double *__restrict__ W, int64_t rows, int m, int64_t ld,
    const double *__restrict__ V, int64_t svc, int64_t sva, int k,
    int64_t rows_next, int64_t n_next, double *__restrict__ Y, int64_t ld_y) {
    constexpr int KS = kMfmaMaxM / 4;  // inner steps of 4 columns of W
    const int lane = lane_id();
    const int lr = lane % 16, lc = lane / 16;
    // V^T operands: A(i, kk) = V(c + kk, a0 + i), lane (i, kk) = (l % 16, l / 16)
    double va[KS][NT];
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int c = 4 * s + lc, a = 16 * t + lr;
            va[s][t] = (c < m && a < k) ? V[(int64_t)c * svc + (int64_t)a * sva] : 0.0;
        }
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / kWave);
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x / kWave) + thread_id() / kWave;
    for (int64_t r0 = wave * kMfmaRowsPerWave; r0 < rows; r0 += nwaves * kMfmaRowsPerWave) {
        double w[2][KS];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int64_t row = r0 + 16 * b + lr;
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                const int c = 4 * s + lc;
                w[b][s] = (row < rows && c < m) ? W[row + ld * c] : 0.0;
            }
        }
        tsmm_double4 acc[2][NT];
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[b][t] = tsmm_double4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            if (4 * s < m) {  // uniform
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int t = 0; t < NT; ++t)
                        acc[b][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(va[s][t], w[b][s], acc[b][t], 0, 0, 0);
            }
        }
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int64_t row = r0 + 16 * b + lr;
            if (row < rows) {
                const int64_t q = row / rows_next;
                const int64_t r = row - q * rows_next;
#pragma unroll
                for (int t = 0; t < NT; ++t)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int a = 16 * t + lc + 4 * v;
                        if (a < k) Y[r + ld_y * (q + n_next * a)] = acc[b][t][v];
                    }
            }
        }
    }
}

// TTSVD_TSMM_MFMA=0 selects the VALU kernel instead (a tuning override).
bool tsmm_mfma_enabled() {
    static bool v = [] {
        const char *e = getenv("TTSVD_TSMM_MFMA");
        return !(e && atoi(e) == 0);
    }();
    return v;
}

// TTSVD_TSMM_X2=0 turns the two-rows-per-lane kernels off (a tuning
// override; both kernels give identical results).
bool tsmm_x2_enabled() {
    static bool v = [] {
        const char *e = getenv("TTSVD_TSMM_X2");
        return !(e && atoi(e) == 0);
    }();
    return v;
}

int tsmm_mfma_launch(const double *W, int64_t rows, int64_t m, int64_t ld, const double *V,
                     int64_t svc, int64_t sva, int64_t k, int64_t n_next, double *Y,
                     int64_t ld_y, hipStream_t s) {
    const int64_t rows_next = rows / n_next;
    const int64_t blocks = std::min<int64_t>(ceil_div(rows, 4 * kMfmaRowsPerWave), 4096);
    char name[64];
    snprintf(name, sizeof(name), "tsmm_mfma_kernel<%d>", k <= 16 ? 1 : 2);
    prof_begin(s, name, (double)rows * m * 8.0 + (double)rows * k * 8.0, 2.0 * (double)rows * m * k);
    if (k <= 16)
        hipLaunchKernelGGL((tsmm_mfma_kernel<1>), dim3((unsigned)blocks), dim3(256), 0, s, W, rows,
                           (int)m, ld, V, svc, sva, (int)k, rows_next, n_next, Y, ld_y);
    else
        hipLaunchKernelGGL((tsmm_mfma_kernel<2>), dim3((unsigned)blocks), dim3(256), 0, s, W, rows,
                           (int)m, ld, V, svc, sva, (int)k, rows_next, n_next, Y, ld_y);
    prof_end(s);
    TTSVD_HIP_TRY(hipGetLastError());
    return TTSVD_OK;
}

// Two adjacent rows of one column as one memory word: bf16 pairs in 32 bits,
// FP32 pairs in 64 bits (the lower address in the low half).
template <typename E> struct RowPair;
template <> struct RowPair<bf16> {
    using word = uint32_t;
    __device__ static inline void split(word u, float &lo, float &hi) {
        lo = __uint_as_float(u << 16);
        hi = __uint_as_float(u & 0xffff0000u);
    }
    __device__ static inline word join(float lo, float hi) {
        return Elem<bf16>::bits(lo) | (Elem<bf16>::bits(hi) << 16);
    }
};
template <> struct RowPair<float> {
    using word = uint64_t;
    __device__ static inline void split(word u, float &lo, float &hi) {
        lo = __uint_as_float((uint32_t)u);
        hi = __uint_as_float((uint32_t)(u >> 32));
    }
    __device__ static inline word join(float lo, float hi) {
        return (word)__float_as_uint(lo) | ((word)__float_as_uint(hi) << 32);
    }
};

// E -> E product (E = bf16 or FP32) with two adjacent rows per lane: every W
// load and every Y store moves one RowPair word instead of two single
// elements.  Used when rows, ld, rows/n_next and ld_y are even and W and Y
// are aligned to the word, so a pair never straddles a column or a block of
// the reshape; the arithmetic (FP32 products, FP32 sums over the columns in
// order, one rounding to the storage type) is that of tsmm_kernel.
template <int KB, int PPT, typename E>
__global__ __launch_bounds__(kTsmmThreads) void tsmm_x2_kernel(
    const E *__restrict__ W, int64_t rows, int m, int64_t ld, const double *__restrict__ V,
    int64_t svc, int64_t sva, int k, int64_t rows_next, int64_t n_next, E *__restrict__ Y,
    int64_t ld_y) {
    using P = RowPair<E>;
    __shared__ float vs[kTsmmChunk][KB];
    const int tid = threadIdx.x;
    const int a0 = blockIdx.y * KB;
    const int64_t base = (int64_t)blockIdx.x * kTsmmThreads * PPT * 2 + 2 * tid;
    const typename P::word *__restrict__ W2 = reinterpret_cast<const typename P::word *>(W);
    typename P::word *__restrict__ Y2 = reinterpret_cast<typename P::word *>(Y);
    int64_t row[PPT];
    bool ok[PPT];
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        row[p] = base + (int64_t)2 * kTsmmThreads * p;  // even; row + 1 < rows when ok
        ok[p] = row[p] < rows;
    }
    float acc[PPT][2][KB];
#pragma unroll
    for (int p = 0; p < PPT; ++p)
#pragma unroll
        for (int a = 0; a < KB; ++a) acc[p][0][a] = acc[p][1][a] = 0.0f;

    for (int c0 = 0; c0 < m; c0 += kTsmmChunk) {
        __syncthreads();
        for (int idx = tid; idx < kTsmmChunk * KB; idx += kTsmmThreads) {
            const int cc = idx / KB, a = idx % KB;
            const int c = c0 + cc, ga = a0 + a;
            vs[cc][a] = (c < m && ga < k) ? (float)V[(int64_t)c * svc + (int64_t)ga * sva] : 0.0f;
        }
        __syncthreads();
        const int nc = min(kTsmmChunk, m - c0);
#pragma unroll 4
        for (int cc = 0; cc < nc; ++cc) {
            float lo[PPT], hi[PPT];
#pragma unroll
            for (int p = 0; p < PPT; ++p) {
                const typename P::word u = ok[p] ? W2[(row[p] + ld * (c0 + cc)) >> 1]
                                                 : (typename P::word)0;
                P::split(u, lo[p], hi[p]);
            }
#pragma unroll
            for (int a = 0; a < KB; ++a) {
                const float vv = vs[cc][a];
#pragma unroll
                for (int p = 0; p < PPT; ++p) {
                    acc[p][0][a] = fmaf(lo[p], vv, acc[p][0][a]);
                    acc[p][1][a] = fmaf(hi[p], vv, acc[p][1][a]);
                }
            }
        }
    }
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        if (!ok[p]) continue;
        const int64_t q = row[p] / rows_next;
        const int64_t r = row[p] - q * rows_next;  // even, r + 1 < rows_next
#pragma unroll
        for (int a = 0; a < KB; ++a) {
            const int ga = a0 + a;
            if (ga < k) Y2[(r + ld_y * (q + n_next * ga)) >> 1] = P::join(acc[p][0][a], acc[p][1][a]);
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

// E -> E with two rows per lane where the shapes allow it.
template <typename E>
static int tsmm_x2_dispatch(const E *W, int64_t rows, int64_t m, int64_t ld, const double *V,
                            int64_t svc, int64_t sva, int64_t k, int64_t n_next, E *Y,
                            int64_t ld_y, hipStream_t s) {
    const int64_t rows_next = rows / n_next;
    const int KB = (int)cpow2((int)std::min<int64_t>(k, 64));
    const int ky = (int)ceil_div(k, KB);
#define TTSVD_TSMM2_CASE(KK, PP)                                                              \
    case KK: {                                                                                \
        dim3 grid((unsigned)ceil_div(rows, (int64_t)kTsmmThreads * 2 * PP), (unsigned)ky);    \
        char name[64];                                                                        \
        snprintf(name, sizeof(name), "tsmm_x2_kernel<%d, %d, %s>", KK, PP, ElemName<E>::get()); \
        prof_begin(s, name, (double)rows * m * sizeof(E) + (double)rows * k * sizeof(E),      \
                   2.0 * (double)rows * m * k);                                               \
        hipLaunchKernelGGL((tsmm_x2_kernel<KK, PP, E>), grid, dim3(kTsmmThreads), 0, s, W,    \
                           rows, (int)m, ld, V, svc, sva, (int)k, rows_next, n_next, Y, ld_y); \
        prof_end(s);                                                                          \
        break;                                                                                \
    }
    switch (KB) {
        TTSVD_TSMM2_CASE(1, 4)
        TTSVD_TSMM2_CASE(2, 4)
        TTSVD_TSMM2_CASE(4, 4)
        TTSVD_TSMM2_CASE(8, 2)
        TTSVD_TSMM2_CASE(16, 2)
        TTSVD_TSMM2_CASE(32, 1)
        TTSVD_TSMM2_CASE(64, 1)
        default:
            return set_error(TTSVD_EUNSUPPORTED, "tsmm: k bucket %d", KB);
    }
#undef TTSVD_TSMM2_CASE
    TTSVD_HIP_TRY(hipGetLastError());
    return TTSVD_OK;
}

// Shapes and alignment that let tsmm_x2_kernel run (word = 2 elements).
template <typename E>
static bool x2_fits(const void *W, int64_t rows, int64_t ld, int64_t n_next, const void *Y,
                    int64_t ld_y) {
    const uintptr_t wmask = 2 * sizeof(E) - 1;
    return rows % 2 == 0 && ld % 2 == 0 && (rows / n_next) % 2 == 0 && ld_y % 2 == 0 &&
           ((uintptr_t)W & wmask) == 0 && ((uintptr_t)Y & wmask) == 0 && tsmm_x2_enabled();
}

int tsmm_launch(const void *W, int dtype, int64_t rows, int64_t m, int64_t ld, const double *V,
                int64_t svc, int64_t sva, int64_t k, int64_t n_next, void *Y, int ydtype,
                int64_t ld_y, hipStream_t s) {
    if (ydtype == TTSVD_F64) {
        switch (dtype) {
            case TTSVD_F64:
                if (m <= kMfmaMaxM && k > 16 && k <= 32 && tsmm_mfma_enabled())
                    return tsmm_mfma_launch((const double *)W, rows, m, ld, V, svc, sva, k, n_next,
                                            (double *)Y, ld_y, s);
                return tsmm_dispatch((const double *)W, rows, m, ld, V, svc, sva, k, n_next, (double *)Y, ld_y, s);
            case TTSVD_F32:
                return tsmm_dispatch((const float *)W, rows, m, ld, V, svc, sva, k, n_next, (double *)Y, ld_y, s);
            case TTSVD_BF16:
                return tsmm_dispatch((const bf16 *)W, rows, m, ld, V, svc, sva, k, n_next, (double *)Y, ld_y, s);
        }
    } else if (ydtype == dtype) {
        switch (dtype) {
            case TTSVD_F32:
                // (FP32 pairs in 64-bit words were measured slower than one
                // 32-bit element per lane: the pair kernel is bf16-only)
                return tsmm_dispatch((const float *)W, rows, m, ld, V, svc, sva, k, n_next, (float *)Y, ld_y, s);
            case TTSVD_BF16:
                if (x2_fits<bf16>(W, rows, ld, n_next, Y, ld_y))
                    return tsmm_x2_dispatch((const bf16 *)W, rows, m, ld, V, svc, sva, k, n_next,
                                            (bf16 *)Y, ld_y, s);
                return tsmm_dispatch((const bf16 *)W, rows, m, ld, V, svc, sva, k, n_next, (bf16 *)Y, ld_y, s);
        }
    }
    return set_error(TTSVD_EUNSUPPORTED, "tsmm: dtype %d -> %d", dtype, ydtype);
}

}  // namespace ttsvd
