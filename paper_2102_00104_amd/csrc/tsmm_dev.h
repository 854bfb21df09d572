// Device body of the fused tall-skinny matrix product and reshape (Sec. 4.1.2
// of arXiv 2102.00104, "TSMM"):  Y <- reshape(W V, (rows/n_next, n_next k)),
// the step W^(i-1) <- reshape(W^(i) V_{:,1:r}, ...) of Algorithm 2, shared by
// the single-tensor kernel and the batched persistent kernel.
//
// W (rows x m, column-major) is streamed once from HBM with coalesced loads:
// thread t of a block owns rows base + t + 256 i (i < RPT), so every wave load
// instruction reads 64 consecutive rows of one column.  The m x k block of V
// is staged through LDS in chunks of columns and read as wave-uniform
// (broadcast) values.  Each block computes up to KB output columns; larger k
// uses several blocks (W is then read once per KB columns).  The reshape is
// pure index arithmetic on the store: element (i, a) of W V goes to
// Y[(i mod rows') + ld_y (i div rows' + n_next a)], rows' = rows/n_next.
#pragma once

#include "common.h"

namespace ttsvd {

constexpr int kTsmmThreads = 256;
constexpr int kTsmmChunk = 32;  // columns of V staged per LDS round

template <int KB, int RPT, typename Tin>
constexpr size_t tsmm_smem() {
    return sizeof(typename Elem<Tin>::acc) * kTsmmChunk * KB;
}

// Block (bx, by): rows bx * NTH RPT ... of W, output columns by * KB ...
// NTH = threads of the workgroup.
template <int KB, int RPT, typename Tin, typename Tout, int NTH = kTsmmThreads>
__device__ __forceinline__ void tsmm_body(
    const Tin *__restrict__ W, int64_t rows, int m, int64_t ld,
    const double *__restrict__ V, int64_t svc, int64_t sva, int k,
    int64_t rows_next, int64_t n_next, Tout *__restrict__ Y, int64_t ld_y,
    int64_t bx, int by, void *smem) {
    using T = typename Elem<Tin>::acc;
    T(*vs)[KB] = reinterpret_cast<T(*)[KB]>(smem);
    const int tid = thread_id();
    const int a0 = by * KB;
    const int64_t base = bx * NTH * RPT + tid;

    int64_t row[RPT];
    bool ok[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        row[i] = base + (int64_t)NTH * i;
        ok[i] = row[i] < rows;
    }
    T acc[RPT][KB];
#pragma unroll
    for (int i = 0; i < RPT; ++i)
#pragma unroll
        for (int a = 0; a < KB; ++a) acc[i][a] = T(0);

    for (int c0 = 0; c0 < m; c0 += kTsmmChunk) {
        __syncthreads();
        for (int idx = tid; idx < kTsmmChunk * KB; idx += NTH) {
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

// Rows per thread for a KB-column block.
__host__ __device__ constexpr int tsmm_rpt(int KB) {
    return KB <= 4 ? 8 : KB <= 16 ? 4 : KB <= 32 ? 2 : 1;
}

}  // namespace ttsvd
