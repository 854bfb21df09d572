// Blocked Householder TSQR level for 128 < m <= 512 columns (tsqr_blk.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace ttsvd {

constexpr int kBlkTR = 1024;         // rows per tile
constexpr int kBlkMaxM = 512;        // widest unfolding handled
constexpr int64_t kBlkMaxWG = 256;   // workgroups per launch (one per CU)

// Workspace doubles of one workgroup: its tile (kBlkTR x ldq, ldq = m rounded
// up to 16).
__host__ __device__ inline int64_t blk_region_doubles(int64_t m) {
    return (int64_t)kBlkTR * ((m + 15) & ~int64_t(15));
}

inline int64_t blk_grid(int64_t ntiles) { return ntiles < kBlkMaxWG ? ntiles : kBlkMaxWG; }

// One level: the m x m factor of every kBlkTR-row tile of W (rows x m,
// column-major, ld) into rows t*out_stride .. + m - 1 of out (ld_out); rows
// >= kvalid of each factor are written as zero.  tree: W is a stack of m x m
// upper-triangular factors (zero row blocks are skipped).  ws holds
// blk_grid(ntiles) * blk_region_doubles(m) doubles.
template <typename Tin>
int tsqr_blk_level(const Tin *W, int64_t rows, int64_t m, int64_t ld, bool tree, int64_t ntiles,
                   double *ws, double *out, int64_t ld_out, int64_t out_stride, int kvalid,
                   hipStream_t s);

}  // namespace ttsvd
