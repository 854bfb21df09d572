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

// Shared tiles (G > 1) need a cooperative launch, which the library orders
// after every earlier cooperative launch on the device.  A thread that runs
// decompositions concurrently with others (the serving workers) turns them
// off for its own calls, so that its TSQR levels stay ordinary launches that
// overlap with the other streams' work.
bool &blk_shared_tiles();

// Workgroups per tile: up to 32 (one per 16-column chunk) while the tiles
// times that fit one launch of kBlkMaxWG resident workgroups; 1 otherwise.
inline int blk_group(int64_t ntiles, int64_t m) {
    const int64_t nch = (m + 15) / 16;
    int G = 1;
    if (!blk_shared_tiles()) return 1;
    while (2 * G <= 32 && 2 * G <= nch && ntiles * 2 * G <= kBlkMaxWG) G *= 2;
    return G;
}

inline int64_t blk_grid(int64_t ntiles, int64_t m) {
    const int G = blk_group(ntiles, m);
    return G > 1 ? ntiles * G : (ntiles < kBlkMaxWG ? ntiles : kBlkMaxWG);
}

// Workspace doubles of one level: the flags of the shared tiles (G > 1) and
// one tile region per tile group.
inline int64_t blk_ws_doubles(int64_t ntiles, int64_t m) {
    const int G = blk_group(ntiles, m);
    const int64_t flags = G > 1 ? (ntiles * ((m + 15) / 16) + 63) / 64 * 32 : 0;  // ints as doubles
    return flags + (blk_grid(ntiles, m) / G) * blk_region_doubles(m);
}

// One level: the m x m factor of every kBlkTR-row tile of W (rows x m,
// column-major, ld) into rows t*out_stride .. + m - 1 of out (ld_out); rows
// >= kvalid of each factor are written as zero.  tree: W is a stack of m x m
// upper-triangular factors (zero row blocks are skipped).  ws holds
// blk_ws_doubles(ntiles, m) doubles.
template <typename Tin>
int tsqr_blk_level(const Tin *W, int64_t rows, int64_t m, int64_t ld, bool tree, int64_t ntiles,
                   double *ws, double *out, int64_t ld_out, int64_t out_stride, int kvalid,
                   hipStream_t s);

}  // namespace ttsvd
