// Blocked Householder TSQR for 128 < m <= 512 columns (the Q-less TSQR of
// Sec. 3.2 of arXiv 2102.00104 with the Householder step of Algorithm 6),
// with the trailing updates on FP64 MFMA.
//
// A workgroup reduces one row tile of kBlkTR = 1024 rows at a time.  The tile
// is copied (widened to FP64, zero padded) into a workspace region of the
// workgroup, in a "row-quad" layout: element (r, c) at ((r/4) ldq + c) 4 +
// r mod 4, ldq = m rounded up to 16, so that every MFMA operand load below
// reads whole 128-byte lines.  Tiles are independent: each yields the m x m
// factor of its rows, the factors are stacked and the next level reduces
// them the same way until one tile remains.  At those tree levels a row block
// of a stacked triangle whose index in its triangle exceeds the current panel
// (and that is no pivot row) is still zero in the panel's columns; it is
// skipped (its reflector entries are zero, so skipping changes nothing).
//
// Per 16-column panel p:
//  * unblocked panel factorization: 16 Householder steps (Algorithm 6) on
//    rows >= p of the panel; lane l of wave w holds rows 128 w + l + 64 i
//    (i < 2) of the 16 panel columns, norms and dot products are reduced
//    across the wave and then across the 8 waves through LDS;
//  * compact WY form: H_p ... H_{p+15} = I - Y T Y^T with T upper triangular
//    and unit diagonal (every reflector has ||v||^2 = 2), T built column by
//    column from dot products of the same reductions;
//  * trailing update C <- C - Y T^T Y^T C for the columns right of the panel,
//    16 at a time, with v_mfma_f64_16x16x4f64: W = Y^T C per wave over its
//    rows, summed across the waves through LDS, W' = T^T W, then C -= Y W'
//    block by block of 16 rows.  Each wave updates only its own rows, so the
//    tile needs no barrier beyond the one per 16 columns for W.
#include <float.h>
#include <stdio.h>

#include <algorithm>

#include "common.h"
#include "driver.h"
#include "tsqr_blk.h"

namespace ttsvd {

constexpr int kBlkWaves = 8;
constexpr int kBlkThreads = kBlkWaves * kWave;
constexpr int kBlkRW = kBlkTR / kBlkWaves;  // rows per wave
constexpr int kBlkRPT = kBlkRW / kWave;     // rows per lane in the panel
constexpr int kBlkKS = kBlkRW / 4;          // 4-row MFMA K-steps per wave
constexpr int kBlkRB = kBlkRW / 16;         // 16-row MFMA row blocks per wave
static_assert(kBlkRW % 16 == 0 && kBlkRPT >= 1, "tile shape");

typedef double blk_d4 __attribute__((ext_vector_type(4)));

struct BlkShared {
    double y[kBlkTR * 16];              // reflectors of the panel, see yl()
    double wpart[kBlkWaves][4][kWave];  // per-wave partial W, D layout
    double red[2][kBlkWaves];           // per-wave partial column norms
    double part[2][kBlkWaves][16];      // per-wave partial dot products
    double u1[2];                       // pivot entry of the current column
    double nx[2][4];                    // next column's pivot rows before the update
    double G[16][17];                   // G(k, j) = y_k . y_j, k < j
    double tl[16][17];                  // T, row-major (padded)
};

// Offset of element (r, c) in a tile region (below 2^31: kBlkTR x 512 doubles).
__device__ __forceinline__ int q4i(int r, int c, int ldq) {
    return ((r >> 2) * ldq + c) * 4 + (r & 3);
}

// Position of Y(r, k) in LDS: row-major, 16 per row, k XOR-swizzled by
// 2 ((r / 2) mod 8).  Both MFMA operand reads are then free of bank
// conflicts: 4 rows x 16 reflectors (W = Y^T C) and 16 rows x 4 reflectors
// (C -= Y W').
__device__ __forceinline__ int yl(int r, int k) { return r * 16 + (k ^ (((r >> 1) & 7) << 1)); }

// Wait until another workgroup has released flag (its writes before the
// release become visible to every thread of this workgroup).  The wait is
// bounded (20 s of the 100 MHz wall clock): the group is resident together by
// construction, so the bound only guarantees that the launch always ends.
constexpr uint64_t kBlkWaitTicks = 20ull * 100000000ull;
__device__ __forceinline__ void blk_wait(int *flag) {
    if (threadIdx.x == 0) {
        const uint64_t t0 = wall_clock64();
        while (__hip_atomic_load(flag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == 0) {
            if (wall_clock64() - t0 > kBlkWaitTicks) break;
            __builtin_amdgcn_s_sleep(1);
        }
        // one agent-scope acquire for the workgroup (the caches it
        // invalidates are shared by all its waves)
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

// Publish this workgroup's global writes so far and set flag: the barrier
// orders every wave's stores before thread 0's agent-scope release, which
// writes back the cache they sit in.
__device__ __forceinline__ void blk_release(int *flag) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_store(flag, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// G workgroups share a tile (G > 1: one tile per group, launched
// cooperatively so that the group is resident together): column chunk ci (16
// columns) belongs to workgroup ci mod G, which copies it in, applies every
// panel's update to it and writes its part of the factor.  All G factor each
// panel redundantly (same arithmetic, same Y and T); the owner of chunk p+1
// updates it first and releases flags[t * nch + p + 1], which the others wait
// for before they load panel p+1.
template <typename Tin>
__global__ __launch_bounds__(kBlkThreads) void tsqr_blk_kernel(
    const Tin *__restrict__ W, int64_t rows, int m, int64_t ld, int tri, int64_t ntiles,
    int G, int *__restrict__ flags, double *__restrict__ ws, double *__restrict__ out,
    int64_t ld_out, int64_t out_row0_stride, int kvalid) {
    __shared__ BlkShared sh;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int w = __builtin_amdgcn_readfirstlane(tid / kWave);  // wave-uniform (scalar)
    const int lr = lane & 15, lg = lane >> 4;
    const int ldq = (m + 15) & ~15;
    const int nch = ldq / 16;
    const int rowb = w * kBlkRW;
    const int g = (int)(blockIdx.x % G);
    const int64_t tg = blockIdx.x / G, ngroups = gridDim.x / G;
    double *tile = ws + tg * blk_region_doubles(m);
    const double eps = DBL_MIN;

    for (int64_t t = tg; t < ntiles; t += ngroups) {
        int *tflags = flags + t * nch;
        const int64_t r0 = t * kBlkTR;
        const int nvalid = (int)min<int64_t>(kBlkTR, rows - r0);
        // row r of the tile is row (r + rphase) mod tri of its stacked triangle
        const int rphase = tri ? (int)(r0 % tri) : 0;
        // copy-in of this workgroup's chunks: coalesced column reads, zero padding
        for (int c = 16 * g; c < ldq; c += (c & 15) == 15 ? 16 * G - 15 : 1) {
            const Tin *src = W + r0 + ld * (c < m ? c : 0);  // uniform
#pragma unroll
            for (int i = 0; i < kBlkTR / kBlkThreads; ++i) {
                const int r = tid + kBlkThreads * i;
                const bool ok = r < nvalid && c < m;
                tile[q4i(r, c, ldq)] = ok ? (double)Elem<Tin>::load(src + r) : 0.0;
            }
        }
        if (G > 1 && g == 0) blk_release(&tflags[0]);
        __syncthreads();

        // panels beyond the valid rows only touch zero rows: skipped
        const int npan = min(ldq, (nvalid + 15) & ~15) / 16;
        for (int pi = 0; pi < npan; ++pi) {
            const int p = pi * 16;
            const bool own_panel = (pi % G) == g;
            if (G > 1 && !own_panel) blk_wait(&tflags[pi]);
            // ---------------------------------------- panel factorization
            double a[kBlkRPT][16];
            double dg[kBlkRPT];
#pragma unroll
            for (int i = 0; i < kBlkRPT; ++i) {
                const int r = rowb + lane + kWave * i;
                dg[i] = 0.0;
#pragma unroll
                for (int k = 0; k < 16; ++k) a[i][k] = tile[q4i(r, p + k, ldq)];
            }
            // ||u||^2 and the pivot of the next column, carried from one step to
            // the next (see the end of a step); `direct` asks for a fresh sum
            double nx_tot = 0.0, nx_u1 = 0.0;
            bool nx_direct = true;
            static_for<0, 16>([&](auto jc) {
                constexpr int j = decltype(jc)::value;
                constexpr int buf = j & 1;
                const int dj = p + j;
                // this lane's first row, opaque to the compiler in every step so
                // that the row tests of all 16 steps are not hoisted together
                int rl = rowb + lane;
                __asm__ volatile("" : "+v"(rl));
                double tot = nx_tot, u1 = nx_u1;
                if (nx_direct) {  // uniform
                    // ||column j below the diagonal||^2 and the pivot u1
                    double s = 0.0;
#pragma unroll
                    for (int i = 0; i < kBlkRPT; ++i) {
                        const int r = rl + kWave * i;
                        if (r > dj) s = fma(a[i][j], a[i][j], s);
                        if (r == dj) sh.u1[buf] = a[i][j];
                    }
                    s = wave_sum(s);
                    if (lane == 0) sh.red[buf][w] = s;
                    __syncthreads();
                    tot = 0.0;
#pragma unroll
                    for (int q = 0; q < kBlkWaves; ++q) tot += sh.red[buf][q];
                    u1 = sh.u1[buf];
                    tot = fma(u1, u1, tot);
                }
                // Algorithm 6: t = ||u||^2 + eps, alpha = -sign(u1) sqrt(t + eps),
                // v = (u - alpha e1) / sqrt(t - alpha u1), ||v||^2 = 2
                double tt = tot + eps;
                const double t2 = tt + eps;
                double alpha = t2 * rsqrt_nr(t2);
                alpha = (u1 > 0.0) ? -alpha : alpha;
                tt = fma(-alpha, u1, tt);
                const double beta = rsqrt_nr(tt);
                double v[kBlkRPT];
#pragma unroll
                for (int i = 0; i < kBlkRPT; ++i) {
                    const int r = rl + kWave * i;
                    v[i] = r > dj ? beta * a[i][j] : (r == dj ? beta * (u1 - alpha) : 0.0);
                    if (r == dj) dg[i] = alpha;
                }
                // v . (every other panel column): trailing columns k > j give
                // the update coefficients, earlier reflectors k < j give
                // G(k, j) = y_k . v (rows < dj of column k hold R entries, but
                // v is zero there)
                // Slot j carries N = ||column j+1 over rows >= dj||^2 before the
                // update: the reflector preserves it, so the next step's
                // ||u||^2 is N - R(dj, j+1)^2 without another reduction (the
                // pivot rows dj and dj+1 of column j+1 and of v go through LDS).
                double d[16];
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    double acc = 0.0;
                    if (k != j) {
#pragma unroll
                        for (int i = 0; i < kBlkRPT; ++i) acc = fma(v[i], a[i][k], acc);
                    } else if (j + 1 < 16) {
#pragma unroll
                        for (int i = 0; i < kBlkRPT; ++i)
                            if (rl + kWave * i >= dj) acc = fma(a[i][j + 1], a[i][j + 1], acc);
                    }
                    d[k] = acc;
                }
                if (j + 1 < 16) {
#pragma unroll
                    for (int i = 0; i < kBlkRPT; ++i) {
                        const int r = rl + kWave * i;
                        if (r == dj) {
                            sh.nx[buf][0] = a[i][(j + 1) & 15];
                            sh.nx[buf][1] = v[i];
                        }
                        if (r == dj + 1) {
                            sh.nx[buf][2] = a[i][(j + 1) & 15];
                            sh.nx[buf][3] = v[i];
                        }
                    }
                }
                const double dsum = wave_reduce_keys<16>(d);  // value lane >> 2
                if ((lane & 3) == 0) sh.part[buf][w][lane >> 2] = dsum;
                __syncthreads();
                // lane k: value k summed over the waves in a fixed order
                double gk = 0.0;
                if (lane < 16) {
#pragma unroll
                    for (int q = 0; q < kBlkWaves; ++q) gk += sh.part[buf][q][lane];
                    if (w == 0 && lane < j) sh.G[lane][j] = gk;
                }
#pragma unroll
                for (int k = j + 1; k < 16; ++k) {
                    const double g = read_lane(gk, k);
#pragma unroll
                    for (int i = 0; i < kBlkRPT; ++i) a[i][k] = fma(-g, v[i], a[i][k]);
                }
                // column j keeps R above the diagonal and the reflector from it down
#pragma unroll
                for (int i = 0; i < kBlkRPT; ++i)
                    if (rl + kWave * i >= dj) a[i][j] = v[i];
                // the next step's ||u||^2 and pivot, identical in every thread
                // (the pivot is the value the update just left in its lane);
                // where the downdate would cancel (the column nearly in the span
                // of the earlier ones), the next step sums afresh
                if (j + 1 < 16) {
                    const double n2 = read_lane(gk, j);
                    const double wn = read_lane(gk, (j + 1) & 15);
                    const double rjn = fma(-wn, sh.nx[buf][1], sh.nx[buf][0]);
                    nx_u1 = fma(-wn, sh.nx[buf][3], sh.nx[buf][2]);
                    nx_tot = fma(-rjn, rjn, n2);
                    nx_direct = !(nx_tot >= 0.25 * n2) || !(n2 > 0.0);
                }
                __builtin_amdgcn_sched_barrier(0);  // keep the steps apart (register pressure)
            });
            // Y to LDS (zero above each reflector's first row); the owner writes
            // the panel's diagonal block of the factor (rows p..p+15) directly
            // to the output (the tile's panel columns may still be read by the
            // other workgroups of the group)
            double *odiag = out + t * out_row0_stride;
#pragma unroll
            for (int i = 0; i < kBlkRPT; ++i) {
                const int r = rowb + lane + kWave * i;
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    sh.y[yl(r, k)] = (r >= p + k) ? a[i][k] : 0.0;
                    if (own_panel && r >= p && r < p + 16 && r < m && p + k < m) {
                        const bool keep = r <= p + k && r < kvalid && r < nvalid;
                        odiag[r + ld_out * (p + k)] = keep ? (r < p + k ? a[i][k] : dg[i]) : 0.0;
                    }
                }
            }
            // T: T(j, j) = 1, T(k, j) = -sum_{k <= q < j} T(k, q) G(q, j); lane k
            // of wave 0 builds row k in LDS (G was written by wave 0 itself)
            if (w == 0) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                if (lane < 16) {
                    // row `lane` of T in registers (T(lane, q) = 0 for q < lane)
                    double tr[16];
#pragma unroll
                    for (int jj = 0; jj < 16; ++jj) {
                        double tj = 0.0;
#pragma unroll
                        for (int q = 0; q < jj; ++q) tj = fma(tr[q], sh.G[q][jj], tj);
                        tr[jj] = (lane < jj) ? -tj : (lane == jj ? 1.0 : 0.0);
                    }
#pragma unroll
                    for (int q = 0; q < 16; ++q) sh.tl[lane][q] = tr[q];
                }
            }
            __syncthreads();

            // ---------------------------------------- trailing update
            if (p + 16 < ldq) {
                double tA[4];  // T^T(i, 4q + kk) = T(4q + kk, i), lane (i, kk) = (lr, lg)
#pragma unroll
                for (int q = 0; q < 4; ++q) tA[q] = sh.tl[4 * q + lg][lr];
                // 16-row blocks of this wave that can hold nonzero reflector
                // entries: rows >= p below the valid rows; in a stack of
                // triangles, the pivot rows (< p + 16) and the rows whose index
                // in their triangle is at most p + 15 (the others are untouched
                // and zero in the panel's columns)
                auto live = [&](int rb) {
                    return rb + 15 >= p && rb < nvalid &&
                           (tri == 0 || rb < p + 16 || ((rb + rphase) % tri) < p + 16);
                };
                // this workgroup's chunks, the next panel's first
                const int c_first = p + 16 + 16 * ((g - (pi + 1) % G + G) % G);
                for (int c0 = c_first; c0 < ldq; c0 += 16 * G) {
                    // Lane parts of the addresses, made opaque to the compiler in
                    // every chunk so that it recomputes the 64 per-block addresses
                    // instead of keeping them all live across the loop.
                    int lt = lr * 4 + lg;  // tile: C(rowb + 4 s + lg, c0 + lr)
                    int la[4], lu[4];      // LDS: Y(rb + 4 u + lg, lr), Y(rb + lr, 4 u + lg)
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        la[u] = yl(4 * u + lg, lr);
                        lu[u] = yl(lr, 4 * u + lg);
                    }
                    __asm__ volatile("" : "+v"(lt));
#pragma unroll
                    for (int u = 0; u < 4; ++u) __asm__ volatile("" : "+v"(la[u]), "+v"(lu[u]));
                    // C(rowb + 4 s + lg, c0 + lr): B operand of W = Y^T C and,
                    // four K-steps at a time, the accumulator of C -= Y W'
                    double cv[kBlkKS];
                    blk_d4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int b = 0; b < kBlkRB; ++b) {
                        const int rb = rowb + 16 * b;
                        if (live(rb)) {  // uniform
#pragma unroll
                            for (int u = 0; u < 4; ++u)
                                cv[4 * b + u] = tile[lt + (((rb >> 2) + u) * ldq + c0) * 4];
#pragma unroll
                            for (int u = 0; u < 4; ++u) {
                                const double ya = sh.y[la[u] + rb * 16];
                                if (u & 1)
                                    acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(ya, cv[4 * b + u], acc1, 0, 0, 0);
                                else
                                    acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(ya, cv[4 * b + u], acc0, 0, 0, 0);
                            }
                        }
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q) sh.wpart[w][q][lane] = acc0[q] + acc1[q];
                    __syncthreads();
                    double wsum[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        double x = 0.0;
#pragma unroll
                        for (int u = 0; u < kBlkWaves; ++u) x += sh.wpart[u][q][lane];
                        wsum[q] = x;
                    }
                    __syncthreads();  // wpart is rewritten by the next chunk
                    // W' = T^T W (D layout: lane (lr, lg), value q = W'(4q + lg, c0 + lr))
                    blk_d4 wp = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int q = 0; q < 4; ++q) wp = __builtin_amdgcn_mfma_f64_16x16x4f64(tA[q], wsum[q], wp, 0, 0, 0);
                    // C(rows, cols) -= Y W', 16 rows at a time: D(i = row, j = col)
                    // with rows rb + 4 u + lg in value u, A = -Y(rb + lr, 4q + lg),
                    // B = W'(4q + lg, c0 + lr)
#pragma unroll
                    for (int b = 0; b < kBlkRB; ++b) {
                        const int rb = rowb + 16 * b;
                        if (live(rb)) {  // uniform
                            blk_d4 D = {cv[4 * b], cv[4 * b + 1], cv[4 * b + 2], cv[4 * b + 3]};
#pragma unroll
                            for (int q = 0; q < 4; ++q)
                                D = __builtin_amdgcn_mfma_f64_16x16x4f64(-sh.y[lu[q] + rb * 16], wp[q], D, 0, 0, 0);
#pragma unroll
                            for (int u = 0; u < 4; ++u) tile[lt + (((rb >> 2) + u) * ldq + c0) * 4] = D[u];
                        }
                    }
                    if (G > 1 && c0 == p + 16) blk_release(&tflags[pi + 1]);
                }
            }
            __syncthreads();
        }
        // this workgroup's columns of the factor: rows above the diagonal block
        // from the tile, the diagonal block written with its panel (if that
        // panel ran), zero below
        for (int c = 16 * g; c < m; c += (c & 15) == 15 ? 16 * G - 15 : 1) {
            double *dst = out + t * out_row0_stride + ld_out * c;  // uniform
            const int c16 = c & ~15;
            for (int r = tid; r < m; r += kBlkThreads) {
                if (r >= c16 && r < c16 + 16 && c16 < npan * 16) continue;
                dst[r] = (r < c16 && r < kvalid && r < nvalid) ? tile[q4i(r, c, ldq)] : 0.0;
            }
        }
        __syncthreads();  // the next tile reuses the region
    }
}

bool &blk_shared_tiles() {
    static thread_local bool on = true;
    return on;
}

__global__ void blk_zero_flags(int *flags, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        flags[i] = 0;
}

template <typename Tin>
int tsqr_blk_level(const Tin *W, int64_t rows, int64_t m, int64_t ld, bool tree, int64_t ntiles,
                   double *ws, double *out, int64_t ld_out, int64_t out_stride, int kvalid,
                   hipStream_t s) {
    if (m <= 0 || m > kBlkMaxM) return set_error(TTSVD_EUNSUPPORTED, "tsqr_blk: m = %lld", (long long)m);
    int tri = (tree && m % 16 == 0) ? (int)m : 0;
    int G = blk_group(ntiles, m);
    const int64_t grid = blk_grid(ntiles, m);
    const int64_t nflags = G > 1 ? ntiles * ((m + 15) / 16) : 0;
    int *flags = reinterpret_cast<int *>(ws);
    double *regions = ws + (G > 1 ? (nflags + 63) / 64 * 32 : 0);
    int mi = (int)m;
    if (G == 1) {
        hipLaunchKernelGGL((tsqr_blk_kernel<Tin>), dim3((unsigned)grid), dim3(kBlkThreads), 0, s, W,
                           rows, mi, ld, tri, ntiles, G, flags, regions, out, ld_out, out_stride,
                           kvalid);
        TTSVD_HIP_TRY(hipGetLastError());
        return TTSVD_OK;
    }
    // a shared tile needs its G workgroups resident together: cooperative launch
    hipLaunchKernelGGL(blk_zero_flags, dim3((unsigned)std::min<int64_t>(64, ceil_div(nflags, 256))),
                       dim3(256), 0, s, flags, nflags);
    TTSVD_HIP_TRY(hipGetLastError());
    void *args[] = {(void *)&W,     (void *)&rows,   (void *)&mi,  (void *)&ld,
                    (void *)&tri,   (void *)&ntiles, (void *)&G,   (void *)&flags,
                    (void *)&regions, (void *)&out,  (void *)&ld_out, (void *)&out_stride,
                    (void *)&kvalid};
    TTSVD_HIP_TRY(coop_launch((const void *)tsqr_blk_kernel<Tin>, dim3((unsigned)grid),
                              dim3(kBlkThreads), args, 0, s));
    return TTSVD_OK;
}

template int tsqr_blk_level<double>(const double *, int64_t, int64_t, int64_t, bool, int64_t,
                                    double *, double *, int64_t, int64_t, int, hipStream_t);
template int tsqr_blk_level<float>(const float *, int64_t, int64_t, int64_t, bool, int64_t,
                                   double *, double *, int64_t, int64_t, int, hipStream_t);
template int tsqr_blk_level<bf16>(const bf16 *, int64_t, int64_t, int64_t, bool, int64_t,
                                  double *, double *, int64_t, int64_t, int, hipStream_t);

}  // namespace ttsvd
