// Batched TSQR TT-SVD: Algorithm 2 of arXiv 2102.00104 applied to many
// independent tensors of different shapes in ONE persistent cooperative
// launch.
//
// All tensors advance in lock step: round s performs TT step d_t - 1 - s of
// every tensor t that still has one.  A round has three kinds of phases,
// separated by grid-wide barriers:
//   * TSQR level L (L = 0, 1, ...): the slices of level L of every active
//     tensor's reduction tree (the same tree as the single-tensor path);
//   * SVD: one workgroup per tensor runs the one-sided Jacobi SVD of R, the
//     truncation rule and the core emission, then derives the shape of the
//     tensor's next step from the rank it chose -- ranks never go back to the
//     host, so tolerances cost no synchronisation;
//   * TSMM: the blocks of every tensor's fused product + reshape.
// Within a phase the work units of all tensors form one list (a prefix sum
// over per-tensor unit counts, computed redundantly by every workgroup from
// device state written before the last barrier) that the workgroups stride
// through, so small and large tensors share the machine.  Every loop has a
// bound known before it starts and every workgroup reaches every barrier, so
// the grid always drains.
// Bodies in this translation unit read the thread index through an opaque
// statement (see thread_id in common.h).
#define TTSVD_PERSISTENT_KERNEL 1

#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"
#include "driver.h"
#include "kernels.h"
#include "profile.h"
#include "svd_dev.h"
#include "tsmm_dev.h"
#include "tsqr_dev.h"

namespace ttsvd {
namespace {

constexpr int kBThreads = 256;  // one wave per SIMD: registers beyond 256 go to AGPRs, not scratch
constexpr int kBWaves = kBThreads / kWave;
constexpr int kBMaxM = 128;
constexpr int kBMaxTensors = 4096;

// Tile set: rows per lane of the row-owner TSQR body (m <= 8) and of the
// cooperative body per column bucket (16, 32, 64, 128).
struct BTiles {
    int rows_rpt;
    int coop_rpt[4];
};
__host__ __device__ constexpr BTiles btiles(int ts) {
    return ts == 0 ? BTiles{8, {16, 8, 4, 2}} : BTiles{4, {8, 4, 2, 1}};
}
// Tile sets the autotuner may choose: set 0 for every storage type, set 1
// (half the rows per lane: more, shorter slices) built for FP32 storage, the
// batched form's type.
constexpr int kBTileSets = 2;
__host__ __device__ inline bool tile_set_built(int dtype, int ts) {
    return ts == 0 || (ts == 1 && dtype == TTSVD_F32);
}

__host__ __device__ inline int bucket_of(int64_t m) {
    return m <= 16 ? 0 : m <= 32 ? 1 : m <= 64 ? 2 : 3;
}
__host__ __device__ inline int64_t btile(int ts, int64_t m) {
    // (a chain of selects: a runtime-indexed array would live in scratch)
    const BTiles t = btiles(ts);
    const int b = bucket_of(m);
    const int rpt = m <= 8 ? t.rows_rpt
                           : b == 0 ? t.coop_rpt[0]
                           : b == 1 ? t.coop_rpt[1]
                           : b == 2 ? t.coop_rpt[2] : t.coop_rpt[3];
    return (int64_t)kWave * rpt;
}

// Shape of one TT step of one tensor.
struct BStep {
    const void *W;       // input work matrix (storage type), column-major
    int64_t ld, rows;
    int m, K;
    void *Y;             // output: next work matrix, or FP64 core 0 after the last step
    int64_t ld_y, n_next;
    int nlev;
    TsqrLevel lv[kTsqrMaxLevels];
};

struct BTask {
    int d, base;         // per-step arrays hold this tensor's steps at base + 0 .. base + d - 1
    int64_t r_max;
    double tol;
    void *wbuf[2];       // ping-pong work matrices
    double *R;           // triangular factor (m x m)
    double *tq[2];       // TSQR tree levels
};

struct GridBarrier;

struct BArgs {
    const BTask *task;
    int ntask;
    BStep *step;
    double *const *core;
    double *const *sigma;
    StepState *st;
    const int64_t *dims;
    int nrounds;
    int ts;
    TsqrPlanParams pr, pc;  // planner parameters, row-owner / cooperative bodies
    GridBarrier *bar;
    uint64_t *clk;  // optional: (time, phase) after every barrier, by workgroup 0
};

__host__ __device__ inline void make_bstep(BStep &s, int ts, TsqrPlanParams pr, TsqrPlanParams pc,
                                           const void *W, int64_t ld, int64_t rows, int64_t m,
                                           void *Y, int64_t n_next) {
    s.W = W;
    s.ld = ld;
    s.rows = rows;
    s.m = (int)m;
    s.K = (int)(rows < m ? rows : m);
    s.Y = Y;
    s.n_next = n_next;
    s.ld_y = rows / n_next;
    s.nlev = tsqr_plan_levels(rows, m, btile(ts, m), m <= 8 ? pr : pc, s.lv);
}

__host__ __device__ inline int64_t tsqr_units(const BStep &sp, int lev) {
    const int64_t ns = sp.lv[lev].nslices;
    return sp.m <= 8 ? (ns + kBWaves - 1) / kBWaves : ns;
}

__device__ __forceinline__ int tsmm_kb(int k) { return cpow2(k < 64 ? k : 64); }

// Rows per thread of the TSMM body for a KB-column block (kept small: the
// persistent kernel holds every body in one register allocation).
__host__ __device__ constexpr int btsmm_rpt(int KB) { return tsmm_rpt(KB); }

__device__ __forceinline__ int64_t tsmm_tx(const BStep &sp, int k) {
    const int64_t per = (int64_t)kBThreads * btsmm_rpt(tsmm_kb(k));
    return (sp.rows + per - 1) / per;
}

// Grid-wide barrier of the persistent launch with a bounded wait: a
// workgroup that waits longer than kBarrierNs (only possible if the grid is
// not co-resident) raises `abort`, and every workgroup that sees it leaves
// the kernel, so the launch always ends; the host then reports the error.
struct GridBarrier {
    unsigned count;  // arrivals at the current barrier
    unsigned gen;    // barriers completed
    unsigned abort;
    unsigned pad;
};
constexpr uint64_t kBarrierTicks = 20ull * 100000000ull;  // 20 s of the 100 MHz clock

__device__ __forceinline__ bool grid_barrier(GridBarrier *b, unsigned &gen, int *flag) {
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        const unsigned target = gen + 1;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned prev =
            __hip_atomic_fetch_add(&b->count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (prev == gridDim.x - 1) {
            __hip_atomic_store(&b->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&b->gen, target, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            const uint64_t t0 = wall_clock64();
            while (__hip_atomic_load(&b->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != target) {
                if (__hip_atomic_load(&b->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    ok = 0;
                    break;
                }
                if (wall_clock64() - t0 > kBarrierTicks) {
                    __hip_atomic_store(&b->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(8);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        gen = target;
        *flag = ok;
    }
    __syncthreads();
    return *flag != 0;
}

// A workgroup-uniform value read from LDS, moved to a scalar register so that
// everything derived from it (tensor parameters, addresses) stays scalar.
__device__ __forceinline__ uint32_t uniform(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}

// Exclusive prefix sums pref[0..n] of count(t) over t < n, by the whole
// workgroup (tmp: blockDim.x entries of LDS).  Returns the total.
template <typename F>
__device__ __forceinline__ uint32_t block_prefix(int n, F count, uint32_t *pref, uint32_t *tmp) {
    const int tid = threadIdx.x, nth = blockDim.x;
    const int per = (n + nth - 1) / nth;
    const int t0 = min(n, tid * per), t1 = min(n, t0 + per);
    uint32_t s = 0;
    for (int t = t0; t < t1; ++t) s += count(t);
    tmp[tid] = s;
    __syncthreads();
    for (int off = 1; off < nth; off <<= 1) {
        const uint32_t v = tid >= off ? tmp[tid - off] : 0u;
        __syncthreads();
        tmp[tid] += v;
        __syncthreads();
    }
    uint32_t base = tmp[tid] - s;
    for (int t = t0; t < t1; ++t) {
        pref[t] = base;
        base += count(t);
    }
    const uint32_t total = uniform(tmp[nth - 1]);
    if (tid == 0) pref[n] = total;
    __syncthreads();
    return total;
}

// Tensor owning unit u: the t with pref[t] <= u < pref[t + 1].
__device__ inline int unit_owner(const uint32_t *pref, int n, uint32_t u) {
    int lo = 0, hi = n;  // pref[lo] <= u < pref[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (uniform(pref[mid]) <= u)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// One TSQR slice (or a group of kBWaves single-wave slices) of one level.
template <typename T, int TS>
__device__ __forceinline__ void tsqr_unit_body(const T *W, int64_t rows, int m, int64_t ld, const TsqrLevel &l,
                               double *out, int64_t ld_out, int kv, int64_t unit, void *smem) {
    constexpr BTiles tl = btiles(TS);
    if (m <= 8) {
        const int M = (int)cpow2(m);
#define TTSVD_B_ROWS(MM)                                                                      \
    case MM:                                                                                  \
        tsqr_rows_body<MM, tl.rows_rpt, T, kBWaves>(W, rows, m, ld, l.rows_per_slice,          \
                                                    l.nslices, out, ld_out, m, kv, unit, smem); \
        break;
        switch (M) {
            TTSVD_B_ROWS(1)
            TTSVD_B_ROWS(2)
            TTSVD_B_ROWS(4)
            default:
                TTSVD_B_ROWS(8)
        }
#undef TTSVD_B_ROWS
    } else if (m <= 16) {
        tsqr_coop_body<16, kBWaves, tl.coop_rpt[0], T>(W, rows, m, ld, l.rows_per_slice, unit, out,
                                                       ld_out, m, kv, smem);
    } else if (m <= 32) {
        tsqr_coop_body<32, kBWaves, tl.coop_rpt[1], T>(W, rows, m, ld, l.rows_per_slice, unit, out,
                                                       ld_out, m, kv, smem);
    } else if (m <= 64) {
        tsqr_coop_body<64, kBWaves, tl.coop_rpt[2], T>(W, rows, m, ld, l.rows_per_slice, unit, out,
                                                       ld_out, m, kv, smem);
    } else {
        tsqr_coop_body<128, kBWaves, tl.coop_rpt[3], T>(W, rows, m, ld, l.rows_per_slice, unit,
                                                        out, ld_out, m, kv, smem);
    }
}

template <typename Tin, int TS>
__device__ __forceinline__ void run_tsqr_unit(const BArgs &a, int t, int s, int lev, int64_t unit, void *smem) {
    const BTask &tk = a.task[t];
    const int j = tk.d - 1 - s;
    const BStep &sp = a.step[tk.base + j];
    const TsqrLevel &l = sp.lv[lev];
    const bool last = lev + 1 == sp.nlev;
    double *out = last ? tk.R : tk.tq[lev & 1];
    const int64_t ld_out = last ? (int64_t)sp.m : l.nslices * sp.m;
    const int kv = last ? sp.K : sp.m;
    if constexpr (std::is_same<Tin, double>::value) {
        // one instantiation serves W and the FP64 tree levels
        const double *in = lev == 0 ? (const double *)sp.W : tk.tq[(lev - 1) & 1];
        tsqr_unit_body<double, TS>(in, l.rows, sp.m, lev == 0 ? sp.ld : l.rows, l, out, ld_out, kv,
                                   unit, smem);
    } else if (lev == 0) {
        tsqr_unit_body<Tin, TS>((const Tin *)sp.W, l.rows, sp.m, sp.ld, l, out, ld_out, kv, unit,
                                smem);
    } else {
        tsqr_unit_body<double, TS>(tk.tq[(lev - 1) & 1], l.rows, sp.m, l.rows, l, out, ld_out, kv,
                                   unit, smem);
    }
}

template <int TS>
__device__ __forceinline__ void run_svd_unit(const BArgs &a, int t, int s, void *smem) {
    const BTask &tk = a.task[t];
    const int j = tk.d - 1 - s;
    const BStep &sp = a.step[tk.base + j];
    StepState *st = a.st + tk.base + j;
    StepState *st0 = a.st + tk.base + tk.d - 1;
    const int m = sp.m, K = sp.K;
    double *sig = a.sigma[tk.base + j];
    double *core = a.core[tk.base + j];
    const int first = (j == tk.d - 1);
    if (m <= 16)
        svd_small_body<16, 8>(tk.R, m, K, m, sig, core, tk.r_max, tk.tol, tk.d - 1, first, st, st0, smem);
    else if (m <= 32)
        svd_small_body<32, 8>(tk.R, m, K, m, sig, core, tk.r_max, tk.tol, tk.d - 1, first, st, st0, smem);
    else if (m <= 64)
        svd_small_body<64, 8>(tk.R, m, K, m, sig, core, tk.r_max, tk.tol, tk.d - 1, first, st, st0, smem);
    else
        svd_small_body<128, 4>(tk.R, m, K, m, sig, core, tk.r_max, tk.tol, tk.d - 1, first, st, st0, smem);
    // Shape of the next step, W^(j-1) = reshape(W^(j) V_r) (rows / n_{j-1}
    // rows, n_{j-1} r columns), from the rank just chosen.
    if (threadIdx.x == 0 && j >= 2) {
        const int64_t r = st->rank;
        const int64_t nj1 = a.dims[tk.base + j - 1];
        void *Y = (j - 1 >= 2) ? tk.wbuf[(tk.d - j) & 1] : (void *)a.core[tk.base];
        make_bstep(a.step[tk.base + j - 1], a.ts, a.pr, a.pc, sp.Y, sp.ld_y, sp.ld_y, nj1 * r, Y,
                   a.dims[tk.base + j - 2]);
    }
}

template <typename Tin>
__device__ __forceinline__ void run_tsmm_unit(const BArgs &a, int t, int s, int64_t unit, void *smem) {
    const BTask &tk = a.task[t];
    const int j = tk.d - 1 - s;
    const BStep &sp = a.step[tk.base + j];
    const int k = (int)a.st[tk.base + j].rank;
    const int KB = tsmm_kb(k);
    const int64_t tx = tsmm_tx(sp, k);
    const int64_t bx = unit % tx;
    const int by = (int)(unit / tx);
    const double *V = a.core[tk.base + j];
    const int64_t rn = sp.ld_y;
#define TTSVD_B_TSMM(KK)                                                                          \
    case KK:                                                                                      \
        if (j >= 2)                                                                               \
            tsmm_body<KK, btsmm_rpt(KK), Tin, Tin, kBThreads>((const Tin *)sp.W, sp.rows, sp.m,   \
                                                             sp.ld, V, k, 1, k, rn, sp.n_next,    \
                                                             (Tin *)sp.Y, sp.ld_y, bx, by, smem); \
        else                                                                                      \
            tsmm_body<KK, btsmm_rpt(KK), Tin, double, kBThreads>(                                 \
                (const Tin *)sp.W, sp.rows, sp.m, sp.ld, V, k, 1, k, rn, sp.n_next,               \
                (double *)sp.Y, sp.ld_y, bx, by, smem);                                           \
        break;
    switch (KB) {
        TTSVD_B_TSMM(1)
        TTSVD_B_TSMM(2)
        TTSVD_B_TSMM(4)
        TTSVD_B_TSMM(8)
        TTSVD_B_TSMM(16)
        TTSVD_B_TSMM(32)
        default:
            TTSVD_B_TSMM(64)
    }
#undef TTSVD_B_TSMM
}

// LDS of the largest body (the m <= 128 SVD) ahead of the prefix arrays.
constexpr size_t kBBodySmem = SvdSmall<128, 4>::smem_bytes();
static_assert(kBBodySmem >= tsqr_coop_smem<128, kBWaves, 16, double>(), "LDS");
static_assert(kBBodySmem >= tsmm_smem<64, 1, double>(), "LDS");

size_t batch_smem_bytes(int ntask) {
    return align256(kBBodySmem) + sizeof(uint32_t) * ((size_t)ntask + 1 + kBThreads);
}

template <typename Tin, int TS>
__global__ __launch_bounds__(kBThreads) void batch_kernel(BArgs a) {
    extern __shared__ __attribute__((aligned(16))) char smem[];
    __shared__ int bar_flag;
    unsigned gen = 0;
    // phase clock: 100 MHz wall clock after each barrier (workgroup 0 only)
    auto stamp = [&](int phase) {
        if (a.clk && blockIdx.x == 0 && threadIdx.x == 0) {
            a.clk[2 * gen] = wall_clock64();
            a.clk[2 * gen + 1] = (uint64_t)phase;
        }
    };
    stamp(-1);
    uint32_t *pref = reinterpret_cast<uint32_t *>(smem + align256(kBBodySmem));
    uint32_t *tmp = pref + a.ntask + 1;

    for (int s = 0; s < a.nrounds; ++s) {
        // TSQR, level by level
        for (int lev = 0; lev < kTsqrMaxLevels; ++lev) {
            auto cnt = [&](int t) -> uint32_t {
                const BTask &tk = a.task[t];
                const int j = tk.d - 1 - s;
                if (j < 1) return 0u;
                const BStep &sp = a.step[tk.base + j];
                return lev < sp.nlev ? (uint32_t)tsqr_units(sp, lev) : 0u;
            };
            const uint32_t total = block_prefix(a.ntask, cnt, pref, tmp);
            if (total == 0) break;  // same value in every workgroup
            for (uint32_t u = blockIdx.x; u < total; u += gridDim.x) {
                const int t = unit_owner(pref, a.ntask, u);
                run_tsqr_unit<Tin, TS>(a, t, s, lev, u - uniform(pref[t]), smem);
                __syncthreads();
            }
            if (!grid_barrier(a.bar, gen, &bar_flag)) return;
            stamp(0);
        }
        // SVD, rank, core, next step's shape
        {
            auto cnt = [&](int t) -> uint32_t { return a.task[t].d - 1 - s >= 1 ? 1u : 0u; };
            const uint32_t total = block_prefix(a.ntask, cnt, pref, tmp);
            for (uint32_t u = blockIdx.x; u < total; u += gridDim.x) {
                const int t = unit_owner(pref, a.ntask, u);
                run_svd_unit<TS>(a, t, s, smem);
                __syncthreads();
            }
            if (!grid_barrier(a.bar, gen, &bar_flag)) return;
            stamp(1);
        }
        // TSMM + reshape
        {
            auto cnt = [&](int t) -> uint32_t {
                const BTask &tk = a.task[t];
                const int j = tk.d - 1 - s;
                if (j < 1) return 0u;
                const BStep &sp = a.step[tk.base + j];
                const int k = (int)a.st[tk.base + j].rank;
                const int64_t ty = (k + tsmm_kb(k) - 1) / tsmm_kb(k);
                return (uint32_t)(tsmm_tx(sp, k) * ty);
            };
            const uint32_t total = block_prefix(a.ntask, cnt, pref, tmp);
            for (uint32_t u = blockIdx.x; u < total; u += gridDim.x) {
                const int t = unit_owner(pref, a.ntask, u);
                run_tsmm_unit<Tin>(a, t, s, u - uniform(pref[t]), smem);
                __syncthreads();
            }
            if (!grid_barrier(a.bar, gen, &bar_flag)) return;
            stamp(2);
        }
    }
}

// ---------------------------------------------------------------- host side

struct BatchPlan {
    int dtype = 0;
    int ntask = 0, nsteps = 0, nrounds = 0;
    std::vector<BTask> task;
    std::vector<BStep> step;
    std::vector<int64_t> dims;
    std::vector<size_t> core_off, sigma_off;   // per step (doubles)
    std::vector<std::vector<StepShape>> shapes;
    std::vector<std::vector<int64_t>> rb;
    size_t cores = 0, sigma = 0;
    // per-task workspace sizes (bytes)
    std::vector<size_t> w0, w1, rbytes, tqbytes;
};

size_t ceil_bytes(size_t elems, size_t es) { return align256(elems * es); }

const void *kernel_ptr(int dtype, int ts) {
    switch (dtype) {
        case TTSVD_F64: return (const void *)batch_kernel<double, 0>;
        case TTSVD_F32:
            return ts == 1 ? (const void *)batch_kernel<float, 1> : (const void *)batch_kernel<float, 0>;
        default: return (const void *)batch_kernel<bf16, 0>;
    }
}

// Validates the batch and computes its layout for the rank upper bounds.
int plan_batch(int count, const ttsvd_tensor *X, const int *d, const int64_t *dims,
               const int64_t *r_max, const double *tol, const ttsvd_batch_config &cfg,
               BatchPlan &bp) {
    if (count < 1 || count > kBMaxTensors)
        return set_error(TTSVD_EINVAL, "batch: count = %d (1..%d)", count, kBMaxTensors);
    if (!X || !d || !dims || !r_max || !tol) return set_error(TTSVD_EINVAL, "batch: NULL pointer");
    if (cfg.tile_set < 0 || cfg.tile_set >= kBTileSets || cfg.min_tiles < 1 || cfg.max_slices < 1)
        return set_error(TTSVD_EINVAL, "batch: bad configuration");
    bp.dtype = X[0].dtype;
    if (!valid_dtype(bp.dtype)) return set_error(TTSVD_EUNSUPPORTED, "batch: dtype %d", bp.dtype);
    if (!tile_set_built(bp.dtype, cfg.tile_set))
        return set_error(TTSVD_EUNSUPPORTED, "batch: tile set %d is not built for dtype %d",
                         cfg.tile_set, bp.dtype);
    const TsqrPlanParams pr{cfg.max_slices * kBWaves, cfg.min_tiles};
    const TsqrPlanParams pc{cfg.max_slices, cfg.min_tiles};
    const size_t es = dtype_size(bp.dtype);
    bp.ntask = count;
    bp.task.resize(count);
    bp.shapes.resize(count);
    bp.rb.resize(count);
    bp.w0.assign(count, 0);
    bp.w1.assign(count, 0);
    bp.rbytes.assign(count, 0);
    bp.tqbytes.assign(count, 0);
    int base = 0;
    double units = 0.0;
    for (int t = 0; t < count; ++t) {
        if (!X[t].data) return set_error(TTSVD_EINVAL, "batch: tensor %d: NULL data", t);
        if (X[t].dtype != bp.dtype)
            return set_error(TTSVD_EUNSUPPORTED, "batch: mixed dtypes (tensor %d)", t);
        if (d[t] < 1 || d[t] > TTSVD_MAX_D)
            return set_error(TTSVD_EINVAL, "batch: tensor %d: d = %d", t, d[t]);
        if (r_max[t] < 1) return set_error(TTSVD_EINVAL, "batch: tensor %d: r_max < 1", t);
        if (!(tol[t] >= 0.0) || !std::isfinite(tol[t]))
            return set_error(TTSVD_EINVAL, "batch: tensor %d: tol", t);
        const int64_t *dm = dims + base;
        int64_t nbar;
        int rc = plan_steps(dm, d[t], r_max[t], bp.shapes[t], bp.rb[t], nbar);
        if (rc != TTSVD_OK) return rc;
        const int64_t lead = nbar / dm[d[t] - 1];
        const int64_t ld0 = X[t].ld_last ? X[t].ld_last : lead;
        if (ld0 < lead) return set_error(TTSVD_EINVAL, "batch: tensor %d: ld_last too small", t);
        BTask &tk = bp.task[t];
        tk.d = d[t];
        tk.base = base;
        tk.r_max = r_max[t];
        tk.tol = tol[t];
        for (int i = 0; i < d[t]; ++i) bp.dims.push_back(dm[i]);
        // workspace for the rank upper bounds; a smaller rank only shrinks m
        int pp = 0;
        for (int i = d[t] - 1; i >= 1; --i) {
            const StepShape &sh = bp.shapes[t][i];
            if (sh.m > kBMaxM)
                return set_error(TTSVD_EUNSUPPORTED,
                                 "batch: tensor %d step %d has %lld > %d columns", t, i + 1,
                                 (long long)sh.m, kBMaxM);
            bp.rbytes[t] = std::max(bp.rbytes[t], (size_t)(sh.m * sh.m) * 8);
            const int64_t rnext = i + 1 < d[t] ? bp.rb[t][i + 1] : 1;
            for (int64_t r = 1; r <= rnext; ++r) {
                const int64_t m = dm[i] * r;
                TsqrLevel lv[kTsqrMaxLevels];
                const int n = tsqr_plan_levels(sh.rows, m, btile(cfg.tile_set, m), m <= 8 ? pr : pc, lv);
                if (n == kTsqrMaxLevels && lv[n - 1].nslices > 1)
                    return set_error(TTSVD_EUNSUPPORTED, "batch: TSQR tree too deep");
                for (int q = 0; q + 1 < n; ++q)
                    bp.tqbytes[t] = std::max(bp.tqbytes[t], (size_t)(lv[q].nslices * m * m) * 8);
            }
            if (i >= 2) {
                size_t &w = pp ? bp.w1[t] : bp.w0[t];
                w = std::max(w, (size_t)(sh.rows * sh.rb) * es);
                pp ^= 1;
            }
            units += (double)sh.rows * sh.m / 64.0;
        }
        base += d[t];
        bp.nrounds = std::max(bp.nrounds, d[t] - 1);
    }
    if (units > 2.0e9) return set_error(TTSVD_EUNSUPPORTED, "batch: too much work for one launch");
    bp.nsteps = base;
    // outputs: cores and singular values for the rank upper bounds
    bp.core_off.assign(base, 0);
    bp.sigma_off.assign(base, 0);
    for (int t = 0; t < count; ++t) {
        const BTask &tk = bp.task[t];
        for (int i = 0; i < tk.d; ++i) {
            bp.core_off[tk.base + i] = bp.cores;
            bp.cores += (size_t)(bp.rb[t][i] * bp.dims[tk.base + i] * bp.rb[t][i + 1]);
            if (i >= 1) {
                bp.sigma_off[tk.base + i] = bp.sigma;
                bp.sigma += (size_t)bp.shapes[t][i].K;
            }
        }
    }
    return TTSVD_OK;
}

std::string batch_signature(int count, const ttsvd_tensor *X, const int *d, const int64_t *dims,
                            const int64_t *r_max, const double *tol) {
    std::string k;
    char buf[64];
    snprintf(buf, sizeof(buf), "%d:%d|", count, X[0].dtype);
    k += buf;
    int base = 0;
    for (int t = 0; t < count; ++t) {
        snprintf(buf, sizeof(buf), "%d,%lld,%.17g,%lld;", d[t], (long long)r_max[t], tol[t],
                 (long long)X[t].ld_last);
        k += buf;
        for (int i = 0; i < d[t]; ++i) {
            snprintf(buf, sizeof(buf), "%lld.", (long long)dims[base + i]);
            k += buf;
        }
        base += d[t];
    }
    return k;
}

std::mutex g_tune_mu;
std::map<std::string, ttsvd_batch_config> g_tuned;

ttsvd_batch_config default_config() {
    ttsvd_batch_config c;
    c.grid = 0;
    c.tile_set = 0;
    c.min_tiles = 4;
    c.max_slices = 256;
    return c;
}

int run_batch(int count, const ttsvd_tensor *X, const int *d, const int64_t *dims,
              const int64_t *r_max, const double *tol, const ttsvd_batch_config &cfg,
              hipStream_t s, ttsvd_tt *out) {
    BatchPlan bp;
    int rc = plan_batch(count, X, d, dims, r_max, tol, cfg, bp);
    if (rc != TTSVD_OK) return rc;
    const int n = bp.ntask, ns = bp.nsteps;
    const TsqrPlanParams pr{cfg.max_slices * kBWaves, cfg.min_tiles};
    const TsqrPlanParams pc{cfg.max_slices, cfg.min_tiles};

    // device layout: [tasks][steps][core ptrs][sigma ptrs][dims][state][sigma][per-task buffers]
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align256(bytes);
        return o;
    };
    const size_t o_task = take(sizeof(BTask) * n);
    const size_t o_step = take(sizeof(BStep) * ns);
    const size_t o_cptr = take(sizeof(double *) * ns);
    const size_t o_sptr = take(sizeof(double *) * ns);
    const size_t o_dims = take(sizeof(int64_t) * ns);
    const size_t o_st = take(sizeof(StepState) * ns);
    const size_t o_sig = take(sizeof(double) * std::max<size_t>(bp.sigma, 1));
    const size_t o_one = take(sizeof(double));
    const size_t o_bar = take(sizeof(GridBarrier));
    const bool clocks = prof_on();
    const size_t nclk = (size_t)bp.nrounds * (kTsqrMaxLevels + 2) + 1;
    const size_t o_clk = take(clocks ? nclk * 2 * sizeof(uint64_t) : 0);
    const size_t meta = off;  // the host image below covers [0, meta): state starts at zero
    std::vector<size_t> o_w0(n), o_w1(n), o_r(n), o_tq(n);
    for (int t = 0; t < n; ++t) {
        o_w0[t] = take(bp.w0[t]);
        o_w1[t] = take(bp.w1[t]);
        o_r[t] = take(bp.rbytes[t]);
        o_tq[t] = take(2 * bp.tqbytes[t]);
    }
    const size_t total = off;

    SharedDev *shared = new SharedDev();
    shared->ptr = result_alloc(std::max<size_t>(bp.cores, 1) * 8);
    if (!shared->ptr) {
        delete shared;
        return set_error(TTSVD_ENOMEM, "batch: cores (%zu doubles)", bp.cores);
    }
    double *cores = (double *)shared->ptr;
    char *ws = (char *)cache_acquire(total);
    if (!ws) {
        result_free(shared->ptr);
        delete shared;
        return set_error(TTSVD_ENOMEM, "batch: workspace of %zu bytes", total);
    }
    auto fail = [&](int code) {
        (void)hipStreamSynchronize(s);
        cache_release(ws);
        result_free(shared->ptr);
        delete shared;
        return code;
    };

    // host image of the metadata
    // One pinned staging buffer (sized once: growing it could free memory a
    // pending copy still reads) carries the metadata in and the results out.
    const size_t r_bar = 0, r_clk = align256(sizeof(GridBarrier));
    const size_t r_st = r_clk + align256(clocks ? nclk * 2 * 8 : 0);
    const size_t r_sig = r_st + align256(sizeof(StepState) * ns);
    const size_t r_end = r_sig + bp.sigma * 8;
    char *stage = (char *)pinned_stage(std::max(meta, r_end));
    if (!stage) return fail(set_error(TTSVD_ENOMEM, "batch: pinned staging"));
    memset(stage, 0, meta);
    char *img = stage;
    BTask *htask = (BTask *)(img + o_task);
    BStep *hstep = (BStep *)(img + o_step);
    double **hcptr = (double **)(img + o_cptr);
    double **hsptr = (double **)(img + o_sptr);
    int64_t *hdims = (int64_t *)(img + o_dims);
    double *sig_dev = (double *)(ws + o_sig);
    *(double *)(img + o_one) = 1.0;
    for (int i = 0; i < ns; ++i) {
        hcptr[i] = cores + bp.core_off[i];
        hsptr[i] = sig_dev + bp.sigma_off[i];
        hdims[i] = bp.dims[i];
    }
    for (int t = 0; t < n; ++t) {
        BTask tk = bp.task[t];
        tk.wbuf[0] = ws + o_w0[t];
        tk.wbuf[1] = ws + o_w1[t];
        tk.R = (double *)(ws + o_r[t]);
        tk.tq[0] = (double *)(ws + o_tq[t]);
        tk.tq[1] = (double *)(ws + o_tq[t] + bp.tqbytes[t]);
        htask[t] = tk;
        if (tk.d >= 2) {
            const int i = tk.d - 1;
            const StepShape &sh = bp.shapes[t][i];
            const int64_t ld0 = X[t].ld_last ? X[t].ld_last : sh.rows;
            void *Y = (i >= 2) ? tk.wbuf[0] : (void *)hcptr[tk.base];
            make_bstep(hstep[tk.base + i], cfg.tile_set, pr, pc, X[t].data, ld0, sh.rows, sh.m, Y,
                       bp.dims[tk.base + i - 1]);
        }
    }
    if (hipMemcpyAsync(ws, img, meta, hipMemcpyHostToDevice, s) != hipSuccess)
        return fail(set_error(TTSVD_EHIP, "batch: metadata copy"));

    // single-mode tensors: core 0 = X (no SVD), as in the single-tensor path
    for (int t = 0; t < n; ++t) {
        if (bp.task[t].d != 1) continue;
        const int64_t n0 = bp.dims[bp.task[t].base];
        rc = tsmm_launch(X[t].data, bp.dtype, n0, 1, n0, (const double *)(ws + o_one), 1, 1, 1, 1,
                         hcptr[bp.task[t].base], TTSVD_F64, n0, s);
        if (rc != TTSVD_OK) return fail(rc);
    }

    if (bp.nrounds >= 1) {
        BArgs args;
        args.task = (const BTask *)(ws + o_task);
        args.ntask = n;
        args.step = (BStep *)(ws + o_step);
        args.core = (double *const *)(ws + o_cptr);
        args.sigma = (double *const *)(ws + o_sptr);
        args.st = (StepState *)(ws + o_st);
        args.dims = (const int64_t *)(ws + o_dims);
        args.nrounds = bp.nrounds;
        args.ts = cfg.tile_set;
        args.pr = pr;
        args.pc = pc;
        args.bar = (GridBarrier *)(ws + o_bar);
        args.clk = clocks ? (uint64_t *)(ws + o_clk) : nullptr;
        const void *fn = kernel_ptr(bp.dtype, cfg.tile_set);
        const size_t lds = batch_smem_bytes(n);
        if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
            return fail(set_error(TTSVD_EHIP, "batch: %zu bytes of LDS", lds));
        int per_cu = 0, dev = 0, ncu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBThreads, lds) != hipSuccess)
            return fail(set_error(TTSVD_EHIP, "batch: occupancy query"));
        if (per_cu < 1) return fail(set_error(TTSVD_EUNSUPPORTED, "batch: kernel does not fit a CU"));
        // Waves that need scratch can be held back by the scratch allocator,
        // which would break the co-residency the grid barrier relies on.
        hipFuncAttributes fa;
        if (hipFuncGetAttributes(&fa, fn) != hipSuccess)
            return fail(set_error(TTSVD_EHIP, "batch: kernel attributes"));
        if (fa.localSizeBytes != 0)
            return fail(set_error(TTSVD_EUNSUPPORTED, "batch: kernel build uses %zu bytes of scratch",
                                  (size_t)fa.localSizeBytes));
        int grid = per_cu * ncu;
        if (cfg.grid > 0) grid = std::min(grid, cfg.grid);
        void *kargs[] = {&args};
        char name[64];
        snprintf(name, sizeof(name), "batch_kernel<%s, %d>",
                 bp.dtype == TTSVD_F64 ? "double" : bp.dtype == TTSVD_F32 ? "float" : "ttsvd::bf16",
                 cfg.tile_set);
        prof_begin(s, name, 0.0, 0.0);
        const hipError_t e = coop_launch(fn, dim3(grid), dim3(kBThreads), kargs, lds, s);
        prof_end(s);
        if (e != hipSuccess)
            return fail(set_error(TTSVD_EHIP, "batch: cooperative launch: %s", hipGetErrorString(e)));
    }

    // (stream order: these copies run after the metadata copy read the buffer)
    if ((clocks && hipMemcpyAsync(stage + r_clk, ws + o_clk, nclk * 2 * 8, hipMemcpyDeviceToHost, s) != hipSuccess) ||
        hipMemcpyAsync(stage + r_bar, ws + o_bar, sizeof(GridBarrier), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(stage + r_st, ws + o_st, sizeof(StepState) * ns, hipMemcpyDeviceToHost, s) != hipSuccess ||
        (bp.sigma && hipMemcpyAsync(stage + r_sig, sig_dev, bp.sigma * 8, hipMemcpyDeviceToHost, s) != hipSuccess))
        return fail(set_error(TTSVD_EHIP, "batch: result copy"));
    if (hipStreamSynchronize(s) != hipSuccess) {
        cache_release(ws);
        result_free(shared->ptr);
        delete shared;
        return set_error(TTSVD_EHIP, "batch: %s", hipGetErrorString(hipGetLastError()));
    }
    cache_release(ws);
    GridBarrier hbar;
    memcpy(&hbar, stage + r_bar, sizeof(hbar));
    std::vector<uint64_t> hclk(clocks ? nclk * 2 : 0);
    if (clocks) memcpy(hclk.data(), stage + r_clk, nclk * 2 * 8);
    std::vector<StepState> hst(ns);
    memcpy(hst.data(), stage + r_st, sizeof(StepState) * ns);
    std::vector<double> hsig(std::max<size_t>(bp.sigma, 1));
    if (bp.sigma) memcpy(hsig.data(), stage + r_sig, bp.sigma * 8);

    if (clocks && bp.nrounds >= 1 && !hbar.abort) {
        // phase durations from the device clock (time between barriers)
        double ph[3] = {0, 0, 0};
        for (unsigned g = 1; g <= hbar.gen && g < nclk; ++g) {
            const int kind = (int)hclk[2 * g + 1];
            if (kind >= 0 && kind < 3) ph[kind] += (double)(hclk[2 * g] - hclk[2 * g - 2]) * 1e-5;
        }
        static const char *kn[3] = {"tsqr phases", "svd phases", "tsmm phases"};
        for (int k = 0; k < 3; ++k) {
            char nm[96];
            snprintf(nm, sizeof(nm), "batch_kernel: %s", kn[k]);
            prof_add(nm, ph[k], 0.0, 0.0);
        }
    }
    if (hbar.abort) {
        result_free(shared->ptr);
        delete shared;
        return set_error(TTSVD_EHIP, "batch: grid barrier timed out (workgroups not co-resident)");
    }
    // results; a non-finite factor in any tensor fails the whole call, and so
    // does a rank outside [1, min(r_max, K)] (the device state must be whole)
    for (int t = 0; t < n; ++t) {
        const BTask &tk = bp.task[t];
        int64_t nb = 1;
        for (int i = 0; i < tk.d; ++i) nb *= bp.dims[tk.base + i];
        int64_t rn = 1;
        for (int i = tk.d - 1; i >= 1; --i) {
            const int64_t m = bp.dims[tk.base + i] * rn;
            const int64_t rows = nb / m;
            const int64_t K = std::min(rows, m);
            const int64_t r = hst[tk.base + i].rank;
            if (r < 1 || r > std::min(tk.r_max, K)) {
                result_free(shared->ptr);
                delete shared;
                return set_error(TTSVD_EHIP, "batch: tensor %d step %d: device reported rank %lld (K = %lld)",
                                 t, i + 1, (long long)r, (long long)K);
            }
            nb = rows * r;
            rn = r;
        }
    }
    for (int t = 0; t < n; ++t) {
        const BTask &tk = bp.task[t];
        for (int i = tk.d - 1; i >= 1; --i)
            if (hst[tk.base + i].nonfinite) {
                result_free(shared->ptr);
                delete shared;
                return set_error(TTSVD_ENONFINITE, "batch: tensor %d: non-finite sigma in step %d",
                                 t, i + 1);
            }
    }
    shared->refs.store(n);
    for (int t = 0; t < n; ++t) {
        const BTask &tk = bp.task[t];
        ttsvd_tt *o = out + t;
        memset(o, 0, sizeof(*o));
        TTPriv *priv = new TTPriv();
        priv->shared = shared;
        o->priv = priv;
        o->d = tk.d;
        o->ranks[0] = o->ranks[tk.d] = 1;
        for (int i = 0; i < tk.d; ++i) {
            o->dims[i] = bp.dims[tk.base + i];
            o->cores[i] = cores + bp.core_off[tk.base + i];
        }
        for (int i = tk.d - 1; i >= 1; --i) o->ranks[i] = hst[tk.base + i].rank;
        double disc = 0.0;
        int64_t nb = 1;
        for (int i = 0; i < tk.d; ++i) nb *= o->dims[i];
        for (int i = tk.d - 1; i >= 1; --i) {
            const int64_t m = o->dims[i] * o->ranks[i + 1];
            const int64_t rows = nb / m;
            const int64_t K = std::min(rows, m);
            double *h = (double *)malloc(sizeof(double) * (size_t)K);
            if (!h) return set_error(TTSVD_ENOMEM, "batch: host sigma");
            memcpy(h, hsig.data() + bp.sigma_off[tk.base + i], sizeof(double) * (size_t)K);
            priv->sigma_host.push_back(h);
            o->sigma[i] = h;
            o->nsigma[i] = K;
            o->discarded2[i] = hst[tk.base + i].discarded2;
            disc += o->discarded2[i];
            nb = rows * o->ranks[i];
        }
        if (tk.d >= 2) {
            o->norm_sigma = std::sqrt(hst[tk.base + tk.d - 1].norm2);
            o->delta = std::sqrt(hst[tk.base + tk.d - 1].delta2);
        }
        o->err_bound = std::sqrt(disc);
    }
    return TTSVD_OK;
}

}  // namespace
}  // namespace ttsvd

using namespace ttsvd;

extern "C" {

int ttsvd_batch_default_config(ttsvd_batch_config *cfg) {
    if (!cfg) return TTSVD_EINVAL;
    *cfg = default_config();
    return TTSVD_OK;
}

int ttsvd_decompose_batch(int count, const ttsvd_tensor *X, const int *d, const int64_t *dims,
                          const int64_t *r_max, const double *tol,
                          const ttsvd_batch_config *cfg, hipStream_t stream, ttsvd_tt *out) {
    clear_error();
    if (!out || !X || !d || !dims || !r_max || !tol || count < 1)
        return set_error(TTSVD_EINVAL, "batch: NULL pointer or empty batch");
    ttsvd_batch_config c = default_config();
    if (cfg) {
        c = *cfg;
    } else {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tuned.find(batch_signature(count, X, d, dims, r_max, tol));
        if (it != g_tuned.end()) c = it->second;
    }
    return run_batch(count, X, d, dims, r_max, tol, c, stream, out);
}

int ttsvd_batch_autotune(int count, const ttsvd_tensor *X, const int *d, const int64_t *dims,
                         const int64_t *r_max, const double *tol, hipStream_t stream,
                         ttsvd_batch_config *best, double *best_ms) {
    clear_error();
    if (!best || !X || !d || !dims || !r_max || !tol || count < 1)
        return set_error(TTSVD_EINVAL, "autotune: NULL pointer or empty batch");
    static const int kMinTiles[] = {2, 4, 8};
    static const int kMaxSlices[] = {64, 256, 1024};
    std::vector<ttsvd_tt> outs(count);
    double best_t = 1e300;
    ttsvd_batch_config bc = default_config();
    int rc = TTSVD_OK;
    const int dtype = X[0].dtype;
    for (int ts = 0; ts < kBTileSets && rc == TTSVD_OK; ++ts) {
        if (!tile_set_built(dtype, ts)) continue;
        for (int mt : kMinTiles)
            for (int mx : kMaxSlices) {
                ttsvd_batch_config c = default_config();
                c.tile_set = ts;
                c.min_tiles = mt;
                c.max_slices = mx;
                // The objective is what a caller sees: host wall time of the
                // call (it returns with its stream synchronised) plus the
                // release of its results.  Warm-up, then the faster of two.
                double ms = 1e300;
                for (int rep = 0; rep < 3 && rc == TTSVD_OK; ++rep) {
                    const auto t0 = std::chrono::steady_clock::now();
                    rc = run_batch(count, X, d, dims, r_max, tol, c, stream, outs.data());
                    if (rc != TTSVD_OK) break;
                    for (auto &o : outs) ttsvd_tt_free(&o);
                    const auto t1 = std::chrono::steady_clock::now();
                    if (rep > 0)
                        ms = std::min(ms, std::chrono::duration<double, std::milli>(t1 - t0).count());
                }
                if (rc != TTSVD_OK) break;
                if (ms < best_t) {
                    best_t = ms;
                    bc = c;
                }
            }
    }
    if (rc != TTSVD_OK) return rc;
    *best = bc;
    if (best_ms) *best_ms = best_t;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[batch_signature(count, X, d, dims, r_max, tol)] = bc;
    return TTSVD_OK;
}

}  // extern "C"
