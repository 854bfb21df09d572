// Small SVD of the triangular factor, truncation and core emission of the
// TSQR TT-SVD (Algorithm 2 of arXiv 2102.00104): the kernels and their
// launcher.  The method (one-sided Jacobi on the rows of R, truncation rule)
// and the single-workgroup body are described in svd_dev.h.
#include <stdio.h>
#include <stdlib.h>

#include <cmath>

#include "common.h"
#include "driver.h"
#include "kernels.h"
#include "profile.h"
#include "svd_dev.h"

namespace ttsvd {

template <int MB, int LPP>
__global__ __launch_bounds__(MB / 2 * LPP) void svd_small_kernel(
    const double *__restrict__ R, int64_t ldr, int K, int m, double *__restrict__ sigma_out,
    double *__restrict__ core_out, int64_t r_max, double tol, int dm1, int first,
    StepState *st, StepState *st0) {
    __shared__ __attribute__((aligned(16))) char smem[SvdSmall<MB, LPP>::smem_bytes()];
    svd_small_body<MB, LPP>(R, ldr, K, m, sigma_out, core_out, r_max, tol, dm1, first, st, st0,
                            smem);
}

// ----------------------------------------------------------------------------
// Large-matrix path (m > 128): block one-sided Jacobi over many workgroups.
//
// The K rows of R (zero-padded to Kp, a multiple of 2B) are split into nb
// blocks of B rows in a global buffer.  A sweep is a round-robin tournament
// over the blocks (nb - 1 block rounds); in each block round workgroup g
// takes block pair g, copies its 2B rows to LDS, rotates them (B parallel
// pairs per round, TPP lanes per pair) and writes them back: a full inner
// sweep over the 2B rows (2B - 1 rounds) in the first block round, which
// pairs every block once, and only the B x B cross pairs (B rounds) in the
// others, so every pair of rows meets at least once per sweep in about
// K + B rounds.  Block rounds are separated by a grid barrier of the
// cooperative launch; a sweep in which no rotation had a relative
// off-diagonal above 1e-9 is the last one (quadratic convergence).  NT
// threads per workgroup: 1024 (B = 16 or 32, one wave or half a wave per
// pair) where the 2B rows fit in LDS, else 256.
// ----------------------------------------------------------------------------
constexpr int kBlockThreads = 256;
constexpr int kBlockThreadsWide = 1024;
constexpr size_t kBlockWideLds = 144 * 1024;
constexpr int kBlockMaxE = 16;  // elements per lane and vector

struct BlockCtl {
    int big[kMaxSweeps];  // per sweep: workgroups that made a large rotation
    int sweeps;           // sweeps performed
    unsigned count, gen;  // grid barrier: arrivals, completed barriers
};

// Zeroes the control block before a launch (an ordinary kernel, so the
// sequence can be captured in a graph).
__global__ void svd_block_ctl_zero(BlockCtl *ctl) {
    int *p = reinterpret_cast<int *>(ctl);
    for (int i = threadIdx.x; i < (int)(sizeof(BlockCtl) / sizeof(int)); i += blockDim.x) p[i] = 0;
}

// Grid barrier of the cooperative launch: one agent-scope atomic per
// workgroup, the last arrival advances the generation.  The wait is bounded
// (20 s of the 100 MHz wall clock; the grid is co-resident by construction,
// so the bound only guarantees that the launch ends).
__device__ __forceinline__ void svd_grid_sync(BlockCtl *ctl, unsigned &gen) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned target = gen + 1;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned prev =
            __hip_atomic_fetch_add(&ctl->count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (prev == gridDim.x - 1) {
            __hip_atomic_store(&ctl->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctl->gen, target, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            const uint64_t t0 = wall_clock64();
            while (__hip_atomic_load(&ctl->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != target) {
                if (wall_clock64() - t0 > 20ull * 100000000ull) break;
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        gen = target;
    }
    __syncthreads();
}

template <int B, int NT>
__global__ __launch_bounds__(NT) void svd_block_kernel(
    const double *__restrict__ R, int64_t ldr, int K, int m, int mp, int nb,
    double *__restrict__ A, BlockCtl *ctl) {
    unsigned gen = 0;  // barriers passed (thread 0)
    constexpr int TPP = NT / B;  // lanes per pair
    static_assert(TPP <= kWave && (TPP & (TPP - 1)) == 0, "pair lanes inside one wave");
    extern __shared__ __attribute__((aligned(16))) double S[];  // 2B rows of mp
    const int tid = threadIdx.x;
    const int kp = nb * B;
    const int ne = mp / TPP;  // elements per lane (even, <= kBlockMaxE)

    // rows of R -> A (zero padding beyond K rows and m columns)
    for (int64_t idx = (int64_t)blockIdx.x * NT + tid; idx < (int64_t)kp * mp;
         idx += (int64_t)gridDim.x * NT) {
        const int vv = (int)(idx / mp), e = (int)(idx % mp);
        A[idx] = (vv < K && e < m) ? R[vv + ldr * e] : 0.0;
    }
    // One counter per sweep (zeroed before the launch) and never reused, so
    // every workgroup reads the same final count for its decision.
    svd_grid_sync(ctl, gen);

    const int pi = tid / TPP;
    const int sub = tid % TPP;
    const double thr = 4.0 * (double)m * 0x1p-52;
    const double thr2 = thr * thr;
    __shared__ int big_wg;

    int sweep = 0;
    for (; sweep < kMaxSweeps; ++sweep) {
        if (tid == 0) big_wg = 0;
        bool big = false;
        for (int br = 0; br < nb - 1; ++br) {
            int bp, bq;
            pair_of(br, blockIdx.x, nb, bp, bq);
            for (int idx = tid; idx < B * mp; idx += NT) {
                const int vv = idx / mp, e = idx % mp;
                S[vv * mp + e] = A[(int64_t)(bp * B + vv) * mp + e];
                S[(B + vv) * mp + e] = A[(int64_t)(bq * B + vv) * mp + e];
            }
            __syncthreads();
            // The first block round pairs every block once: a full sweep over
            // its 2B rows also covers the pairs inside each block.  Later
            // block rounds rotate only the B x B cross pairs (row pi of block
            // bp with row (pi + round) mod B of block bq), so a sweep takes
            // about K + B rounds instead of 2K.
            const int nrounds = (br == 0) ? 2 * B - 1 : B;
            for (int round = 0; round < nrounds; ++round) {
                int p, q;
                if (br == 0) {
                    pair_of(round, pi, 2 * B, p, q);
                } else {
                    p = pi;
                    q = B + (pi + round) % B;
                }
                double *ap = S + p * mp + 2 * sub;
                double *aq = S + q * mp + 2 * sub;
                double x[kBlockMaxE], y[kBlockMaxE];
                double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
                for (int e = 0; e < kBlockMaxE; ++e) {
                    if (e < ne) {
                        x[e] = ap[2 * TPP * (e / 2) + (e & 1)];
                        y[e] = aq[2 * TPP * (e / 2) + (e & 1)];
                        al = fma(x[e], x[e], al);
                        be = fma(y[e], y[e], be);
                        ga = fma(x[e], y[e], ga);
                    }
                }
                al = group_sum<TPP>(al);
                be = group_sum<TPP>(be);
                ga = group_sum<TPP>(ga);
                const double g2a = ga * ga;
                if (g2a > thr2 * al * be && al > kTinyNorm2 && be > kTinyNorm2) {
                    const double dlt = be - al;
                    const double g2 = ga + ga;
                    const double h = fma(dlt, dlt, g2 * g2);
                    const double den = fabs(dlt) + h * rsqrt_nr(h);
                    const double t = (dlt < 0.0 ? -g2 : g2) * rcp_nr(den);
                    const double c = rsqrt_nr(fma(t, t, 1.0));
                    const double s = c * t;
                    big |= g2a > kBigRel2 * al * be;
#pragma unroll
                    for (int e = 0; e < kBlockMaxE; ++e) {
                        if (e < ne) {
                            ap[2 * TPP * (e / 2) + (e & 1)] = fma(c, x[e], -s * y[e]);
                            aq[2 * TPP * (e / 2) + (e & 1)] = fma(s, x[e], c * y[e]);
                        }
                    }
                }
                __syncthreads();
            }
            for (int idx = tid; idx < B * mp; idx += NT) {
                const int vv = idx / mp, e = idx % mp;
                A[(int64_t)(bp * B + vv) * mp + e] = S[vv * mp + e];
                A[(int64_t)(bq * B + vv) * mp + e] = S[(B + vv) * mp + e];
            }
            svd_grid_sync(ctl, gen);
        }
        if (big) big_wg = 1;
        __syncthreads();
        if (tid == 0 && big_wg) atomicAdd(&ctl->big[sweep], 1);
        svd_grid_sync(ctl, gen);
        const int nbig = __atomic_load_n(&ctl->big[sweep], __ATOMIC_RELAXED);
        if (nbig == 0) {
            ++sweep;
            break;
        }
        __syncthreads();
    }
    if (blockIdx.x == 0 && tid == 0) ctl->sweeps = sweep;
}

// Singular values, truncation and core of the rotated rows A (kp x mp).
__global__ __launch_bounds__(1024) void svd_block_finish_kernel(
    const double *__restrict__ A, int K, int m, int mp, const BlockCtl *ctl,
    double *__restrict__ sigma_out, double *__restrict__ core_out, int64_t r_max, double tol,
    int dm1, int first, StepState *st, StepState *st0) {
    extern __shared__ double smem[];
    double *sig = smem;
    int *order = (int *)(sig + K);
    svd_epilogue(A, mp, K, m, sig, order, sigma_out, core_out, r_max, tol, dm1, first,
                       ctl->sweeps, st, st0);
}

namespace {

// Block shape of the large-matrix path: B rows per block with 2 B rows of
// mp (m rounded up to 2 TPP) in LDS, TPP = nt / B: 1024 threads with
// B = 32 or 16 in at most 144 KiB where that fits, else 256 threads in at
// most 64 KiB.
struct BlockShape {
    int B, tpp, mp, nb, kp, nt;
};
BlockShape block_shape(int64_t K, int64_t m) {
    BlockShape b{32, 0, 0, 0, 0, kBlockThreadsWide};
    for (int B : {32, 16}) {
        b.B = B;
        b.tpp = kBlockThreadsWide / B;
        b.mp = (int)ceil_div(m, 2 * b.tpp) * 2 * b.tpp;
        if ((size_t)2 * B * b.mp * 8 <= kBlockWideLds && b.mp / b.tpp <= kBlockMaxE) {
            b.nb = (int)ceil_div(K, 2 * b.B) * 2;
            b.kp = b.nb * b.B;
            return b;
        }
    }
    b.B = 32;
    b.nt = kBlockThreads;
    for (;;) {
        b.tpp = kBlockThreads / b.B;
        b.mp = (int)ceil_div(m, 2 * b.tpp) * 2 * b.tpp;
        if ((int64_t)2 * b.B * b.mp * 8 <= 64 * 1024 || b.B == 4) break;
        b.B /= 2;
    }
    b.nb = (int)ceil_div(K, 2 * b.B) * 2;
    b.kp = b.nb * b.B;
    return b;
}
}  // namespace

size_t svd_scratch_bytes(int64_t K, int64_t m) {
    if (m <= 128) return 0;
    const BlockShape b = block_shape(K, m);
    return (size_t)b.kp * b.mp * sizeof(double) + sizeof(BlockCtl) + 256;
}

// Lanes per Jacobi pair of the small-matrix kernel (TTSVD_SVD_LPP = 8 or 16,
// a tuning override; default 8).
int svd_lpp() {
    static int v = [] {
        const char *e = getenv("TTSVD_SVD_LPP");
        return (e && atoi(e) == 16) ? 16 : 8;
    }();
    return v;
}

int svd_launch(const double *R, int64_t ldr, int64_t K, int64_t m, double *sigma_out,
               double *core_out, int64_t r_max, double tol, int dm1, int first,
               StepState *state, StepState *state0, void *scratch, size_t scratch_bytes,
               hipStream_t s) {
    if (K < 1 || m < 1 || K > m || m > 4096)
        return set_error(TTSVD_EINVAL, "svd: bad shape K=%lld m=%lld", (long long)K, (long long)m);
    if (scratch_bytes < svd_scratch_bytes(K, m))
        return set_error(TTSVD_EINVAL, "svd: scratch %zu < %zu bytes", scratch_bytes,
                         svd_scratch_bytes(K, m));
    if (m <= 128) {
        const int MB = m <= 16 ? 16 : m <= 32 ? 32 : m <= 64 ? 64 : 128;
        const int lpp = MB == 16 ? 8 : MB == 128 ? 4 : svd_lpp();
        char name[64];
        snprintf(name, sizeof(name), "svd_small_kernel<%d, %d>", MB, lpp);
        prof_begin(s, name, (double)(m * m) * 8.0 + (double)(K * m) * 8.0, 0.0);
#define TTSVD_SVD_SMALL(MM, LL)                                                                \
    hipLaunchKernelGGL((svd_small_kernel<MM, LL>), dim3(1), dim3(MM / 2 * LL), 0, s, R, ldr,   \
                       (int)K, (int)m, sigma_out, core_out, r_max, tol, dm1, first, state, state0)
        if (MB == 16)
            TTSVD_SVD_SMALL(16, 8);
        else if (MB == 32 && lpp == 16)
            TTSVD_SVD_SMALL(32, 16);
        else if (MB == 32)
            TTSVD_SVD_SMALL(32, 8);
        else if (MB == 64 && lpp == 16)
            TTSVD_SVD_SMALL(64, 16);
        else if (MB == 64)
            TTSVD_SVD_SMALL(64, 8);
        else
            TTSVD_SVD_SMALL(128, 4);
#undef TTSVD_SVD_SMALL
        prof_end(s);
        TTSVD_HIP_TRY(hipGetLastError());
        return TTSVD_OK;
    }
    if (m > 1024)
        return set_error(TTSVD_EUNSUPPORTED, "svd: m = %lld > 1024", (long long)m);
    const BlockShape b = block_shape(K, m);
    if (b.mp / b.tpp > kBlockMaxE)
        return set_error(TTSVD_EUNSUPPORTED, "svd: block shape for m = %lld", (long long)m);
    double *A = (double *)scratch;
    BlockCtl *ctl = (BlockCtl *)(A + (size_t)b.kp * b.mp);
    char name[64];
    snprintf(name, sizeof(name), "svd_block_kernel<%d, %d>", b.B, b.nt);
    prof_begin(s, name, (double)(m * m) * 8.0 + (double)(K * m) * 8.0, 0.0);
    const size_t lds = (size_t)2 * b.B * b.mp * sizeof(double);
    int nbk = b.nb / 2;
    void *args[] = {(void *)&R, (void *)&ldr, (void *)&K, (void *)&m, (void *)&b.mp,
                    (void *)&b.nb, (void *)&A, (void *)&ctl};
    int Ki = (int)K, mi = (int)m, mpi = b.mp, nbi = b.nb;
    args[2] = &Ki;
    args[3] = &mi;
    args[4] = &mpi;
    args[5] = &nbi;
    const void *fn;
    if (b.nt == kBlockThreadsWide)
        fn = b.B == 32 ? (const void *)svd_block_kernel<32, kBlockThreadsWide>
                       : (const void *)svd_block_kernel<16, kBlockThreadsWide>;
    else
        fn = b.B == 32   ? (const void *)svd_block_kernel<32, kBlockThreads>
             : b.B == 16 ? (const void *)svd_block_kernel<16, kBlockThreads>
             : b.B == 8  ? (const void *)svd_block_kernel<8, kBlockThreads>
                         : (const void *)svd_block_kernel<4, kBlockThreads>;
    hipLaunchKernelGGL(svd_block_ctl_zero, dim3(1), dim3(64), 0, s, ctl);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && lds > 64 * 1024)
        e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess) e = coop_launch(fn, dim3(nbk), dim3(b.nt), args, lds, s);
    prof_end(s);
    if (e != hipSuccess)
        return set_error(TTSVD_EHIP, "svd: cooperative launch: %s", hipGetErrorString(e));
    prof_begin(s, "svd_block_finish_kernel", (double)(K * m) * 8.0, 0.0);
    hipLaunchKernelGGL(svd_block_finish_kernel, dim3(1), dim3(1024), (size_t)K * 12 + 16, s, A,
                       (int)K, (int)m, b.mp, ctl, sigma_out, core_out, r_max, tol, dm1, first,
                       state, state0);
    prof_end(s);
    TTSVD_HIP_TRY(hipGetLastError());
    return TTSVD_OK;
}

}  // namespace ttsvd
