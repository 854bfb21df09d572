// Small SVD of the triangular factor, truncation and core emission: the
// "calculate small SVD", "choose rank" and "T^(i) <- reshape(V^T)" steps of
// Algorithm 2 of arXiv 2102.00104, in FP64, in one workgroup.
//
// SVD: one-sided Jacobi (Hestenes) applied to the K rows of R, i.e. to the
// columns of A = R^T (K vectors of length m).  Plane rotations of pairs of
// rows make them mutually orthogonal; then R = J diag(sigma) V^T with the
// rotated rows b_k = sigma_k V_{:,k}, so sigma_k = ||b_k|| and the right
// singular vectors are the normalised rotated rows -- no separate V has to
// be accumulated.  Pairs are visited in round-robin (tournament) order so that
// the K/2 rotations of one round are independent and run in parallel, one
// group of lanes per pair.
//
// Truncation: delta^2 = tol^2/(d-1) ||Sigma||_F^2 in the first step; the rank
// is min(r_max, r_delta) with r_delta the smallest j such that
// sigma_{j+1}^2 + ... <= delta^2 (tails summed from the smallest value),
// clamped to [1, K]; tol = 0 means r = min(r_max, K).  Singular values below
// kSigmaFloor are counted as zero in these sums: they are the ~1e-154
// diagonal entries the eps_FP safeguard of the Householder step leaves for
// exactly zero columns, not data.
#include <stdio.h>
#include <stdlib.h>

#include <cmath>

#include <hip/hip_cooperative_groups.h>

#include "common.h"
#include "kernels.h"
#include "profile.h"

namespace ttsvd {

constexpr double kSigmaFloor = 1e-150;
constexpr int kMaxSweeps = 40;

__device__ inline void pair_of(int round, int i, int kp, int &p, int &q) {
    const int n1 = kp - 1;
    if (i == 0) {
        p = 0;
        q = 1 + round % n1;
    } else {
        p = 1 + (round + i) % n1;
        q = 1 + (round - i + n1) % n1;
    }
}

// Singular values, their descending order, the truncation rule and the core
// T[a + r c] = b_{order[a]}[c] / sigma_{order[a]} from the K rotated rows
// A[v * lda + e] (v < K, e < m).  sig and order are K-entry shared arrays.
template <int NT, typename ARef>
__device__ void svd_epilogue(ARef A, int lda, int K, int m, double *sig, int *order,
                             double *__restrict__ sigma_out, double *__restrict__ core_out,
                             int64_t r_max, double tol, int dm1, int first, int sweep,
                             StepState *st, StepState *st0) {
    const int tid = threadIdx.x;
    // Singular values and their descending order (stable rank sort).
    for (int v = tid; v < K; v += NT) {
        const double *av = A + (int64_t)v * lda;
        double s2 = 0.0;
        for (int e = 0; e < m; ++e) s2 = fma(av[e], av[e], s2);
        sig[v] = std::sqrt(s2);
    }
    __syncthreads();
    // NaN keys sort last (as -1), so the ranks always form a permutation.
    for (int v = tid; v < K; v += NT) {
        const double sv = isnan(sig[v]) ? -1.0 : sig[v];
        int pos = 0;
        for (int u = 0; u < K; ++u) {
            const double su = isnan(sig[u]) ? -1.0 : sig[u];
            pos += (su > sv) || (su == sv && u < v);
        }
        order[pos] = v;
    }
    __syncthreads();

    __shared__ int64_t rank_sh;
    if (tid == 0) {
        int nonfinite = 0;
        double norm2 = 0.0;
        for (int i = K - 1; i >= 0; --i) {
            const double s = sig[order[i]];
            if (!isfinite(s)) nonfinite = 1;
            const double se = s > kSigmaFloor ? s : 0.0;
            norm2 = fma(se, se, norm2);
        }
        if (first) {
            st0->norm2 = norm2;
            st0->delta2 = (tol * tol / (double)dm1) * norm2;
        }
        const double delta2 = st0->delta2;
        int64_t r;
        if (tol == 0.0) {
            r = min<int64_t>(r_max, K);
        } else {
            int64_t r_delta = K;
            double acc = 0.0;
            for (int i = K - 1; i >= 0; --i) {
                const double s = sig[order[i]];
                const double se = s > kSigmaFloor ? s : 0.0;
                acc = fma(se, se, acc);
                if (acc <= delta2)
                    r_delta = i;
                else
                    break;
            }
            r = max<int64_t>(1, min<int64_t>(min<int64_t>(r_max, r_delta), K));
        }
        double disc = 0.0;
        for (int i = K - 1; i >= (int)r; --i) {
            const double s = sig[order[i]];
            const double se = s > kSigmaFloor ? s : 0.0;
            disc = fma(se, se, disc);
        }
        st->rank = r;
        st->discarded2 = disc;
        st->sweeps = sweep;
        st->nonfinite = nonfinite;
        rank_sh = r;
    }
    __syncthreads();
    const int64_t r = rank_sh;
    for (int i = tid; i < K; i += NT) sigma_out[i] = sig[order[i]];
    for (int64_t idx = tid; idx < r * m; idx += NT) {
        const int a = (int)(idx % r), c = (int)(idx / r);
        const int v = order[a];
        core_out[idx] = A[(int64_t)v * lda + c] / sig[v];
    }
}


// Rows whose squared norm is below this are left alone by the rotations
// (eps_FP artefacts of exactly zero columns have squared norms ~1e-308).
constexpr double kTinyNorm2 = 1e-280;
// Squared relative off-diagonal above which a sweep is not yet the last.
constexpr double kBigRel2 = 1e-18;

// Small-matrix path, K <= m <= MB <= 64: the rows live in LDS, LPP lanes
// work on one pair (LPP lanes), dot products are reduced with DPP inside the
// group, one barrier per round.  Lane `sub` of a group handles the 16-byte
// chunks at elements 2 LPP c + 2 sub, so each LDS instruction of a group
// touches contiguous bytes (no bank conflicts inside the group).
template <int MB, int LPP>
__global__ __launch_bounds__(MB / 2 * LPP) void svd_small_kernel(
    const double *__restrict__ R, int64_t ldr, int K, int m, double *__restrict__ sigma_out,
    double *__restrict__ core_out, int64_t r_max, double tol, int dm1, int first,
    StepState *st, StepState *st0) {
    constexpr int NT = MB / 2 * LPP;
    constexpr int E = MB / LPP;     // elements per lane (E / 2 chunks of two)
    constexpr int CS = 2 * LPP;     // elements per chunk row of a group
    static_assert(E % 2 == 0, "two elements per chunk");
    constexpr int LDA = MB + 2;     // row stride (keeps 16-byte alignment)
    __shared__ __attribute__((aligned(16))) double A[MB * LDA];
    __shared__ double sig[MB];
    __shared__ int order[MB];
    __shared__ int rot_count;
    const int tid = threadIdx.x;
    const int kp = K + (K & 1);
    const int n1 = kp - 1;

    for (int idx = tid; idx < MB * MB; idx += NT) {
        const int vv = idx / MB, e = idx % MB;
        A[vv * LDA + e] = (vv < K && e < m) ? R[vv + ldr * e] : 0.0;
    }
    __syncthreads();

    const int pi = tid / LPP;       // pair handled by this group
    const int sub = tid % LPP;
    const bool active = pi < kp / 2;
    const double thr = 4.0 * (double)m * 0x1p-52;
    const double thr2 = thr * thr;

    int sweep = 0;
    for (; sweep < kMaxSweeps; ++sweep) {
        if (tid == 0) rot_count = 0;
        __syncthreads();
        int local = 0;
        bool big = false;
        for (int round = 0; round < n1; ++round) {
            if (active) {
                int p, q;
                if (pi == 0) {
                    p = 0;
                    q = 1 + round;
                } else {
                    int x = round + pi;
                    x = x >= n1 ? x - n1 : x;
                    int y = round - pi;
                    y = y < 0 ? y + n1 : y;
                    p = 1 + x;
                    q = 1 + y;
                }
                double *ap = A + p * LDA + 2 * sub;
                double *aq = A + q * LDA + 2 * sub;
                double x[E], y[E];
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    x[e] = ap[CS * (e / 2) + (e & 1)];
                    y[e] = aq[CS * (e / 2) + (e & 1)];
                }
                double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    al = fma(x[e], x[e], al);
                    be = fma(y[e], y[e], be);
                    ga = fma(x[e], y[e], ga);
                }
                al = group_sum<LPP>(al);
                be = group_sum<LPP>(be);
                ga = group_sum<LPP>(ga);
                const double g2a = ga * ga;
                if (g2a > thr2 * al * be && al > kTinyNorm2 && be > kTinyNorm2) {
                    // rotation zeroing the (p, q) entry of [a_p a_q]^T [a_p a_q]:
                    // t = 2 ga sign(be - al) / (|be - al| + sqrt((be - al)^2 + 4 ga^2)),
                    // sign(0) = +1: the smaller root of t^2 + 2 zeta t - 1 = 0,
                    // zeta = (be - al) / (2 ga), written without dividing by ga.
                    const double dlt = be - al;
                    const double g2 = ga + ga;
                    const double h = fma(dlt, dlt, g2 * g2);
                    const double den = fabs(dlt) + h * rsqrt_nr(h);
                    const double t = (dlt < 0.0 ? -g2 : g2) * rcp_nr(den);
                    const double c = rsqrt_nr(fma(t, t, 1.0));
                    const double s = c * t;
                    big |= g2a > kBigRel2 * al * be;
#pragma unroll
                    for (int e = 0; e < E; ++e) {
                        ap[CS * (e / 2) + (e & 1)] = fma(c, x[e], -s * y[e]);
                        aq[CS * (e / 2) + (e & 1)] = fma(s, x[e], c * y[e]);
                    }
                    local += (sub == 0);
                }
            }
            __syncthreads();
        }
        // rot_count: groups that rotated this sweep (low 16 bits) and groups
        // that rotated a pair with relative off-diagonal above 1e-9 (high
        // bits).  Jacobi converges quadratically, so a sweep whose rotations
        // were all below 1e-9 leaves off-diagonals at the 1e-18 level and
        // needs no checking sweep.
        const int contrib = (local ? 1 : 0) + (big ? (1 << 16) : 0);
        if (contrib && sub == 0) atomicAdd(&rot_count, contrib);
        __syncthreads();
        const int rc = rot_count;
        __syncthreads();
        if (rc == 0) break;
        if ((rc >> 16) == 0) {
            ++sweep;
            break;
        }
    }
    svd_epilogue<NT>(A, LDA, K, m, sig, order, sigma_out, core_out, r_max, tol, dm1, first, sweep,
                     st, st0);
}

// ----------------------------------------------------------------------------
// Large-matrix path (m > 64): block one-sided Jacobi over many workgroups.
//
// The K rows of R (zero-padded to Kp, a multiple of 2B) are split into nb
// blocks of B rows in a global buffer.  A sweep is a round-robin tournament
// over the blocks (nb - 1 block rounds); in each block round workgroup g
// takes block pair g, copies its 2B rows to LDS, runs one full inner Jacobi
// sweep over them (2B - 1 rounds of B parallel pairs, TPP lanes per pair)
// and writes them back.  Block rounds are separated by a grid barrier of the
// cooperative launch; a sweep in which no rotation had a relative
// off-diagonal above 1e-9 is the last one (quadratic convergence).
// ----------------------------------------------------------------------------
constexpr int kBlockThreads = 256;
constexpr int kBlockMaxE = 16;  // elements per lane and vector

struct BlockCtl {
    int big[kMaxSweeps];  // per sweep: workgroups that made a large rotation
    int sweeps;           // sweeps performed
};

template <int B>
__global__ __launch_bounds__(kBlockThreads) void svd_block_kernel(
    const double *__restrict__ R, int64_t ldr, int K, int m, int mp, int nb,
    double *__restrict__ A, BlockCtl *ctl) {
    namespace cg = cooperative_groups;
    cg::grid_group grid = cg::this_grid();
    constexpr int TPP = kBlockThreads / B;  // lanes per pair
    extern __shared__ __attribute__((aligned(16))) double S[];  // 2B rows of mp
    const int tid = threadIdx.x;
    const int kp = nb * B;
    const int ne = mp / TPP;  // elements per lane (even, <= kBlockMaxE)

    // rows of R -> A (zero padding beyond K rows and m columns)
    for (int64_t idx = (int64_t)blockIdx.x * kBlockThreads + tid; idx < (int64_t)kp * mp;
         idx += (int64_t)gridDim.x * kBlockThreads) {
        const int vv = (int)(idx / mp), e = (int)(idx % mp);
        A[idx] = (vv < K && e < m) ? R[vv + ldr * e] : 0.0;
    }
    // One counter per sweep, zeroed before the first grid barrier and never
    // reused, so every workgroup reads the same final count for its decision.
    if (blockIdx.x == 0 && tid < kMaxSweeps) ctl->big[tid] = 0;
    grid.sync();

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
            for (int idx = tid; idx < B * mp; idx += kBlockThreads) {
                const int vv = idx / mp, e = idx % mp;
                S[vv * mp + e] = A[(int64_t)(bp * B + vv) * mp + e];
                S[(B + vv) * mp + e] = A[(int64_t)(bq * B + vv) * mp + e];
            }
            __syncthreads();
            for (int round = 0; round < 2 * B - 1; ++round) {
                int p, q;
                pair_of(round, pi, 2 * B, p, q);
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
            for (int idx = tid; idx < B * mp; idx += kBlockThreads) {
                const int vv = idx / mp, e = idx % mp;
                A[(int64_t)(bp * B + vv) * mp + e] = S[vv * mp + e];
                A[(int64_t)(bq * B + vv) * mp + e] = S[(B + vv) * mp + e];
            }
            grid.sync();
        }
        if (big) big_wg = 1;
        __syncthreads();
        if (tid == 0 && big_wg) atomicAdd(&ctl->big[sweep], 1);
        grid.sync();
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
    svd_epilogue<1024>(A, mp, K, m, sig, order, sigma_out, core_out, r_max, tol, dm1, first,
                       ctl->sweeps, st, st0);
}

namespace {

// Block shape of the large-matrix path: B rows per block with 2 B rows of
// mp (m rounded up to 2 TPP) in at most 64 KiB of LDS, TPP = 256 / B.
struct BlockShape {
    int B, tpp, mp, nb, kp;
};
BlockShape block_shape(int64_t K, int64_t m) {
    BlockShape b{32, 0, 0, 0, 0};
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
    if (m <= 64) return 0;
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
               StepState *state, StepState *state0, void *scratch, hipStream_t s) {
    if (K < 1 || m < 1 || K > m || m > 4096)
        return set_error(TTSVD_EINVAL, "svd: bad shape K=%lld m=%lld", (long long)K, (long long)m);
    if (m <= 64) {
        const int MB = m <= 16 ? 16 : m <= 32 ? 32 : 64;
        const int lpp = MB == 16 ? 8 : svd_lpp();
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
        else if (lpp == 16)
            TTSVD_SVD_SMALL(64, 16);
        else
            TTSVD_SVD_SMALL(64, 8);
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
    snprintf(name, sizeof(name), "svd_block_kernel<%d>", b.B);
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
    hipError_t e;
    switch (b.B) {
        case 32: e = hipLaunchCooperativeKernel((const void *)svd_block_kernel<32>, dim3(nbk), dim3(kBlockThreads), args, lds, s); break;
        case 16: e = hipLaunchCooperativeKernel((const void *)svd_block_kernel<16>, dim3(nbk), dim3(kBlockThreads), args, lds, s); break;
        case 8: e = hipLaunchCooperativeKernel((const void *)svd_block_kernel<8>, dim3(nbk), dim3(kBlockThreads), args, lds, s); break;
        default: e = hipLaunchCooperativeKernel((const void *)svd_block_kernel<4>, dim3(nbk), dim3(kBlockThreads), args, lds, s); break;
    }
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
