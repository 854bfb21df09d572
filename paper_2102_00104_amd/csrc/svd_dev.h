// Device bodies of the small SVD of the triangular factor, the truncation
// rule and the core emission (the "calculate small SVD", "choose rank" and
// "T^(i) <- reshape(V^T)" steps of Algorithm 2 of arXiv 2102.00104), shared
// by the single-tensor kernels and the batched persistent kernel.
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
#pragma once

#include <cmath>

#include "common.h"
#include "kernels.h"

namespace ttsvd {

constexpr double kSigmaFloor = 1e-150;
constexpr int kMaxSweeps = 40;

// Rows whose squared norm is below this are left alone by the rotations
// (eps_FP artefacts of exactly zero columns have squared norms ~1e-308).
constexpr double kTinyNorm2 = 1e-280;
// Squared relative off-diagonal above which a sweep is not yet the last.
constexpr double kBigRel2 = 1e-18;

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
// Every thread of the workgroup takes part.
template <typename ARef>
__device__ void svd_epilogue(ARef A, int lda, int K, int m, double *sig, int *order,
                             double *__restrict__ sigma_out, double *__restrict__ core_out,
                             int64_t r_max, double tol, int dm1, int first, int sweep,
                             StepState *st, StepState *st0) {
    const int tid = thread_id();
    const int nth = blockDim.x;
    // Singular values and their descending order (stable rank sort).
    for (int v = tid; v < K; v += nth) {
        const double *av = A + (int64_t)v * lda;
        double s2 = 0.0;
        for (int e = 0; e < m; ++e) s2 = fma(av[e], av[e], s2);
        sig[v] = std::sqrt(s2);
    }
    __syncthreads();
    // NaN keys sort last (as -1), so the ranks always form a permutation.
    for (int v = tid; v < K; v += nth) {
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
    for (int i = tid; i < K; i += nth) sigma_out[i] = sig[order[i]];
    for (int64_t idx = tid; idx < r * m; idx += nth) {
        const int a = (int)(idx % r), c = (int)(idx / r);
        const int v = order[a];
        // an exactly zero row (possible only for an unfolding passed without
        // its QR) has no direction: its core row is zero
        const double sv = sig[v];
        core_out[idx] = sv > 0.0 ? A[(int64_t)v * lda + c] / sv : 0.0;
    }
    // the caller may reuse sig / order / A after this point
    __syncthreads();
}

// Small-matrix path, K <= m <= MB <= 128, one workgroup.  LPP lanes work on
// one pair of rows ("slot"); lane `sub` of a slot holds the 16-byte chunks at
// elements 2 LPP c + 2 sub of both rows in registers (E elements each), dot
// products are reduced with DPP inside the slot.
//
// Ordering (recursive halving; every pair once per sweep, P - 1 rounds for
// P = K rounded up to a power of two, zero rows beyond K): at level L the
// rows form blocks of 2h rows, h = P / 2^(L+1); slot i (block i / h, local
// index li = i mod h) pairs row A = block*2h + li with row
// B = block*2h + h + (li + r) mod h in round r = 0..h-1.  Each slot keeps its
// A row in registers for the whole level; only the B rows move, one slot
// down per round, through their rows in LDS -- half the LDS traffic of an
// ordering that moves both rows -- and when a block lies inside one wave the
// round needs only a wave-level fence instead of a workgroup barrier.  At the
// end of a level every row goes back to LDS and the next level regroups.
// The first (P/2) * LPP threads compute; any further threads only join the
// barriers.
template <int MB, int LPP>
struct SvdSmall {
    static constexpr int NT = MB / 2 * LPP;  // computing threads (P = MB)
    static constexpr int E = MB / LPP;       // elements per lane (E / 2 chunks of two)
    static constexpr int CS = 2 * LPP;       // elements per chunk row of a group
    // Row stride in doubles: the smallest >= MB with LDA = 2 LPP (mod 32).  A
    // 16-lane pass of a 16-byte LDS access covers 16 / LPP slots of LPP lanes
    // (16 LPP bytes each) on consecutive rows; rows 16 LPP bytes apart modulo
    // the 256 bytes of the 64 banks put those slots on disjoint banks.  (Even,
    // so rows stay 16-byte aligned.)
    static constexpr int lda() {
        int l = MB;
        while (l % 32 != (2 * LPP) % 32) ++l;
        return l;
    }
    static constexpr int LDA = lda();
    static constexpr int SPW = kWave / LPP;  // slots per wave
    static_assert(E % 2 == 0, "two elements per chunk");
    static constexpr size_t smem_bytes() {
        return sizeof(double) * (MB * LDA + MB) + sizeof(int) * (MB + 4);
    }
};

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int MB, int LPP>
__device__ __forceinline__ void svd_small_body(
    const double *__restrict__ R, int64_t ldr, int K, int m, double *__restrict__ sigma_out,
    double *__restrict__ core_out, int64_t r_max, double tol, int dm1, int first,
    StepState *st, StepState *st0, void *smem) {
    using C = SvdSmall<MB, LPP>;
    constexpr int E = C::E, CS = C::CS, LDA = C::LDA, SPW = C::SPW;
    double *A = reinterpret_cast<double *>(smem);
    double *sig = A + MB * LDA;
    int *order = reinterpret_cast<int *>(sig + MB);
    int *rot_count = order + MB;
    const int tid = thread_id();
    const int nth = blockDim.x;
    int P = 1;
    while (P < K) P <<= 1;  // rows K..P-1 are zero

    for (int idx = tid; idx < MB * MB; idx += nth) {
        const int vv = idx / MB, e = idx % MB;
        A[vv * LDA + e] = (vv < K && e < m) ? R[vv + ldr * e] : 0.0;
    }
    __syncthreads();

    const int slot = tid / LPP;
    const int sub = tid % LPP;
    const bool active = slot < P / 2;
    const double thr = 4.0 * (double)m * 0x1p-52;
    const double thr2 = thr * thr;

    auto load = [&](int row, double (&v)[E]) {
        const double *p = A + row * LDA + 2 * sub;
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = p[CS * (e / 2) + (e & 1)];
    };
    auto store = [&](int row, const double (&v)[E]) {
        double *p = A + row * LDA + 2 * sub;
#pragma unroll
        for (int e = 0; e < E; ++e) p[CS * (e / 2) + (e & 1)] = v[e];
    };

    int sweep = 0;
    for (; sweep < kMaxSweeps; ++sweep) {
        if (tid == 0) *rot_count = 0;
        __syncthreads();
        int local = 0;
        bool big = false;
        for (int h = P >> 1; h >= 1; h >>= 1) {
            // h is a power of two: shifts and masks, no integer division
            const int lh = __builtin_ctz(h);
            const int blk = slot >> lh, li = slot & (h - 1);
            const int ra = blk * 2 * h + li;
            const int rb0 = blk * 2 * h + h;
            const bool in_wave = h <= SPW;  // the B rows of a block never leave a wave
            double x[E], y[E];
            if (active) {
                load(ra, x);
                load(rb0 + li, y);
            }
            for (int r = 0; r < h; ++r) {
                if (active) {
                    // two interleaved accumulators halve the dependent FMA chains
                    double al0 = 0.0, be0 = 0.0, ga0 = 0.0, al1 = 0.0, be1 = 0.0, ga1 = 0.0;
#pragma unroll
                    for (int e = 0; e < E; e += 2) {
                        al0 = fma(x[e], x[e], al0);
                        be0 = fma(y[e], y[e], be0);
                        ga0 = fma(x[e], y[e], ga0);
                        al1 = fma(x[e + 1], x[e + 1], al1);
                        be1 = fma(y[e + 1], y[e + 1], be1);
                        ga1 = fma(x[e + 1], y[e + 1], ga1);
                    }
                    double al = group_sum<LPP>(al0 + al1);
                    double be = group_sum<LPP>(be0 + be1);
                    double ga = group_sum<LPP>(ga0 + ga1);
                    const double g2a = ga * ga;
                    if (g2a > thr2 * al * be && al > kTinyNorm2 && be > kTinyNorm2) {
                        // rotation zeroing the (A, B) entry of [a_A a_B]^T [a_A a_B]:
                        // t = 2 ga sign(be - al) / (|be - al| + sqrt((be - al)^2 + 4 ga^2)),
                        // sign(0) = +1: the smaller root of t^2 + 2 zeta t - 1 = 0,
                        // zeta = (be - al) / (2 ga), written without dividing by ga.
                        const double dlt = be - al;
                        const double g2 = ga + ga;
                        const double hh = fma(dlt, dlt, g2 * g2);
                        // (t only steers the iteration: one Newton step; c must make
                        // c^2 (1 + t^2) = 1 to working precision: two)
                        const double den = fabs(dlt) + hh * rsqrt_nr1(hh);
                        const double t = (dlt < 0.0 ? -g2 : g2) * rcp_nr1(den);
                        const double c = rsqrt_nr(fma(t, t, 1.0));
                        const double s = c * t;
                        big |= g2a > kBigRel2 * al * be;
#pragma unroll
                        for (int e = 0; e < E; ++e) {
                            const double xe = x[e];
                            x[e] = fma(c, xe, -s * y[e]);
                            y[e] = fma(s, xe, c * y[e]);
                        }
                        local += (sub == 0);
                    }
                    // B moves one slot down: write it back, then take the next one
                    store(rb0 + ((li + r) & (h - 1)), y);
                }
                if (r + 1 < h) {
                    if (in_wave)
                        wave_lds_sync();
                    else
                        __syncthreads();
                    // the row loaded here was stored this round by the slot
                    // above; the next round overwrites only this slot's own
                    // row, so no second barrier is needed
                    if (active) load(rb0 + ((li + r + 1) & (h - 1)), y);
                }
            }
            if (active) store(ra, x);
            __syncthreads();  // all rows in LDS before the next level regroups them
        }
        // rot_count: groups that rotated this sweep (low 16 bits) and groups
        // that rotated a pair with relative off-diagonal above 1e-9 (high
        // bits).  Jacobi converges quadratically, so a sweep whose rotations
        // were all below 1e-9 leaves off-diagonals at the 1e-18 level and
        // needs no checking sweep.
        const int contrib = (local ? 1 : 0) + (big ? (1 << 16) : 0);
        if (contrib && sub == 0) atomicAdd(rot_count, contrib);
        __syncthreads();
        const int rc = *rot_count;
        __syncthreads();
        if (rc == 0) break;
        if ((rc >> 16) == 0) {
            ++sweep;
            break;
        }
    }
    svd_epilogue(A, LDA, K, m, sig, order, sigma_out, core_out, r_max, tol, dm1, first, sweep,
                 st, st0);
}

}  // namespace ttsvd
