// Device bodies and reduction-tree planner of the rank-preserving Q-less
// TSQR (Sec. 3.2 of arXiv 2102.00104), shared by the per-level kernels of the
// single-tensor path and by the batched persistent kernel.
//
// Householder step (Algorithm 6): for column j, the reflector acts on the
// vector u = (R_jj ; M_{:,j}); with eps the smallest normalized number,
//   t = ||u||^2 + eps,  alpha = -sign(u_1) sqrt(t + eps),
//   t <- t - alpha u_1,  u_1 <- u_1 - alpha,  v = u / sqrt(t)   (||v||^2 = 2),
// R_jj <- alpha, and every trailing column x = (R_jk ; M_{:,k}) becomes
// x - (v^T x) v.  The eps terms keep the step free of branches and divisions
// by zero for zero columns.
//
// A body processes one "slice" (a contiguous range of rows) of W and writes
// the slice's triangular factor as m rows of the stacked output; the caller
// supplies the slice index and the LDS scratch.
#pragma once

#include "common.h"

namespace ttsvd {

// ----------------------------------------------------------------------------
// Row-owner wave body, m <= M <= 8: each of the WAVES waves of a workgroup
// reduces its own slice (slice = vblock * WAVES + wave).
//
// Lane l holds rows (tile_base + l + 64 i), i < RPT, of the current row tile
// and row l of the wave's triangular factor, all in registers.  Column dot
// products are reduced across the wave with wave_allreduce_vec.
// ----------------------------------------------------------------------------
constexpr int kRowsWaves = 4;  // waves (= slices) per workgroup

template <int M, int RPT, typename Tin, int WAVES = kRowsWaves>
constexpr size_t tsqr_rows_smem() {
    return sizeof(typename Elem<Tin>::acc) * WAVES * kWave;
}

// The body proper, with the row tile supplied by `load(base, r0, r1, a)`:
// a[i][c] = element (base + lane + 64 i, c) of the slice [r0, r1), zero for
// rows >= r1 and columns >= m.
template <int M, int RPT, typename T, int WAVES, typename Load>
__device__ __forceinline__ void tsqr_rows_core(
    int64_t rows, int m, int64_t rows_per_slice, int64_t nslices, double *__restrict__ out,
    int64_t ld_out, int64_t out_row0_stride, int kvalid, int64_t vblock, void *smem,
    Load load) {
    constexpr int CH = (M < 16) ? M : 16;  // trailing columns per reduction
    const int lane = lane_id();
    const int wid = thread_id() / kWave;
    const int64_t slice = vblock * WAVES + wid;
    if (slice >= nslices) return;  // uniform per wave
    const int64_t r0 = slice * rows_per_slice;
    const int64_t r1 = min(rows, r0 + rows_per_slice);
    T *lds = reinterpret_cast<T *>(smem) + wid * kWave;
    const T eps = EpsFP<T>::value();

    T R[M];
#pragma unroll
    for (int k = 0; k < M; ++k) R[k] = T(0);
    T a[RPT][M];

    for (int64_t base = r0; base < r1; base += (int64_t)kWave * RPT) {
        load(base, r0, r1, a);
#pragma unroll
        for (int j = 0; j < M; ++j) {
            if (j < m) {
            const bool own = (lane == j);
            T s = T(0);
#pragma unroll
            for (int i = 0; i < RPT; ++i) s = fma(a[i][j], a[i][j], s);
            const T rjj = own ? R[j] : T(0);
            s = fma(rjj, rjj, s);
            s = wave_sum(s);
            const T u1 = read_lane(R[j], j);
            T t = s + eps;
            T alpha = dev_sqrt(t + eps);
            alpha = (u1 > T(0)) ? -alpha : alpha;
            t = fma(-alpha, u1, t);
            const T beta = T(1) / dev_sqrt(t);
            T v[RPT];
#pragma unroll
            for (int i = 0; i < RPT; ++i) v[i] = beta * a[i][j];
            const T vr = own ? beta * (u1 - alpha) : T(0);
            if (own) R[j] = alpha;
#pragma unroll
            for (int kc = j + 1; kc < M; kc += CH) {
                if (kc < m) {
                T p[CH];
#pragma unroll
                for (int q = 0; q < CH; ++q) {
                    const int k = kc + q;
                    if (k < M) {
                        T acc = vr * R[k];
#pragma unroll
                        for (int i = 0; i < RPT; ++i) acc = fma(v[i], a[i][k], acc);
                        p[q] = acc;
                    } else {
                        p[q] = T(0);
                    }
                }
                wave_allreduce_vec<CH>(p, lds);
#pragma unroll
                for (int q = 0; q < CH; ++q) {
                    const int k = kc + q;
                    if (k < M) {
#pragma unroll
                        for (int i = 0; i < RPT; ++i) a[i][k] = fma(-p[q], v[i], a[i][k]);
                        R[k] = fma(-p[q], vr, R[k]);
                    }
                }
                }
            }
            }
        }
    }
    // Row `lane` of this slice's factor -> stacked output row slice*m + lane.
    if (lane < m) {
        const int64_t orow = slice * out_row0_stride + lane;
        const bool keep = lane < kvalid;
#pragma unroll
        for (int c = 0; c < M; ++c)
            if (c < m) out[orow + ld_out * c] = keep ? (double)R[c] : 0.0;
    }
}

template <int M, int RPT, typename Tin, int WAVES = kRowsWaves>
__device__ __forceinline__ void tsqr_rows_body(
    const Tin *__restrict__ W, int64_t rows, int m, int64_t ld, int64_t rows_per_slice,
    int64_t nslices, double *__restrict__ out, int64_t ld_out, int64_t out_row0_stride,
    int kvalid, int64_t vblock, void *smem) {
    using T = typename Elem<Tin>::acc;
    tsqr_rows_core<M, RPT, T, WAVES>(
        rows, m, rows_per_slice, nslices, out, ld_out, out_row0_stride, kvalid, vblock, smem,
        [&](int64_t base, int64_t r0, int64_t r1, T (&a)[RPT][M]) {
            const int lane = lane_id();
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                const int64_t row = base + lane + (int64_t)kWave * i;
                const bool ok = row < r1;
                const int64_t rc = ok ? row : r0;
#pragma unroll
                for (int c = 0; c < M; ++c)
                    a[i][c] = load_or_zero(W + rc + ld * (c < m ? c : 0), ok && c < m);
            }
        });
}

// ----------------------------------------------------------------------------
// Cooperative row-owner body, 8 < m <= M <= 128: NW waves share one row tile
// and reduce one slice.
//
// Column k of the tile belongs to wave k mod NW (slot k / NW), so every wave
// has trailing work at every step.  Lane l of each wave holds the rows
// (tile_base + l + 64 i), i < RPT, of its columns and rows l + 64 s
// (s < M / 64) of the factor R restricted to its columns.  Reflectors are
// published through LDS (double-buffered, one barrier per column) with a
// look-ahead of one: while the other waves apply reflector j to their
// trailing columns, the wave that owns column j+1 first updates that column,
// builds reflector j+1 and publishes it, and only then updates the rest of
// its columns.
// ----------------------------------------------------------------------------
template <int M, int NW, int RPT, typename Tin>
constexpr size_t tsqr_coop_smem() {
    using T = typename Elem<Tin>::acc;
    return sizeof(T) * (2 * RPT * kWave + 2 + NW * kWave);
}

// The body proper, with this wave's columns of the row tile supplied by
// `load(base, r0, r1, a)`: a[i][kk] = element (base + lane + 64 i, NW kk + w)
// of the slice [r0, r1), zero for rows >= r1 and columns >= m.
//
// TRI (M = 64, NW = RPT = 8): the tile is a stack of 8 upper-triangular
// 64 x 64 factors (a tree level), loaded so that register i of a lane holds
// rows 8 i .. 8 i + 7 of its factor (a[i][kk] = row 64 (lane / 8) + 8 i +
// lane mod 8 of the tile).  Column j of every factor is zero below row j and
// stays so (a reflector for column j only mixes rows <= j of each factor), so
// reflector j and its dot products and updates involve registers i <= j / 8
// only: the others are skipped.
template <int M, int NW, int RPT, typename T, typename Load, bool TRI = false>
__device__ __forceinline__ void tsqr_coop_core(
    int64_t rows, int m, int64_t rows_per_slice, int64_t slice, double *__restrict__ out,
    int64_t ld_out, int64_t out_row0_stride, int kvalid, void *smem, Load load) {
    constexpr int MW = M / NW;
    constexpr int RS = (M + kWave - 1) / kWave;  // rows of R per lane
    static_assert(MW * NW == M, "M must be a multiple of NW");
    static_assert(RS == 1 || kWave % NW == 0, "row sets need NW | 64");
    static_assert(!TRI || (M == 64 && NW == 8 && RPT == 8), "stacked-factor layout");
    // registers of a lane that can be nonzero in the columns of slot S
    auto nact = [](auto slot_c) constexpr { return TRI ? decltype(slot_c)::value + 1 : RPT; };
    T(*vbuf)[RPT][kWave] = reinterpret_cast<T(*)[RPT][kWave]>(smem);
    T *vrbuf = reinterpret_cast<T *>(smem) + 2 * RPT * kWave;

    const int lane = lane_id();
    const int w = thread_id() / kWave;
    const int64_t r0 = slice * rows_per_slice;
    const int64_t r1 = min(rows, r0 + rows_per_slice);
    T *lds = vrbuf + 2 + w * kWave;
    const T eps = EpsFP<T>::value();

    // R[s][k]: row 64 s + lane, column NW k + w of the factor.
    T R[RS][MW];
#pragma unroll
    for (int s = 0; s < RS; ++s)
#pragma unroll
        for (int k = 0; k < MW; ++k) R[s][k] = T(0);
    T a[RPT][MW];

    // Householder reflector of column jn, held by this wave in slot S
    // (Algorithm 6): u = (R_jn,jn ; tile column), alpha = -sign(u_1) ||u||,
    // v = (u - alpha e_1) / sqrt(t) with ||v||^2 = 2, published to LDS.
    // Row jn of R is row set NW S / 64 (compile time, NW | 64).
    auto reflector = [&](auto slot_c, int jn) {
        constexpr int S = decltype(slot_c)::value;
        constexpr int RSET = (NW * S) / kWave;
        constexpr int NA = nact(slot_c);
        const bool own = (lane == (jn & (kWave - 1)));
        T s = T(0);
#pragma unroll
        for (int i = 0; i < NA; ++i) s = fma(a[i][S], a[i][S], s);
        const T rjj = own ? R[RSET][S] : T(0);
        s = fma(rjj, rjj, s);
        s = wave_sum(s);
        const T u1 = read_lane(R[RSET][S], jn & (kWave - 1));
        T t = s + eps;
        const T t2 = t + eps;
        T alpha = t2 * rsqrt_nr(t2);
        alpha = (u1 > T(0)) ? -alpha : alpha;
        t = fma(-alpha, u1, t);
        const T beta = rsqrt_nr(t);
        const int buf = jn & 1;
#pragma unroll
        for (int i = 0; i < NA; ++i) vbuf[buf][i][lane] = beta * a[i][S];
        if (own) {
            vrbuf[buf] = beta * (u1 - alpha);
            R[RSET][S] = alpha;
        }
    };

    for (int64_t base = r0; base < r1; base += (int64_t)kWave * RPT) {
        load(base, r0, r1, a);
        if (w == 0) reflector(std::integral_constant<int, 0>{}, 0);
        static_for<0, MW>([&](auto jjc) {
            constexpr int jj = decltype(jjc)::value;
            constexpr int NT = MW - jj;  // slots jj..MW-1 may trail column j
            constexpr int RSET = (NW * jj) / kWave;  // row set of row j
            constexpr int NA = nact(jjc);  // registers where reflector j can be nonzero
            for (int o = 0; o < NW; ++o) {
                const int j = NW * jj + o;
                if (j >= m) break;
                const int buf = j & 1;
                __syncthreads();  // reflector j is in vbuf[buf]
                T v[NA];
#pragma unroll
                for (int i = 0; i < NA; ++i) v[i] = vbuf[buf][i][lane];
                const T vr = (lane == (j & (kWave - 1))) ? vrbuf[buf] : T(0);
                const bool first = (w > o);  // slot jj trails column j only in later waves
                T p[NT];
#pragma unroll
                for (int q = 0; q < NT; ++q) {
                    T acc = vr * R[RSET][jj + q];
#pragma unroll
                    for (int i = 0; i < NA; ++i) acc = fma(v[i], a[i][jj + q], acc);
                    p[q] = (q == 0 && !first) ? T(0) : acc;
                }
                wave_allreduce_vec<NT>(p, lds);
                auto update = [&](int q) {
#pragma unroll
                    for (int qq = 0; qq < NT; ++qq) {
                        if (qq == q) {
#pragma unroll
                            for (int i = 0; i < NA; ++i) a[i][jj + qq] = fma(-p[qq], v[i], a[i][jj + qq]);
                            R[RSET][jj + qq] = fma(-p[qq], vr, R[RSET][jj + qq]);
                        }
                    }
                };
                // look-ahead: column j+1 is slot jj of wave o+1, or slot jj+1 of wave 0
                int qn = -1;
                if (j + 1 < m) {
                    if (o + 1 < NW) {
                        if (w == o + 1) {
                            qn = 0;
                            update(0);
                            reflector(std::integral_constant<int, jj>{}, j + 1);
                        }
                    } else if constexpr (jj + 1 < MW) {
                        if (w == 0) {
                            qn = 1;
                            update(1);
                            reflector(std::integral_constant<int, jj + 1>{}, j + 1);
                        }
                    }
                }
#pragma unroll
                for (int q = 0; q < NT; ++q)
                    if ((q > 0 || first) && q != qn) update(q);
            }
        });
        // the first reflector of the next tile reuses buffer 0
        __syncthreads();
    }
#pragma unroll
    for (int s = 0; s < RS; ++s) {
        const int row = kWave * s + lane;
        if (row < m) {
            const int64_t orow = slice * out_row0_stride + row;
            const bool keep = row < kvalid;
#pragma unroll
            for (int kk = 0; kk < MW; ++kk) {
                const int c = NW * kk + w;
                if (c < m) out[orow + ld_out * c] = keep ? (double)R[s][kk] : 0.0;
            }
        }
    }
}

template <int M, int NW, int RPT, typename Tin, bool TRI = false>
__device__ __forceinline__ void tsqr_coop_body(
    const Tin *__restrict__ W, int64_t rows, int m, int64_t ld, int64_t rows_per_slice,
    int64_t slice, double *__restrict__ out, int64_t ld_out, int64_t out_row0_stride,
    int kvalid, void *smem) {
    using T = typename Elem<Tin>::acc;
    constexpr int MW = M / NW;
    auto load = [&](int64_t base, int64_t r0, int64_t r1, T (&a)[RPT][MW]) {
            const int lane = lane_id();
            const int w = thread_id() / kWave;
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                const int64_t row = TRI ? base + 64 * (lane >> 3) + 8 * i + (lane & 7)
                                        : base + lane + (int64_t)kWave * i;
                const bool ok = row < r1;
                const int64_t rc = ok ? row : r0;
#pragma unroll
                for (int kk = 0; kk < MW; ++kk) {
                    const int c = NW * kk + w;
                    a[i][kk] = load_or_zero(W + rc + ld * (c < m ? c : 0), ok && c < m);
                }
            }
        };
    tsqr_coop_core<M, NW, RPT, T, decltype(load), TRI>(
        rows, m, rows_per_slice, slice, out, ld_out, out_row0_stride, kvalid, smem, load);
}

// ----------------------------------------------------------------------------
// Planner: the levels of the reduction tree for (rows, m).  Level 0 reads W;
// every further level reduces the stacked (nslices * m) x m factors of the
// previous one, until one slice remains.  The shape depends only on (rows, m)
// and the planner parameters, so the tree (and the result) is deterministic.
// ----------------------------------------------------------------------------
constexpr int kTsqrMaxLevels = 16;

struct TsqrLevel {
    int64_t rows;            // rows of this level's input
    int64_t nslices;
    int64_t rows_per_slice;
};

struct TsqrPlanParams {
    int64_t max_slices;      // slices of level 0 and later levels
    int64_t min_tiles;       // a slice spans at least this many row tiles
};

// Level plan for an m-column input whose row tile is `tile` rows.
__host__ __device__ inline int tsqr_plan_levels(int64_t rows, int64_t m, int64_t tile,
                                                TsqrPlanParams pp, TsqrLevel *lv) {
    int n = 0;
    int64_t r = rows;
    for (;;) {
        const int64_t mr = pp.min_tiles * tile > 4 * m ? pp.min_tiles * tile : 4 * m;
        int64_t ns = (r + mr - 1) / mr;
        ns = ns < 1 ? 1 : ns;
        ns = ns > pp.max_slices ? pp.max_slices : ns;
        const int64_t per = (r + ns - 1) / ns;
        const int64_t rps = (per + tile - 1) / tile * tile;
        ns = (r + rps - 1) / rps;
        lv[n++] = TsqrLevel{r, ns, rps};
        if (ns == 1 || n == kTsqrMaxLevels) break;
        r = ns * m;
    }
    return n;
}

}  // namespace ttsvd
