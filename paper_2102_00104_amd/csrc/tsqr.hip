// Rank-preserving Q-less TSQR (Sec. 3.2 of arXiv 2102.00104) for gfx950.
//
// The triangular factor R of a tall-skinny W is computed without forming Q:
// each wave (m <= 8) or workgroup (m > 8) runs a flat reduction over a
// contiguous slice of rows, applying the Householder step of Algorithm 6 to
// [R; M] for every row tile M; the slices' triangular factors are stacked into
// a (slices*m) x m matrix and reduced the same way, level by level, until one
// slice remains.  The tree's shape depends only on (rows, m), so results are
// deterministic.  W is never written.
//
// The Householder step and the device bodies are in tsqr_dev.h.
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <type_traits>
#include <vector>

#include "common.h"
#include "kernels.h"
#include "profile.h"
#include "tsqr_blk.h"
#include "tsqr_dev.h"

namespace ttsvd {

// Per-level kernels of the single-tensor path: one workgroup per vblock.
template <int M, int RPT, typename Tin>
__global__ __launch_bounds__(kRowsWaves *kWave) void tsqr_rows_kernel(
    const Tin *__restrict__ W, int64_t rows, int m, int64_t ld,
    int64_t rows_per_slice, int64_t nslices, double *__restrict__ out,
    int64_t ld_out, int64_t out_row0_stride, int kvalid) {
    __shared__ __attribute__((aligned(16))) char smem[tsqr_rows_smem<M, RPT, Tin>()];
    tsqr_rows_body<M, RPT, Tin>(W, rows, m, ld, rows_per_slice, nslices, out, ld_out,
                                out_row0_stride, kvalid, blockIdx.x, smem);
}

template <int M, int NW, int RPT, typename Tin>
__global__ __launch_bounds__(NW *kWave) void tsqr_coop_kernel(
    const Tin *__restrict__ W, int64_t rows, int m, int64_t ld,
    int64_t rows_per_slice, int64_t nslices, double *__restrict__ out,
    int64_t ld_out, int64_t out_row0_stride, int kvalid) {
    __shared__ __attribute__((aligned(16))) char smem[tsqr_coop_smem<M, NW, RPT, Tin>()];
    (void)nslices;
    tsqr_coop_body<M, NW, RPT, Tin>(W, rows, m, ld, rows_per_slice, blockIdx.x, out, ld_out,
                                    out_row0_stride, kvalid, smem);
}

// Tree levels of m = 64: the tile is 8 stacked triangular factors, and the
// reflectors skip the rows that are still zero (tsqr_coop_core with TRI).
__global__ __launch_bounds__(8 * kWave) void tsqr_coop_tri_kernel(
    const double *__restrict__ W, int64_t rows, int m, int64_t ld, int64_t rows_per_slice,
    int64_t nslices, double *__restrict__ out, int64_t ld_out, int64_t out_row0_stride,
    int kvalid) {
    __shared__ __attribute__((aligned(16))) char smem[tsqr_coop_smem<64, 8, 8, double>()];
    (void)nslices;
    tsqr_coop_body<64, 8, 8, double, true>(W, rows, m, ld, rows_per_slice, blockIdx.x, out,
                                           ld_out, out_row0_stride, kvalid, smem);
}

// Product and first TSQR level of the next unfolding in one pass (the TSMM of
// Sec. 4.1.2 followed by the flat reduction of Sec. 3.2): for the next
// unfolding Y = reshape(W V, (rows_n, NN k)) with NN k <= M <= 8 columns,
// every wave builds its row tiles of Y from W and V (row y, column q + NN a of
// Y is row y + q rows_n of W V, column a), stores them and reduces them in the
// same registers, so Y is not read back for its QR.  The product accumulates
// over the columns of W in ascending order exactly as the TSMM kernel does,
// and the reduction is the rows body itself: Y and the factors equal those of
// the separate launches bit for bit.  W has mp <= 8 columns, V is FP64
// (V(c, a) = V[c svc + a sva]).
template <int M, int NN, int RPT, typename Tin>
__global__ __launch_bounds__(kRowsWaves *kWave) void tsmm_qr_kernel(
    const Tin *__restrict__ W, int mp, int64_t ld, const double *__restrict__ V, int64_t svc,
    int64_t sva, int k, Tin *__restrict__ Y, int64_t rows_n, int64_t rows_per_slice,
    int64_t nslices, double *__restrict__ out, int64_t ld_out, int64_t out_row0_stride,
    int kvalid) {
    using T = typename Elem<Tin>::acc;
    constexpr int KB = M / NN;  // columns of V per block of Y columns
    static_assert(KB * NN == M, "NN must divide M");
    __shared__ __attribute__((aligned(16))) char smem[tsqr_rows_smem<M, RPT, Tin>()];
    __shared__ T vs[8][KB];
    for (int idx = threadIdx.x; idx < 8 * KB; idx += blockDim.x) {
        const int c = idx / KB, a = idx % KB;
        vs[c][a] = (c < mp && a < k) ? (T)V[c * svc + a * sva] : T(0);
    }
    __syncthreads();
    tsqr_rows_core<M, RPT, T, kRowsWaves>(
        rows_n, NN * k, rows_per_slice, nslices, out, ld_out, out_row0_stride, kvalid,
        blockIdx.x, smem, [&](int64_t base, int64_t r0, int64_t r1, T (&y)[RPT][M]) {
            const int lane = lane_id();
            int64_t rc[RPT];
            bool ok[RPT];
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                const int64_t row = base + lane + (int64_t)kWave * i;
                ok[i] = row < r1;
                rc[i] = ok[i] ? row : r0;
            }
#pragma unroll
            for (int i = 0; i < RPT; ++i)
#pragma unroll
                for (int c = 0; c < M; ++c) y[i][c] = T(0);
            for (int c = 0; c < mp; ++c) {
                T vv[KB];
#pragma unroll
                for (int a = 0; a < KB; ++a) vv[a] = vs[c][a];
#pragma unroll
                for (int q = 0; q < NN; ++q)
#pragma unroll
                    for (int i = 0; i < RPT; ++i) {
                        const T w = load_or_zero(W + (rc[i] + q * rows_n) + ld * c, ok[i]);
#pragma unroll
                        for (int a = 0; a < KB; ++a) y[i][q + NN * a] = fma(w, vv[a], y[i][q + NN * a]);
                    }
            }
#pragma unroll
            for (int i = 0; i < RPT; ++i)
#pragma unroll
                for (int q = 0; q < NN; ++q)
#pragma unroll
                    for (int a = 0; a < KB; ++a) {
                        T &e = y[i][q + NN * a];
                        e = Elem<Tin>::round(e);  // the value Y holds
                        if (ok[i] && a < k) Elem<Tin>::store(Y + rc[i] + rows_n * (q + NN * a), e);
                    }
        });
}

// The same fusion for a next unfolding of 8 < NN k <= M <= 32 columns, with
// the cooperative body: wave w holds the columns NW kk + w of the tile, which
// are q + NN a with q = w mod NN and a = (NW / NN) kk + w / NN (NN divides
// NW), so a wave reads a single row block of W (rows y + q rows_n).  W has
// mp <= kTqMaxMp columns.
constexpr int kTqMaxMp = 32;

template <int M, int NW, int RPT, int NN, typename Tin>
__global__ __launch_bounds__(NW *kWave) void tsmm_qr_coop_kernel(
    const Tin *__restrict__ W, int mp, int64_t ld, const double *__restrict__ V, int64_t svc,
    int64_t sva, int k, Tin *__restrict__ Y, int64_t rows_n, int64_t rows_per_slice,
    double *__restrict__ out, int64_t ld_out, int64_t out_row0_stride, int kvalid) {
    using T = typename Elem<Tin>::acc;
    constexpr int MW = M / NW;
    constexpr int KB = M / NN;
    static_assert(NW % NN == 0 && KB * NN == M, "NN must divide NW and M");
    __shared__ __attribute__((aligned(16))) char smem[tsqr_coop_smem<M, NW, RPT, Tin>()];
    __shared__ T vs[kTqMaxMp][KB];
    for (int idx = threadIdx.x; idx < kTqMaxMp * KB; idx += blockDim.x) {
        const int c = idx / KB, a = idx % KB;
        vs[c][a] = (c < mp && a < k) ? (T)V[c * svc + a * sva] : T(0);
    }
    __syncthreads();
    tsqr_coop_core<M, NW, RPT, T>(
        rows_n, NN * k, rows_per_slice, blockIdx.x, out, ld_out, out_row0_stride, kvalid, smem,
        [&](int64_t base, int64_t r0, int64_t r1, T (&y)[RPT][MW]) {
            const int lane = lane_id();
            const int w = thread_id() / kWave;
            const int q = w % NN, a0 = w / NN;
            int64_t rc[RPT];
            bool ok[RPT];
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                const int64_t row = base + lane + (int64_t)kWave * i;
                ok[i] = row < r1;
                rc[i] = (ok[i] ? row : r0) + q * rows_n;
            }
#pragma unroll
            for (int i = 0; i < RPT; ++i)
#pragma unroll
                for (int kk = 0; kk < MW; ++kk) y[i][kk] = T(0);
            for (int c = 0; c < mp; ++c) {
                T vv[MW];
#pragma unroll
                for (int kk = 0; kk < MW; ++kk) vv[kk] = vs[c][(NW / NN) * kk + a0];
#pragma unroll
                for (int i = 0; i < RPT; ++i) {
                    const T x = load_or_zero(W + rc[i] + ld * c, ok[i]);
#pragma unroll
                    for (int kk = 0; kk < MW; ++kk) y[i][kk] = fma(x, vv[kk], y[i][kk]);
                }
            }
#pragma unroll
            for (int i = 0; i < RPT; ++i)
#pragma unroll
                for (int kk = 0; kk < MW; ++kk) {
                    const int a = (NW / NN) * kk + a0;
                    T &e = y[i][kk];
                    e = Elem<Tin>::round(e);  // the value Y holds
                    if (ok[i] && a < k)
                        Elem<Tin>::store(Y + (rc[i] - q * rows_n) + rows_n * (q + NN * a), e);
                }
        });
}

// ----------------------------------------------------------------------------
// Column-group workgroup kernel, 128 < m <= 1024 / G.
//
// The 1024 threads form groups of G adjacent lanes; group k owns column k of
// the current NB-row tile (lane q of the group holds the rows q + G i,
// i < NBL, in registers) and column k of the workgroup's triangular factor
// (row-major in global scratch, read and written only by lane 0 of the
// group).  For column j the G lanes of group j build the reflector (norm
// reduced inside the group) and publish it through LDS; every group with
// k > j then applies it to its column: the dot product over its rows is
// reduced inside the group, followed by the rank-1 update.  Rows of the
// factor are fetched four steps ahead (step j writes only row j), which keeps
// the global-memory latency of the factor off the serial chain of column
// steps.
// ----------------------------------------------------------------------------
constexpr int kColsThreads = 1024;

template <int G, int NBL, typename Tin>
__global__ __launch_bounds__(kColsThreads) void tsqr_cols_kernel(
    const Tin *__restrict__ W, int64_t rows, int m, int64_t ld,
    int64_t rows_per_slice, int64_t nslices, double *__restrict__ rws,
    double *__restrict__ out, int64_t ld_out, int64_t out_row0_stride,
    int kvalid) {
    using T = typename Elem<Tin>::acc;
    constexpr int NB = G * NBL;
    // vbuf[b][q NBL + i]: reflector entry of tile row q + G i (double-buffered)
    __shared__ __attribute__((aligned(16))) T vbuf[2][NB];
    __shared__ T vrbuf[2];
    const int tid = threadIdx.x;
    const int k = tid / G, q = tid % G;
    const bool col = k < m;
    const bool lead = col && q == 0;
    const int64_t slice = blockIdx.x;
    const int64_t r0 = slice * rows_per_slice;
    const int64_t r1 = min(rows, r0 + rows_per_slice);
    double *Rk = rws + slice * (int64_t)m * m + (col ? k : 0);  // Rk[j m] = R(j, k)
    const T eps = EpsFP<T>::value();

    if (lead)
        for (int j = 0; j < m; ++j) Rk[(int64_t)j * m] = 0.0;

    T a[NBL];
    for (int64_t base = r0; base < r1; base += NB) {
#pragma unroll
        for (int i = 0; i < NBL; ++i) {
            const int64_t row = base + q + (int64_t)G * i;
            const bool ok = col && row < r1;
            a[i] = load_or_zero(W + (row < r1 ? row : r0) + ld * (col ? k : 0), ok);
        }
        // Column step j with rv = R(j, k) (lane 0 of the group).
        auto step = [&](const int j, const double rv) {
            const int buf = j & 1;
            if (k == j) {
                // reflector of column j (Algorithm 6): u = (R_jj ; tile column)
                const T u1 = group_sum<G>(q == 0 ? (T)rv : T(0));
                T s0 = T(0), s1 = T(0), s2 = T(0), s3 = T(0);
#pragma unroll
                for (int i = 0; i < NBL; i += 4) {
                    s0 = fma(a[i], a[i], s0);
                    if (i + 1 < NBL) s1 = fma(a[i + 1], a[i + 1], s1);
                    if (i + 2 < NBL) s2 = fma(a[i + 2], a[i + 2], s2);
                    if (i + 3 < NBL) s3 = fma(a[i + 3], a[i + 3], s3);
                }
                T s = group_sum<G>((s0 + s1) + (s2 + s3));
                s = fma(u1, u1, s);
                T t = s + eps;
                const T t2 = t + eps;
                T alpha = t2 * rsqrt_nr(t2);
                alpha = (u1 > T(0)) ? -alpha : alpha;
                t = fma(-alpha, u1, t);
                const T beta = rsqrt_nr(t);
#pragma unroll
                for (int i = 0; i < NBL; ++i) vbuf[buf][q * NBL + i] = beta * a[i];
                if (q == 0) {
                    vrbuf[buf] = beta * (u1 - alpha);
                    Rk[(int64_t)j * m] = (double)alpha;
                }
            }
            __syncthreads();
            if (col && k > j) {
                const T vr = vrbuf[buf];
                // The lane's NBL reflector entries are read from LDS once and
                // kept in registers where they fit next to the tile (up to
                // 128 bytes); otherwise they are read again for the update,
                // which keeps a 1024-thread workgroup within its registers.
                constexpr bool kHold = NBL * sizeof(T) <= 128;
                const T *vb = &vbuf[buf][q * NBL];
                T v[kHold ? NBL : 1];
                if constexpr (kHold) {
#pragma unroll
                    for (int i = 0; i < NBL; ++i) v[i] = vb[i];
                }
                auto vi = [&](int i) -> T {
                    if constexpr (kHold) return v[i];
                    else return vb[i];
                };
                T p0 = (q == 0) ? vr * (T)rv : T(0), p1 = T(0), p2 = T(0), p3 = T(0);
#pragma unroll
                for (int i = 0; i < NBL; i += 4) {
                    p0 = fma(vi(i), a[i], p0);
                    if (i + 1 < NBL) p1 = fma(vi(i + 1), a[i + 1], p1);
                    if (i + 2 < NBL) p2 = fma(vi(i + 2), a[i + 2], p2);
                    if (i + 3 < NBL) p3 = fma(vi(i + 3), a[i + 3], p3);
                }
                const T p = group_sum<G>((p0 + p1) + (p2 + p3));
                if constexpr (!kHold) __asm__ volatile("" ::: "memory");  // re-read vb
#pragma unroll
                for (int i = 0; i < NBL; ++i) a[i] = fma(-p, vi(i), a[i]);
                if (q == 0) Rk[(int64_t)j * m] = (double)fma(-p, vr, (T)rv);
            }
        };
        // Steps in groups of four; rows j0 + 4 .. j0 + 7 of the factor are
        // fetched while steps j0 .. j0 + 3 run (step j writes only row j).
        auto ldR = [&](int j) -> double { return (lead && j < m) ? Rk[(int64_t)j * m] : 0.0; };
        double rq0 = ldR(0), rq1 = ldR(1), rq2 = ldR(2), rq3 = ldR(3);
        for (int j0 = 0; j0 < m; j0 += 4) {
            const double n0 = ldR(j0 + 4), n1 = ldR(j0 + 5), n2 = ldR(j0 + 6), n3 = ldR(j0 + 7);
            step(j0, rq0);
            if (j0 + 1 < m) step(j0 + 1, rq1);
            if (j0 + 2 < m) step(j0 + 2, rq2);
            if (j0 + 3 < m) step(j0 + 3, rq3);
            rq0 = n0;
            rq1 = n1;
            rq2 = n2;
            rq3 = n3;
        }
        // vbuf parity restarts with the next tile: wait for all readers.
        __syncthreads();
    }
    // Stacked output: factor row j -> out row slice*m + j.
    if (lead)
        for (int j = 0; j < m; ++j) {
            const double v = (j <= k && j < kvalid) ? Rk[(int64_t)j * m] : 0.0;
            out[slice * out_row0_stride + j + ld_out * k] = v;
        }
}

// ----------------------------------------------------------------------------
// Planner: the levels of the reduction tree for (rows, m).
// ----------------------------------------------------------------------------
namespace {

constexpr int64_t kMaxWaveSlices = 2048;  // single-wave slices: 256 CUs x 8 waves
constexpr int64_t kMaxCoopSlices = 512;   // cooperative slices: up to 2 per CU
constexpr int64_t kMaxColsSlices = 256;   // 1024-thread slices: 1 per CU
// rows per lane of the column-group kernel: 32 with one lane per column, 16
// with two or four (register budget of a 1024-thread workgroup in FP64)
constexpr int cols_rows_per_lane(int g) { return g == 1 ? 32 : 16; }

// Kernel family and shape for m columns.
enum class Kind { Rows, Coop, Blk, Cols };
struct Shape {
    Kind kind;
    int M;       // column bucket (Rows, Coop)
    int nw;      // waves per workgroup (Coop)
    int rpt;     // rows per lane per tile (Rows, Coop)
    int g;       // lanes per column (Cols)
    int64_t tile;
};

// Cooperative-kernel configurations per column bucket: waves per workgroup
// and rows per lane.  Entry 0 is the default; TTSVD_COOP_VARIANT selects
// another one (a tuning override, the result does not depend on it beyond
// the summation order).
struct CoopCfg {
    int nw, rpt;
};
constexpr CoopCfg kCoop16[3] = {{4, 16}, {8, 16}, {16, 16}};
constexpr CoopCfg kCoop32[3] = {{4, 8}, {8, 16}, {16, 8}};
constexpr CoopCfg kCoop64[3] = {{8, 8}, {4, 4}, {16, 4}};
constexpr CoopCfg kCoop128[3] = {{8, 2}, {4, 2}, {16, 2}};

int coop_variant() {
    static int v = [] {
        const char *e = getenv("TTSVD_COOP_VARIANT");
        int x = e ? atoi(e) : 0;
        return (x >= 0 && x < 3) ? x : 0;
    }();
    return v;
}

CoopCfg coop_cfg(int M) {
    const int v = coop_variant();
    return M == 16 ? kCoop16[v] : M == 32 ? kCoop32[v] : M == 64 ? kCoop64[v] : kCoop128[v];
}

// TTSVD_TSQR_TRI=0 runs the tree levels of m = 64 with the general
// cooperative kernel instead of the stacked-triangle one (a tuning override).
bool tri_enabled() {
    static bool v = [] {
        const char *e = getenv("TTSVD_TSQR_TRI");
        return !(e && atoi(e) == 0);
    }();
    return v;
}

// TTSVD_TSQR_BLK=0 selects the column-group kernel for 128 < m <= 512 instead
// of the blocked one (a tuning override).
bool blk_enabled() {
    static bool v = [] {
        const char *e = getenv("TTSVD_TSQR_BLK");
        return !(e && atoi(e) == 0);
    }();
    return v;
}

Shape shape_for(int64_t m) {
    Shape sh{Kind::Cols, 0, 0, 0, 0, 0};
    if (m <= 8) {
        sh.kind = Kind::Rows;
        sh.M = (int)cpow2((int)m);
        sh.rpt = 8;
        sh.tile = (int64_t)kWave * sh.rpt;
    } else if (m <= 128) {
        sh.kind = Kind::Coop;
        sh.M = (int)cpow2((int)m);
        const CoopCfg c = coop_cfg(sh.M);
        sh.nw = c.nw;
        sh.rpt = c.rpt;
        sh.tile = (int64_t)kWave * sh.rpt;
    } else if (m <= kBlkMaxM && blk_enabled()) {
        sh.kind = Kind::Blk;
        sh.tile = kBlkTR;
    } else {
        sh.g = m <= 256 ? 4 : m <= 512 ? 2 : 1;
        sh.tile = (int64_t)sh.g * cols_rows_per_lane(sh.g);
    }
    return sh;
}

using Level = TsqrLevel;

// Row tiles a slice spans at least for the wave and cooperative kernels:
// one tile per slice gives the shortest sequential chain for small steps
// (more, shorter tree levels); large steps are capped by the slice count
// anyway.  TTSVD_TSQR_MIN_TILES overrides it (a tuning knob).
int64_t min_tiles() {
    static int64_t v = [] {
        const char *e = getenv("TTSVD_TSQR_MIN_TILES");
        const long x = e ? atol(e) : 1;
        return (int64_t)((x >= 1 && x <= 64) ? x : 1);
    }();
    return v;
}

std::vector<Level> plan(int64_t rows, int64_t m) {
    const Shape sh = shape_for(m);
    if (sh.kind == Kind::Blk) {
        // one tile per slice; every level stacks the tiles' factors
        std::vector<Level> lv;
        int64_t r = rows;
        for (;;) {
            const int64_t ns = std::max<int64_t>(1, ceil_div(r, sh.tile));
            lv.push_back(Level{r, ns, sh.tile});
            if (ns == 1 || (int)lv.size() == kTsqrMaxLevels) break;
            r = ns * m;
        }
        return lv;
    }
    TsqrPlanParams pp;
    if (sh.kind == Kind::Rows)
        pp = {kMaxWaveSlices, min_tiles()};
    else if (sh.kind == Kind::Coop)
        pp = {kMaxCoopSlices, min_tiles()};
    else
        pp = {kMaxColsSlices, 8};
    TsqrLevel lv[kTsqrMaxLevels];
    const int n = tsqr_plan_levels(rows, m, sh.tile, pp, lv);
    return std::vector<Level>(lv, lv + n);
}

size_t level_out_doubles(const Level &l, int64_t m) { return (size_t)(l.nslices * m) * (size_t)m; }

// Sizes (doubles) of the two ping-pong buffers of the stacked factors: level i
// (all but the last, which writes R) writes buffer i mod 2.
void level_buffers(const std::vector<Level> &lv, int64_t m, size_t buf[2]) {
    buf[0] = buf[1] = 0;
    for (size_t i = 0; i + 1 < lv.size(); ++i)
        buf[i & 1] = std::max(buf[i & 1], level_out_doubles(lv[i], m));
}

template <typename Tin>
int launch_level_raw(const Tin *W, int64_t rows, int64_t m, int64_t ld, const Level &l,
                     double *out, int64_t ld_out, int64_t out_stride, int kvalid,
                     double *rws, bool tree, hipStream_t s);

template <typename Tin> const char *tname();
template <> const char *tname<double>() { return "double"; }
template <> const char *tname<float>() { return "float"; }
template <> const char *tname<bf16>() { return "ttsvd::bf16"; }

template <typename Tin>
int launch_level(const Tin *W, int64_t rows, int64_t m, int64_t ld, const Level &l,
                 double *out, int64_t ld_out, int64_t out_stride, int kvalid,
                 double *rws, bool tree, hipStream_t s) {
    char name[96];
    const Shape sh = shape_for(m);
    if (sh.kind == Kind::Rows)
        snprintf(name, sizeof(name), "tsqr_rows_kernel<%d, %d, %s>", sh.M, sh.rpt, tname<Tin>());
    else if (sh.kind == Kind::Coop && tree && m == 64 && sh.nw == 8 && sh.rpt == 8 && tri_enabled() &&
             std::is_same<Tin, double>::value && l.rows_per_slice % 64 == 0)
        snprintf(name, sizeof(name), "tsqr_coop_tri_kernel");
    else if (sh.kind == Kind::Coop)
        snprintf(name, sizeof(name), "tsqr_coop_kernel<%d, %d, %d, %s>", sh.M, sh.nw, sh.rpt,
                 tname<Tin>());
    else if (sh.kind == Kind::Blk)
        snprintf(name, sizeof(name), "tsqr_blk_kernel<%s>", tname<Tin>());
    else
        snprintf(name, sizeof(name), "tsqr_cols_kernel<%d, %d, %s>", sh.g, cols_rows_per_lane(sh.g), tname<Tin>());
    prof_begin(s, name, (double)rows * (double)m * sizeof(Tin), 2.0 * (double)rows * (double)m * (double)m);
    int rc = launch_level_raw(W, rows, m, ld, l, out, ld_out, out_stride, kvalid, rws, tree, s);
    prof_end(s);
    return rc;
}

template <typename Tin>
int launch_level_raw(const Tin *W, int64_t rows, int64_t m, int64_t ld, const Level &l,
                     double *out, int64_t ld_out, int64_t out_stride, int kvalid,
                     double *rws, bool tree, hipStream_t s) {
    const Shape sh = shape_for(m);
    if (sh.kind == Kind::Rows) {
        dim3 grid((unsigned)ceil_div(l.nslices, kRowsWaves)), block(kRowsWaves * kWave);
#define TTSVD_ROWS_CASE(MM)                                                                 \
    case MM:                                                                                \
        hipLaunchKernelGGL((tsqr_rows_kernel<MM, 8, Tin>), grid, block, 0, s, W, rows,     \
                           (int)m, ld, l.rows_per_slice, l.nslices, out, ld_out, out_stride, \
                           kvalid);                                                         \
        break;
        switch (sh.M) {
            TTSVD_ROWS_CASE(1)
            TTSVD_ROWS_CASE(2)
            TTSVD_ROWS_CASE(4)
            TTSVD_ROWS_CASE(8)
            default:
                return set_error(TTSVD_EUNSUPPORTED, "tsqr: bad column bucket %d", sh.M);
        }
#undef TTSVD_ROWS_CASE
    } else if (sh.kind == Kind::Coop && tree && m == 64 && sh.nw == 8 && sh.rpt == 8 && tri_enabled() &&
               std::is_same<Tin, double>::value && l.rows_per_slice % 64 == 0) {
        hipLaunchKernelGGL(tsqr_coop_tri_kernel, dim3((unsigned)l.nslices), dim3(8 * kWave), 0, s,
                           (const double *)W, rows, (int)m, ld, l.rows_per_slice, l.nslices, out,
                           ld_out, out_stride, kvalid);
    } else if (sh.kind == Kind::Coop) {
        dim3 grid((unsigned)l.nslices), block(sh.nw * kWave);
#define TTSVD_COOP_LAUNCH(MM, NN, RR)                                                         \
    hipLaunchKernelGGL((tsqr_coop_kernel<MM, NN, RR, Tin>), grid, block, 0, s, W, rows, (int)m, \
                       ld, l.rows_per_slice, l.nslices, out, ld_out, out_stride, kvalid)
#define TTSVD_COOP_CASE(MM, TABLE)                                                             \
    case MM:                                                                                  \
        if (sh.nw == TABLE[0].nw && sh.rpt == TABLE[0].rpt)                                    \
            TTSVD_COOP_LAUNCH(MM, TABLE[0].nw, TABLE[0].rpt);                                  \
        else if (sh.nw == TABLE[1].nw && sh.rpt == TABLE[1].rpt)                               \
            TTSVD_COOP_LAUNCH(MM, TABLE[1].nw, TABLE[1].rpt);                                  \
        else                                                                                  \
            TTSVD_COOP_LAUNCH(MM, TABLE[2].nw, TABLE[2].rpt);                                  \
        break;
        switch (sh.M) {
            TTSVD_COOP_CASE(16, kCoop16)
            TTSVD_COOP_CASE(32, kCoop32)
            TTSVD_COOP_CASE(64, kCoop64)
            TTSVD_COOP_CASE(128, kCoop128)
            default:
                return set_error(TTSVD_EUNSUPPORTED, "tsqr: bad column bucket %d", sh.M);
        }
#undef TTSVD_COOP_LAUNCH
#undef TTSVD_COOP_CASE
    } else if (sh.kind == Kind::Blk) {
        return tsqr_blk_level(W, rows, m, ld, tree, l.nslices, rws, out, ld_out, out_stride,
                              kvalid, s);
    } else {
        dim3 grid((unsigned)l.nslices), block(kColsThreads);
#define TTSVD_COLS_CASE(GG)                                                                   \
    case GG:                                                                                  \
        hipLaunchKernelGGL((tsqr_cols_kernel<GG, cols_rows_per_lane(GG), Tin>), grid, block, 0, s, \
                           W, rows, (int)m, ld, l.rows_per_slice, l.nslices, rws, out, ld_out, \
                           out_stride, kvalid);                                               \
        break;
        switch (sh.g) {
            TTSVD_COLS_CASE(1)
            TTSVD_COLS_CASE(2)
            TTSVD_COLS_CASE(4)
            default:
                return set_error(TTSVD_EUNSUPPORTED, "tsqr: bad column group %d", sh.g);
        }
#undef TTSVD_COLS_CASE
    }
    TTSVD_HIP_TRY(hipGetLastError());
    return TTSVD_OK;
}

}  // namespace

size_t tsqr_workspace_bytes(int dtype, int64_t rows, int64_t m) {
    (void)dtype;
    std::vector<Level> lv = plan(rows, m);
    size_t buf[2] = {0, 0}, rws = 0;
    level_buffers(lv, m, buf);
    if (shape_for(m).kind == Kind::Blk)
        for (const Level &l : lv) rws = std::max(rws, (size_t)blk_ws_doubles(l.nslices, m));
    else if (m > 128)
        for (const Level &l : lv) rws = std::max(rws, (size_t)(l.nslices * m) * (size_t)m);
    return (buf[0] + buf[1] + rws) * sizeof(double) + 256;
}

namespace {

// Levels from..end of the TSQR of W; levels before `from` have already
// written their stacked factors where this function would have.
int tsqr_levels(const void *W, int dtype, int64_t rows, int64_t m, int64_t ld, double *R,
                int64_t ldr, void *ws, size_t ws_bytes, hipStream_t s, size_t from) {
    if (m > 1024) return set_error(TTSVD_EUNSUPPORTED, "tsqr: cols = %lld > 1024", (long long)m);
    std::vector<Level> lv = plan(rows, m);
    size_t buf[2] = {0, 0};
    level_buffers(lv, m, buf);
    if (ws_bytes < tsqr_workspace_bytes(dtype, rows, m))
        return set_error(TTSVD_EINVAL, "tsqr: workspace too small");
    double *b0 = (double *)ws;
    double *b1 = b0 + buf[0];
    double *rws = b1 + buf[1];
    const int kvalid = (int)std::min<int64_t>(rows, m);
    const double *in = nullptr;
    if (from > 0 && from < lv.size()) in = ((from - 1) & 1) ? b1 : b0;
    for (size_t i = from; i < lv.size(); ++i) {
        const Level &l = lv[i];
        const bool last = (i + 1 == lv.size());
        double *out = last ? R : ((i & 1) ? b1 : b0);
        const int64_t ld_out = last ? ldr : l.nslices * m;
        const int kv = last ? kvalid : (int)m;
        int rc;
        if (i == 0) {
            switch (dtype) {
                case TTSVD_F64:
                    rc = launch_level((const double *)W, rows, m, ld, l, out, ld_out, m, kv, rws, false, s);
                    break;
                case TTSVD_F32:
                    rc = launch_level((const float *)W, rows, m, ld, l, out, ld_out, m, kv, rws, false, s);
                    break;
                case TTSVD_BF16:
                    rc = launch_level((const bf16 *)W, rows, m, ld, l, out, ld_out, m, kv, rws, false, s);
                    break;
                default:
                    return set_error(TTSVD_EUNSUPPORTED, "tsqr: dtype %d", dtype);
            }
        } else {
            rc = launch_level(in, l.rows, m, l.rows, l, out, ld_out, m, kv, rws, true, s);
        }
        if (rc != TTSVD_OK) return rc;
        in = out;
    }
    return TTSVD_OK;
}

}  // namespace

int tsqr_launch(const void *W, int dtype, int64_t rows, int64_t m, int64_t ld, double *R,
                int64_t ldr, void *ws, size_t ws_bytes, hipStream_t s) {
    return tsqr_levels(W, dtype, rows, m, ld, R, ldr, ws, ws_bytes, s, 0);
}

int tsqr_launch_after_first(int dtype, int64_t rows, int64_t m, double *R, int64_t ldr,
                            void *ws, size_t ws_bytes, hipStream_t s) {
    return tsqr_levels(nullptr, dtype, rows, m, rows, R, ldr, ws, ws_bytes, s, 1);
}

bool tsmm_qr_applies(int dtype, int64_t rows, int64_t m, int64_t k, int64_t n_next) {
    const int64_t mn = n_next * k;
    if (!((dtype == TTSVD_F64 || dtype == TTSVD_F32 || dtype == TTSVD_BF16) && m >= 1 && k >= 1 &&
          (n_next == 2 || n_next == 4) && rows % n_next == 0 && rows / n_next > mn))
        return false;
    const Shape sh = shape_for(mn);
    if (mn <= 8) return m <= 8 && sh.kind == Kind::Rows;
    // the cooperative shapes instantiated below (default configurations)
    return mn <= 32 && m <= kTqMaxMp && sh.kind == Kind::Coop && sh.nw == 4 &&
           sh.rpt == (sh.M == 16 ? 16 : 8);
}

template <typename Tin>
static int tsmm_qr_typed(const Tin *W, int64_t rows, int64_t m, int64_t ld, const double *V,
                         int64_t svc, int64_t sva, int64_t k, int64_t n_next, Tin *Y,
                         const Level &l, double *out, int64_t ld_out, int kvalid, hipStream_t s) {
    const int64_t rows_n = rows / n_next;
    const int M = cpow2((int)(n_next * k));
    char name[96];
    const double bytes = (double)rows * (double)(m + k) * sizeof(Tin);
    const double flops = 2.0 * (double)rows * (double)m * (double)k +
                         2.0 * (double)rows_n * (double)(n_next * k) * (double)(n_next * k);
    if (M > 8) {
        const Shape sh = shape_for(n_next * k);
        snprintf(name, sizeof(name), "tsmm_qr_coop_kernel<%d, %d, %d, %d, %s>", sh.M, sh.nw, sh.rpt,
                 (int)n_next, tname<Tin>());
        prof_begin(s, name, bytes, flops);
        dim3 grid((unsigned)l.nslices), block(sh.nw * kWave);
#define TTSVD_TQC(MM, RR, NN)                                                                  \
    hipLaunchKernelGGL((tsmm_qr_coop_kernel<MM, 4, RR, NN, Tin>), grid, block, 0, s, W, (int)m,  \
                       ld, V, svc, sva, (int)k, Y, rows_n, l.rows_per_slice, out, ld_out,         \
                       n_next * k, kvalid)
        if (M == 16 && n_next == 2)
            TTSVD_TQC(16, 16, 2);
        else if (M == 16 && n_next == 4)
            TTSVD_TQC(16, 16, 4);
        else if (M == 32 && n_next == 2)
            TTSVD_TQC(32, 8, 2);
        else if (M == 32 && n_next == 4)
            TTSVD_TQC(32, 8, 4);
        else {
            prof_end(s);
            return set_error(TTSVD_EUNSUPPORTED, "tsmm_qr: M = %d, n_next = %lld", M, (long long)n_next);
        }
#undef TTSVD_TQC
        prof_end(s);
        TTSVD_HIP_TRY(hipGetLastError());
        return TTSVD_OK;
    }
    dim3 grid((unsigned)ceil_div(l.nslices, kRowsWaves)), block(kRowsWaves * kWave);
    snprintf(name, sizeof(name), "tsmm_qr_kernel<%d, %d, 8, %s>", M, (int)n_next, tname<Tin>());
    prof_begin(s, name, bytes, flops);
#define TTSVD_TQ(MM, NN)                                                                         \
    hipLaunchKernelGGL((tsmm_qr_kernel<MM, NN, 8, Tin>), grid, block, 0, s, W, (int)m, ld, V, svc, \
                       sva, (int)k, Y, rows_n, l.rows_per_slice, l.nslices, out, ld_out,          \
                       n_next * k, kvalid)
    if (M == 2 && n_next == 2)
        TTSVD_TQ(2, 2);
    else if (M == 4 && n_next == 2)
        TTSVD_TQ(4, 2);
    else if (M == 4 && n_next == 4)
        TTSVD_TQ(4, 4);
    else if (M == 8 && n_next == 2)
        TTSVD_TQ(8, 2);
    else if (M == 8 && n_next == 4)
        TTSVD_TQ(8, 4);
    else {
        prof_end(s);
        return set_error(TTSVD_EUNSUPPORTED, "tsmm_qr: M = %d, n_next = %lld", M, (long long)n_next);
    }
#undef TTSVD_TQ
    prof_end(s);
    TTSVD_HIP_TRY(hipGetLastError());
    return TTSVD_OK;
}

int tsmm_qr_launch(const void *W, int dtype, int64_t rows, int64_t m, int64_t ld,
                   const double *V, int64_t svc, int64_t sva, int64_t k, int64_t n_next, void *Y,
                   double *R, int64_t ldr, void *ws, size_t ws_bytes, hipStream_t s,
                   int *levels_done) {
    if (!tsmm_qr_applies(dtype, rows, m, k, n_next))
        return set_error(TTSVD_EUNSUPPORTED, "tsmm_qr: shape");
    const int64_t rows_n = rows / n_next, mn = n_next * k;
    std::vector<Level> lv = plan(rows_n, mn);
    size_t buf[2] = {0, 0};
    level_buffers(lv, mn, buf);
    if (ws_bytes < tsqr_workspace_bytes(dtype, rows_n, mn))
        return set_error(TTSVD_EINVAL, "tsmm_qr: workspace too small");
    const bool last = lv.size() == 1;
    double *out = last ? R : (double *)ws;  // where level 0 of the TSQR of Y writes
    const int64_t ld_out = last ? ldr : lv[0].nslices * mn;
    const int kv = last ? (int)std::min<int64_t>(rows_n, mn) : (int)mn;
    int rc;
    switch (dtype) {
        case TTSVD_F64:
            rc = tsmm_qr_typed((const double *)W, rows, m, ld, V, svc, sva, k, n_next, (double *)Y,
                               lv[0], out, ld_out, kv, s);
            break;
        case TTSVD_F32:
            rc = tsmm_qr_typed((const float *)W, rows, m, ld, V, svc, sva, k, n_next, (float *)Y,
                               lv[0], out, ld_out, kv, s);
            break;
        default:
            rc = tsmm_qr_typed((const bf16 *)W, rows, m, ld, V, svc, sva, k, n_next, (bf16 *)Y,
                               lv[0], out, ld_out, kv, s);
            break;
    }
    if (rc == TTSVD_OK) *levels_done = 1;
    return rc;
}

}  // namespace ttsvd
