// C ABI of libttsvd and the host driver of the TSQR TT-SVD (Algorithm 2 of
// arXiv 2102.00104).  Validation happens before anything is enqueued; no C++
// exception crosses the ABI.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "common.h"
#include "driver.h"
#include "kernels.h"

namespace ttsvd {

namespace {
thread_local char g_err[512] = "";
}

int set_error(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

void clear_error() { g_err[0] = 0; }

bool valid_dtype(int dt) { return dt == TTSVD_F64 || dt == TTSVD_F32 || dt == TTSVD_BF16; }

namespace {
// Device state of one decomposition: per-step ranks and discarded energy plus
// the threshold set by the first step.
struct DecompState {
    StepState step[TTSVD_MAX_D];
    double one;  // 1.0, the 1 x 1 "V" used to copy a single-mode tensor
};
}  // namespace

int plan_steps(const int64_t *dims, int d, int64_t r_max, std::vector<StepShape> &steps,
               std::vector<int64_t> &rb, int64_t &nbar_out) {
    int64_t nbar = 1;
    for (int i = 0; i < d; ++i) {
        if (dims[i] < 1) return set_error(TTSVD_EINVAL, "dims[%d] = %lld < 1", i, (long long)dims[i]);
        if (nbar > (int64_t(1) << 62) / dims[i])
            return set_error(TTSVD_EINVAL, "product of dims overflows");
        nbar *= dims[i];
    }
    nbar_out = nbar;
    rb.assign(d + 1, 1);
    steps.assign(d, StepShape{0, 0, 0, 0});
    int64_t nb = nbar;
    for (int i = d - 1; i >= 1; --i) {
        StepShape st;
        st.m = dims[i] * rb[i + 1];
        st.rows = nb / st.m;
        st.K = std::min(st.rows, st.m);
        st.rb = std::min(r_max, st.K);
        rb[i] = st.rb;
        steps[i] = st;
        nb = st.rows * st.rb;
    }
    return TTSVD_OK;
}

namespace {
struct Footprint {
    size_t wbuf[2] = {0, 0};   // ping-pong work matrices (elements)
    size_t rbuf = 0;           // doubles
    size_t tsqr_ws = 0;        // bytes
    size_t svd_ws = 0;         // bytes
    size_t sigma = 0;          // doubles
    size_t cores = 0;          // doubles
    std::vector<size_t> core_off, sigma_off;
};

Footprint footprint(const int64_t *dims, int d, int dtype, const std::vector<StepShape> &steps,
                    const std::vector<int64_t> &rb) {
    Footprint f;
    f.core_off.assign(d, 0);
    f.sigma_off.assign(d, 0);
    for (int i = 0; i < d; ++i) {
        f.core_off[i] = f.cores;
        f.cores += (size_t)(rb[i] * dims[i] * rb[i + 1]);
    }
    int pp = 0;
    for (int i = d - 1; i >= 1; --i) {
        const StepShape &s = steps[i];
        f.rbuf = std::max(f.rbuf, (size_t)(s.m * s.m));
        // The TSQR tree and the SVD scratch are not monotone in the column
        // count (fewer columns can mean more slices or a larger Jacobi block),
        // so size them for every rank the previous step may choose.
        const int64_t rn_max = (i + 1 < d) ? rb[i + 1] : 1;
        for (int64_t rn = 1; rn <= rn_max; ++rn) {
            const int64_t m = dims[i] * rn;
            f.tsqr_ws = std::max(f.tsqr_ws, tsqr_workspace_bytes(dtype, s.rows, m));
            f.svd_ws = std::max(f.svd_ws, svd_scratch_bytes(std::min(s.rows, m), m));
        }
        f.sigma_off[i] = f.sigma;
        f.sigma += (size_t)s.K;
        if (i >= 2) {
            f.wbuf[pp] = std::max(f.wbuf[pp], (size_t)(s.rows * s.rb));
            pp ^= 1;
        }
    }
    return f;
}

// Offsets (bytes) of the parts of a decomposition's workspace: the two
// ping-pong work matrices, R, the TSQR tree, the SVD scratch, sigma and the
// device state, each 256-byte aligned.
struct WsLayout {
    size_t w0, w1, r, tq, sv, sg, st, total;
};

WsLayout ws_layout(const Footprint &f, size_t es) {
    WsLayout l;
    l.w0 = 0;
    l.w1 = l.w0 + align256(f.wbuf[0] * es);
    l.r = l.w1 + align256(f.wbuf[1] * es);
    l.tq = l.r + align256(f.rbuf * 8);
    l.sv = l.tq + align256(f.tsqr_ws);
    l.sg = l.sv + align256(f.svd_ws);
    l.st = l.sg + align256(f.sigma * 8);
    l.total = l.st + align256(sizeof(DecompState));
    return l;
}

}  // namespace

namespace {
struct CacheBlock {
    void *p;
    size_t bytes;
    int dev;
    bool busy;
};
std::mutex g_cache_mu;
std::vector<CacheBlock> g_cache;
constexpr size_t kCacheIdleBytes = size_t(32) << 30;  // idle memory kept per device

// Frees idle blocks of device `dev`, largest first, until at most `keep`
// idle bytes remain (called without the lock held).
void cache_trim(int dev, size_t keep) {
    std::vector<void *> drop;
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        size_t idle = 0;
        for (const CacheBlock &b : g_cache)
            if (!b.busy && b.dev == dev) idle += b.bytes;
        while (idle > keep) {
            int big = -1;
            for (int i = 0; i < (int)g_cache.size(); ++i)
                if (!g_cache[i].busy && g_cache[i].dev == dev &&
                    (big < 0 || g_cache[i].bytes > g_cache[big].bytes))
                    big = i;
            if (big < 0) break;
            idle -= g_cache[big].bytes;
            drop.push_back(g_cache[big].p);
            g_cache.erase(g_cache.begin() + big);
        }
    }
    for (void *p : drop) (void)hipFree(p);
}

void release_cb(void *p) { cache_release(p); }
}  // namespace

void *cache_acquire(size_t bytes) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    bytes = align256(std::max<size_t>(bytes, 1));
    {
        // best fit among idle blocks that are not much larger than asked for
        std::lock_guard<std::mutex> lk(g_cache_mu);
        const size_t limit = std::max(2 * bytes, bytes + (size_t(64) << 20));
        int best = -1;
        for (int i = 0; i < (int)g_cache.size(); ++i) {
            const CacheBlock &b = g_cache[i];
            if (!b.busy && b.dev == dev && b.bytes >= bytes && b.bytes <= limit &&
                (best < 0 || b.bytes < g_cache[best].bytes))
                best = i;
        }
        if (best >= 0) {
            g_cache[best].busy = true;
            return g_cache[best].p;
        }
    }
    cache_trim(dev, kCacheIdleBytes);  // bound the idle memory before growing
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        cache_trim(dev, 0);  // give idle blocks back and try once more
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
    }
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_cache.push_back(CacheBlock{p, bytes, dev, true});
    return p;
}

// (also called from host callbacks: no HIP calls here)
void cache_release(void *p) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_cache_mu);
    for (CacheBlock &b : g_cache)
        if (b.p == p) {
            b.busy = false;
            break;
        }
}

hipError_t cache_release_async(void *p, hipStream_t s) {
    return hipLaunchHostFunc(s, release_cb, p);
}

void *result_alloc(size_t bytes) { return cache_acquire(bytes); }

void result_free(void *p) {
    if (!p) return;
    (void)hipDeviceSynchronize();
    cache_release(p);
}

void *pinned_stage(size_t bytes) {
    // (released only with the thread: the runtime may be gone by the time a
    // thread-local destructor would run at process exit)
    thread_local void *buf = nullptr;
    thread_local size_t cap = 0;
    if (bytes <= cap) return buf;
    size_t want = std::max<size_t>(bytes, std::max<size_t>(2 * cap, 1 << 16));
    void *p = nullptr;
    if (hipHostMalloc(&p, want, hipHostMallocDefault) != hipSuccess) return nullptr;
    if (buf) (void)hipHostFree(buf);
    buf = p;
    cap = want;
    return buf;
}

hipError_t coop_launch(const void *fn, dim3 grid, dim3 block, void **args, size_t lds,
                       hipStream_t s) {
    // A ring of events per device: an event is re-recorded only long after
    // the waits on its previous recording were enqueued, and none is
    // destroyed while a stream may still wait on it.
    constexpr int kRing = 64;
    static std::mutex mu;
    static hipEvent_t ring[64][kRing] = {};
    static int next[64] = {};
    static bool any[64] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    const int prev = (next[dev] + kRing - 1) % kRing;
    if (any[dev]) {
        e = hipStreamWaitEvent(s, ring[dev][prev], 0);
        if (e != hipSuccess) return e;
    }
    e = hipLaunchCooperativeKernel(fn, grid, block, args, lds, s);
    if (e != hipSuccess) return e;
    hipEvent_t &ev = ring[dev][next[dev]];
    if (!ev) {
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) return e;
    }
    e = hipEventRecord(ev, s);
    if (e != hipSuccess) return e;
    next[dev] = (next[dev] + 1) % kRing;
    any[dev] = true;
    return hipSuccess;
}

}  // namespace ttsvd

using namespace ttsvd;

extern "C" {

const char *ttsvd_version(void) { return "libttsvd 0.1 (gfx950)"; }

const char *ttsvd_last_error(void) { return g_err; }

const char *ttsvd_strerror(int code) {
    switch (code) {
        case TTSVD_OK: return "success";
        case TTSVD_EINVAL: return "invalid argument";
        case TTSVD_ENOMEM: return "out of memory";
        case TTSVD_EHIP: return "HIP runtime error";
        case TTSVD_ENONFINITE: return "non-finite triangular factor";
        case TTSVD_EUNSUPPORTED: return "unsupported";
        default: return "unknown error";
    }
}

size_t ttsvd_tsqr_workspace_size(int dtype, int64_t rows, int64_t cols) {
    if (!valid_dtype(dtype) || rows < 1 || cols < 1 || cols > 1024) return 0;
    return tsqr_workspace_bytes(dtype, rows, cols);
}

int ttsvd_tsqr_r(const void *W, int dtype, int64_t rows, int64_t cols, int64_t ld, double *R,
                 int64_t ldr, void *ws, size_t ws_bytes, hipStream_t stream) {
    clear_error();
    if (!W || !R) return set_error(TTSVD_EINVAL, "tsqr_r: NULL pointer");
    if (rows < 1 || cols < 1 || ld < rows || ldr < cols)
        return set_error(TTSVD_EINVAL, "tsqr_r: bad sizes rows=%lld cols=%lld ld=%lld ldr=%lld",
                         (long long)rows, (long long)cols, (long long)ld, (long long)ldr);
    if (!valid_dtype(dtype)) return set_error(TTSVD_EUNSUPPORTED, "tsqr_r: dtype %d", dtype);
    if (cols > 1024) return set_error(TTSVD_EUNSUPPORTED, "tsqr_r: cols > 1024");
    const size_t need = tsqr_workspace_bytes(dtype, rows, cols);
    void *own = nullptr;
    if (!ws) {
        own = cache_acquire(need);
        if (!own) return set_error(TTSVD_ENOMEM, "tsqr_r: workspace of %zu bytes", need);
        ws = own;
        ws_bytes = need;
    } else if (ws_bytes < need) {
        return set_error(TTSVD_EINVAL, "tsqr_r: workspace %zu < %zu bytes", ws_bytes, need);
    }
    int rc = tsqr_launch(W, dtype, rows, cols, ld, R, ldr, ws, ws_bytes, stream);
    if (own) {
        // back to the cache once the launches before this point have run
        hipError_t e = cache_release_async(own, stream);
        if (e != hipSuccess) {
            (void)hipStreamSynchronize(stream);
            cache_release(own);
            if (rc == TTSVD_OK) rc = set_error(TTSVD_EHIP, "tsqr_r: release: %s", hipGetErrorString(e));
        }
    }
    return rc;
}

int ttsvd_gemm_reshape(const void *W, int dtype, int64_t rows, int64_t cols, int64_t ld,
                       const double *V, int64_t ldv, int64_t k, int64_t n_next, void *Y,
                       int64_t ld_y, hipStream_t stream) {
    clear_error();
    if (!W || !V || !Y) return set_error(TTSVD_EINVAL, "gemm_reshape: NULL pointer");
    if (rows < 1 || cols < 1 || k < 1 || n_next < 1 || ld < rows || ldv < cols)
        return set_error(TTSVD_EINVAL, "gemm_reshape: bad sizes");
    if (rows % n_next != 0) return set_error(TTSVD_EINVAL, "gemm_reshape: rows %% n_next != 0");
    if (ld_y < rows / n_next) return set_error(TTSVD_EINVAL, "gemm_reshape: ld_y < rows/n_next");
    if (cols > (int64_t(1) << 30)) return set_error(TTSVD_EUNSUPPORTED, "gemm_reshape: cols too large");
    if (k > 256) return set_error(TTSVD_EUNSUPPORTED, "gemm_reshape: k > 256");
    if (!valid_dtype(dtype)) return set_error(TTSVD_EUNSUPPORTED, "gemm_reshape: dtype %d", dtype);
    return tsmm_launch(W, dtype, rows, cols, ld, V, 1, ldv, k, n_next, Y, dtype, ld_y, stream);
}

size_t ttsvd_footprint_bytes(const int64_t *dims, int d, int64_t r_max, int dtype) {
    if (!dims || d < 1 || d > TTSVD_MAX_D || r_max < 1 || !valid_dtype(dtype)) return 0;
    std::vector<StepShape> steps;
    std::vector<int64_t> rb;
    int64_t nbar;
    if (plan_steps(dims, d, r_max, steps, rb, nbar) != TTSVD_OK) return 0;
    Footprint f = footprint(dims, d, dtype, steps, rb);
    return ws_layout(f, dtype_size(dtype)).total + align256(f.cores * 8);
}

void ttsvd_tt_free(ttsvd_tt *tt) {
    if (!tt) return;
    TTPriv *p = (TTPriv *)tt->priv;
    if (p) {
        if (p->cores_dev) result_free(p->cores_dev);
        if (p->shared && p->shared->refs.fetch_sub(1) == 1) {
            result_free(p->shared->ptr);
            delete p->shared;
        }
        for (double *s : p->sigma_host) free(s);
        delete p;
    }
    memset(tt, 0, sizeof(*tt));
}

// TTSVD_TSMM_QR=0 keeps the product and the next step's first TSQR level as
// separate launches (a tuning override; the results are the same).
static bool tsmm_qr_enabled() {
    static bool v = [] {
        const char *e = getenv("TTSVD_TSMM_QR");
        return !(e && atoi(e) == 0);
    }();
    return v;
}

static int decompose_impl(const ttsvd_tensor *X, const int64_t *dims, int d, int64_t r_max,
                          double tol, void *ws_in, size_t ws_bytes, double *cores_in,
                          size_t cores_doubles, ttsvd_tt *out) {
    clear_error();
    if (!X || !X->data || !dims || !out) return set_error(TTSVD_EINVAL, "decompose: NULL pointer");
    if (d < 1 || d > TTSVD_MAX_D) return set_error(TTSVD_EINVAL, "decompose: d = %d", d);
    if (r_max < 1) return set_error(TTSVD_EINVAL, "decompose: r_max < 1");
    if (!(tol >= 0.0) || !std::isfinite(tol)) return set_error(TTSVD_EINVAL, "decompose: tol");
    if (!valid_dtype(X->dtype)) return set_error(TTSVD_EUNSUPPORTED, "decompose: dtype %d", X->dtype);
    std::vector<StepShape> steps;
    std::vector<int64_t> rb;
    int64_t nbar;
    int rc = plan_steps(dims, d, r_max, steps, rb, nbar);
    if (rc != TTSVD_OK) return rc;
    const int64_t lead = nbar / dims[d - 1];
    const int64_t ld0 = X->ld_last ? X->ld_last : lead;
    if (ld0 < lead) return set_error(TTSVD_EINVAL, "decompose: ld_last < n_1...n_{d-1}");
    for (int i = d - 1; i >= 1; --i)
        if (steps[i].m > 1024)
            return set_error(TTSVD_EUNSUPPORTED, "decompose: step with %lld > 1024 columns",
                             (long long)steps[i].m);

    const int dt = X->dtype;
    const size_t es = dtype_size(dt);
    Footprint f = footprint(dims, d, dt, steps, rb);
    const WsLayout lay = ws_layout(f, es);
    if (ws_in && ws_bytes < lay.total)
        return set_error(TTSVD_EINVAL, "decompose: workspace %zu < %zu bytes", ws_bytes, lay.total);
    if (ws_in && ((uintptr_t)ws_in & 255))
        return set_error(TTSVD_EINVAL, "decompose: workspace not 256-byte aligned");
    if (cores_in && cores_doubles < f.cores)
        return set_error(TTSVD_EINVAL, "decompose: core buffer %zu < %zu doubles", cores_doubles,
                         f.cores);

    memset(out, 0, sizeof(*out));
    const hipStream_t s = X->stream;

    TTPriv *priv = new TTPriv();
    out->priv = priv;
    out->d = d;
    for (int i = 0; i < d; ++i) out->dims[i] = dims[i];

    double *cores_base = cores_in;
    if (!cores_base) {
        priv->cores_dev = (double *)result_alloc(std::max<size_t>(f.cores, 1) * 8);
        if (!priv->cores_dev) {
            ttsvd_tt_free(out);
            return set_error(TTSVD_ENOMEM, "decompose: cores (%zu doubles)", f.cores);
        }
        cores_base = priv->cores_dev;
    }
    for (int i = 0; i < d; ++i) out->cores[i] = cores_base + f.core_off[i];

    // One workspace for everything temporary: the caller's, or a library
    // cache block released before returning (after the stream is synchronised).
    char *ws = (char *)ws_in;
    const bool own_ws = (ws == nullptr);
    if (own_ws) ws = (char *)cache_acquire(lay.total);
    if (own_ws && !ws) {
        ttsvd_tt_free(out);
        return set_error(TTSVD_ENOMEM, "decompose: workspace of %zu bytes", lay.total);
    }
    void *wbuf[2] = {ws + lay.w0, ws + lay.w1};
    double *Rbuf = (double *)(ws + lay.r);
    void *tq = ws + lay.tq;
    void *sv = ws + lay.sv;
    double *sig_dev = (double *)(ws + lay.sg);
    DecompState *state = (DecompState *)(ws + lay.st);
    DecompState hstate;
    memset(&hstate, 0, sizeof(hstate));
    hstate.one = 1.0;

#define TTSVD_STEP_TRY(expr)                  \
    do {                                      \
        int rc_ = (expr);                     \
        if (rc_ != TTSVD_OK) {                \
            (void)hipStreamSynchronize(s);    \
            if (own_ws) cache_release(ws);    \
            ttsvd_tt_free(out);               \
            return rc_;                       \
        }                                     \
    } while (0)
#define TTSVD_STEP_HIP(expr)                                                            \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            TTSVD_STEP_TRY(set_error(TTSVD_EHIP, "%s: %s", #expr, hipGetErrorString(e_))); \
    } while (0)

    TTSVD_STEP_HIP(hipMemcpyAsync(state, &hstate, sizeof(hstate), hipMemcpyHostToDevice, s));

    std::vector<int64_t> ranks(d + 1, 1);
    if (d == 1) {
        TTSVD_STEP_TRY(tsmm_launch(X->data, dt, dims[0], 1, dims[0], &state->one, 1, 1, 1, 1,
                                   out->cores[0], TTSVD_F64, dims[0], s));
    } else {
        const void *Wcur = X->data;
        int64_t ld = ld0;
        int64_t nb = nbar;
        int pp = 0;
        int pre_levels = 0;  // levels of this step's TSQR done with the previous product
        for (int i = d - 1; i >= 1; --i) {
            const int64_t m = dims[i] * ranks[i + 1];
            const int64_t rows = nb / m;
            const int64_t K = std::min(rows, m);
            // R from the QR decomposition of W^(i).  A wide FP64 unfolding
            // (rows <= m) goes to the SVD as it is: its rows have the singular
            // values and right singular vectors of R, and the Jacobi SVD
            // orthogonalises rows, so the QR would only add a launch.
            const bool wide = dt == TTSVD_F64 && rows <= m;
            if (pre_levels)  // level 0 came with the previous product
                TTSVD_STEP_TRY(tsqr_launch_after_first(dt, rows, m, Rbuf, m, tq, f.tsqr_ws, s));
            else if (!wide)
                TTSVD_STEP_TRY(tsqr_launch(Wcur, dt, rows, m, ld, Rbuf, m, tq, f.tsqr_ws, s));
            // small SVD, rank, core T^(i)
            TTSVD_STEP_TRY(svd_launch(wide ? (const double *)Wcur : Rbuf, wide ? ld : m, K, m,
                                      sig_dev + f.sigma_off[i], out->cores[i], r_max, tol, d - 1,
                                      i == d - 1, &state->step[i], &state->step[d - 1], sv,
                                      f.svd_ws, s));
            int64_t r;
            if (tol == 0.0) {
                r = std::min(r_max, K);
            } else {
                StepState *stage = (StepState *)pinned_stage(sizeof(StepState));
                if (!stage) TTSVD_STEP_TRY(set_error(TTSVD_ENOMEM, "decompose: pinned staging"));
                TTSVD_STEP_HIP(hipMemcpyAsync(stage, &state->step[i], sizeof(StepState), hipMemcpyDeviceToHost, s));
                TTSVD_STEP_HIP(hipStreamSynchronize(s));
                const StepState hs = *stage;
                if (hs.nonfinite)
                    TTSVD_STEP_TRY(set_error(TTSVD_ENONFINITE, "decompose: non-finite sigma in step %d", i + 1));
                r = hs.rank;
                if (r < 1 || r > std::min(r_max, K))
                    TTSVD_STEP_TRY(set_error(TTSVD_EHIP, "decompose: step %d: device reported rank %lld (K = %lld)",
                                             i + 1, (long long)r, (long long)K));
            }
            ranks[i] = r;
            // W^(i-1) = reshape(W^(i) V_{:,1:r}); the last product is core T^(1)
            const int64_t n_next = dims[i - 1];
            void *Y = (i >= 2) ? wbuf[pp] : (void *)out->cores[0];
            const int ydt = (i >= 2) ? dt : TTSVD_F64;
            const int64_t ld_y = rows / n_next;
            pre_levels = 0;
            if (i >= 2 && tsmm_qr_enabled() && tsmm_qr_applies(dt, rows, m, r, n_next))
                TTSVD_STEP_TRY(tsmm_qr_launch(Wcur, dt, rows, m, ld, out->cores[i], r, 1, r, n_next,
                                              Y, Rbuf, n_next * r, tq, f.tsqr_ws, s, &pre_levels));
            else
                TTSVD_STEP_TRY(tsmm_launch(Wcur, dt, rows, m, ld, out->cores[i], r, 1, r, n_next, Y,
                                           ydt, ld_y, s));
            Wcur = Y;
            ld = ld_y;
            nb = rows * r;
            pp ^= 1;
        }
    }

    const size_t stage_bytes = align256(sizeof(hstate)) + f.sigma * 8;
    char *stage = (char *)pinned_stage(stage_bytes);
    if (!stage) TTSVD_STEP_TRY(set_error(TTSVD_ENOMEM, "decompose: pinned staging"));
    TTSVD_STEP_HIP(hipMemcpyAsync(stage, state, sizeof(hstate), hipMemcpyDeviceToHost, s));
    if (f.sigma)
        TTSVD_STEP_HIP(hipMemcpyAsync(stage + align256(sizeof(hstate)), sig_dev, f.sigma * 8,
                                      hipMemcpyDeviceToHost, s));
    TTSVD_STEP_HIP(hipStreamSynchronize(s));
    if (own_ws) cache_release(ws);
    memcpy(&hstate, stage, sizeof(hstate));
    std::vector<double> sig_host(std::max<size_t>(f.sigma, 1));
    if (f.sigma) memcpy(sig_host.data(), stage + align256(sizeof(hstate)), f.sigma * 8);
    // the ranks the device reports must be the ones the steps ran with
    for (int i = d - 1; i >= 1; --i)
        if (hstate.step[i].rank != ranks[i]) {
            (void)hipStreamSynchronize(s);
            ttsvd_tt_free(out);
            return set_error(TTSVD_EHIP, "decompose: step %d: device reported rank %lld, ran with %lld",
                             i + 1, (long long)hstate.step[i].rank, (long long)ranks[i]);
        }

    double disc_sum = 0.0;
    for (int i = d - 1; i >= 1; --i) {
        const StepState &st = hstate.step[i];
        if (st.nonfinite) {
            (void)hipStreamSynchronize(s);
            ttsvd_tt_free(out);
            return set_error(TTSVD_ENONFINITE, "decompose: non-finite sigma in step %d", i + 1);
        }
        ranks[i] = st.rank;
        out->discarded2[i] = st.discarded2;
        disc_sum += st.discarded2;
        const int64_t K = steps[i].K;  // K only depends on ranks to the right
        double *h = (double *)malloc(sizeof(double) * (size_t)K);
        if (!h) {
            ttsvd_tt_free(out);
            return set_error(TTSVD_ENOMEM, "decompose: host sigma");
        }
        priv->sigma_host.push_back(h);
        out->sigma[i] = h;
        out->nsigma[i] = 0;
    }
    // Recompute K from the actual ranks (tol > 0 can shrink later steps).
    {
        int64_t nb = nbar;
        for (int i = d - 1; i >= 1; --i) {
            const int64_t m = dims[i] * ranks[i + 1];
            const int64_t rows = nb / m;
            const int64_t K = std::min(rows, m);
            memcpy(out->sigma[i], sig_host.data() + f.sigma_off[i], sizeof(double) * (size_t)K);
            out->nsigma[i] = K;
            nb = rows * ranks[i];
        }
    }
    for (int i = 0; i <= d; ++i) out->ranks[i] = ranks[i];
    if (getenv("TTSVD_DEBUG")) {
        for (int i = d - 1; i >= 1; --i)
            fprintf(stderr, "[ttsvd] step %d: m=%lld rank=%lld sweeps=%lld discarded2=%.3e\n", i + 1,
                    (long long)(dims[i] * ranks[i + 1]), (long long)ranks[i],
                    (long long)hstate.step[i].sweeps, hstate.step[i].discarded2);
    }
    out->norm_sigma = std::sqrt(hstate.step[d - 1 >= 1 ? d - 1 : 0].norm2);
    out->delta = std::sqrt(hstate.step[d - 1 >= 1 ? d - 1 : 0].delta2);
    out->err_bound = std::sqrt(disc_sum);
    (void)hipStreamSynchronize(s);
    return TTSVD_OK;
#undef TTSVD_STEP_TRY
#undef TTSVD_STEP_HIP
}

size_t ttsvd_workspace_size(const int64_t *dims, int d, int64_t r_max, int dtype) {
    if (!dims || d < 1 || d > TTSVD_MAX_D || r_max < 1 || !valid_dtype(dtype)) return 0;
    std::vector<StepShape> steps;
    std::vector<int64_t> rb;
    int64_t nbar;
    if (plan_steps(dims, d, r_max, steps, rb, nbar) != TTSVD_OK) return 0;
    return ws_layout(footprint(dims, d, dtype, steps, rb), dtype_size(dtype)).total;
}

size_t ttsvd_cores_size(const int64_t *dims, int d, int64_t r_max) {
    if (!dims || d < 1 || d > TTSVD_MAX_D || r_max < 1) return 0;
    std::vector<StepShape> steps;
    std::vector<int64_t> rb;
    int64_t nbar;
    if (plan_steps(dims, d, r_max, steps, rb, nbar) != TTSVD_OK) return 0;
    return footprint(dims, d, TTSVD_F64, steps, rb).cores;
}

int ttsvd_decompose(const ttsvd_tensor *X, const int64_t *dims, int d, int64_t r_max, double tol,
                    ttsvd_tt *out) {
    return decompose_impl(X, dims, d, r_max, tol, nullptr, 0, nullptr, 0, out);
}

int ttsvd_decompose_ws(const ttsvd_tensor *X, const int64_t *dims, int d, int64_t r_max,
                       double tol, void *ws, size_t ws_bytes, double *cores,
                       size_t cores_doubles, ttsvd_tt *out) {
    clear_error();
    if (!ws || !cores) return set_error(TTSVD_EINVAL, "decompose_ws: NULL workspace or cores");
    return decompose_impl(X, dims, d, r_max, tol, ws, ws_bytes, cores, cores_doubles, out);
}

}  // extern "C"
