// Two-sided TSQR TT-SVD (Algorithm 4, Sec. 3.1.3): steps alternate between
// the right-most and the left-most remaining mode (i = d, 1, d-1, 2, ...).
// A right step is the step of Algorithm 2.  A left step needs the QR of the
// transposed left unfolding L^T (rest x r n); its SVD R = U S V^T gives
// L = V S (Q U)^T, so the left core is V_r and the remainder is
// (L^T V_r)^T.  Between steps the remainder is reordered by a transpose
// kernel (the reshape/transpose lines of Algorithm 4): after a right step
// into the layout whose tall-skinny matrix is L^T, after a left step back
// into the layout of the right unfolding.  The TSQR, small SVD and TSMM are
// the kernels of Algorithm 2.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"
#include "driver.h"
#include "kernels.h"
#include "profile.h"

namespace ttsvd {
namespace {

// out (Q x P, column-major) = in (P x Q, column-major)^T.  Tiles of 32 x 32
// through LDS (one padding column against bank conflicts), 32 x 8 threads,
// each thread moving four elements; the tiles are numbered along one grid
// dimension (tile (bp, bq) is block bp + nbp bq).
template <typename E>
__global__ __launch_bounds__(256) void transpose_tiled(const E *__restrict__ in,
                                                       E *__restrict__ out, int64_t P,
                                                       int64_t Q, int64_t nbp) {
    __shared__ E tile[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int64_t bp = (int64_t)blockIdx.x % nbp, bq = (int64_t)blockIdx.x / nbp;
    const int64_t p0 = bp * 32, q0 = bq * 32;
#pragma unroll
    for (int k = 0; k < 32; k += 8) {
        const int64_t p = p0 + tx, q = q0 + ty + k;
        if (p < P && q < Q) tile[ty + k][tx] = in[p + P * q];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 32; k += 8) {
        const int64_t q = q0 + tx, p = p0 + ty + k;
        if (p < P && q < Q) out[q + Q * p] = tile[tx][ty + k];
    }
}

// The same for P <= 16 (the short side of a left unfolding): thread q reads
// the P consecutive elements of column q and writes element q of each output
// column (consecutive threads, consecutive addresses).
template <typename E, int PM>
__global__ __launch_bounds__(256) void transpose_short_p(const E *__restrict__ in,
                                                         E *__restrict__ out, int P, int64_t Q) {
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < Q;
         q += (int64_t)gridDim.x * 256) {
        E v[PM];
#pragma unroll
        for (int p = 0; p < PM; ++p)
            if (p < P) v[p] = in[p + (int64_t)P * q];
#pragma unroll
        for (int p = 0; p < PM; ++p)
            if (p < P) out[q + Q * p] = v[p];
    }
}

// ... and for Q <= 16 (a tall remainder of rank r): thread p reads element p
// of each of the Q columns and writes its Q consecutive outputs.
template <typename E, int QM>
__global__ __launch_bounds__(256) void transpose_short_q(const E *__restrict__ in,
                                                         E *__restrict__ out, int64_t P, int Q) {
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < P;
         p += (int64_t)gridDim.x * 256) {
        E v[QM];
#pragma unroll
        for (int q = 0; q < QM; ++q)
            if (q < Q) v[q] = in[p + P * q];
#pragma unroll
        for (int q = 0; q < QM; ++q)
            if (q < Q) out[q + (int64_t)Q * p] = v[q];
    }
}

template <typename E>
int transpose_e(const void *in, void *out, int64_t P, int64_t Q, hipStream_t s) {
    if (P <= 16) {
        const unsigned blocks = (unsigned)std::min<int64_t>(ceil_div(Q, 256), 8192);
        hipLaunchKernelGGL((transpose_short_p<E, 16>), dim3(blocks), dim3(256), 0, s,
                           (const E *)in, (E *)out, (int)P, Q);
    } else if (Q <= 16) {
        const unsigned blocks = (unsigned)std::min<int64_t>(ceil_div(P, 256), 8192);
        hipLaunchKernelGGL((transpose_short_q<E, 16>), dim3(blocks), dim3(256), 0, s,
                           (const E *)in, (E *)out, P, (int)Q);
    } else {
        const int64_t nbp = ceil_div(P, 32), nb = nbp * ceil_div(Q, 32);
        if (nb > INT32_MAX) return set_error(TTSVD_EUNSUPPORTED, "transpose: %lld tiles", (long long)nb);
        hipLaunchKernelGGL((transpose_tiled<E>), dim3((unsigned)nb), dim3(256), 0, s,
                           (const E *)in, (E *)out, P, Q, nbp);
    }
    TTSVD_HIP_TRY(hipGetLastError());
    return TTSVD_OK;
}

// Transpose of a P x Q column-major matrix of `es`-byte elements.
int transpose_launch(const void *in, void *out, int64_t P, int64_t Q, size_t es, hipStream_t s) {
    char name[64];
    snprintf(name, sizeof(name), "transpose<%zu bytes>", es);
    prof_begin(s, name, 2.0 * (double)P * (double)Q * (double)es, 0.0);
    int rc;
    if (es == 8)
        rc = transpose_e<uint64_t>(in, out, P, Q, s);
    else if (es == 4)
        rc = transpose_e<uint32_t>(in, out, P, Q, s);
    else
        rc = transpose_e<uint16_t>(in, out, P, Q, s);
    prof_end(s);
    return rc;
}

// Per-step device buffers, taken from the library cache and returned after
// the step has synchronised.
struct StepBufs {
    void *p[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    ~StepBufs() {
        for (void *q : p) cache_release(q);
    }
};

}  // namespace
}  // namespace ttsvd

using namespace ttsvd;

extern "C" {

int ttsvd_decompose_two_sided(const ttsvd_tensor *X, const int64_t *dims, int d, int64_t r_max,
                              double tol, ttsvd_tt *out) {
    clear_error();
    if (!X || !X->data || !dims || !out) return set_error(TTSVD_EINVAL, "two_sided: NULL pointer");
    if (d < 1 || d > TTSVD_MAX_D) return set_error(TTSVD_EINVAL, "two_sided: d = %d", d);
    if (r_max < 1) return set_error(TTSVD_EINVAL, "two_sided: r_max < 1");
    if (!(tol >= 0.0) || !std::isfinite(tol)) return set_error(TTSVD_EINVAL, "two_sided: tol");
    if (!valid_dtype(X->dtype)) return set_error(TTSVD_EUNSUPPORTED, "two_sided: dtype %d", X->dtype);
    const int dt = X->dtype;
    const size_t es = dtype_size(dt);
    int64_t nbar = 1;
    for (int i = 0; i < d; ++i) {
        if (dims[i] < 1) return set_error(TTSVD_EINVAL, "two_sided: dims[%d] < 1", i);
        if (nbar > (int64_t(1) << 62) / dims[i]) return set_error(TTSVD_EINVAL, "two_sided: size overflow");
        nbar *= dims[i];
    }
    if (X->ld_last && X->ld_last != nbar / dims[d - 1])
        return set_error(TTSVD_EUNSUPPORTED, "two_sided: padded last-mode stride");
    if (d <= 2) return ttsvd_decompose(X, dims, d, r_max, tol, out);  // one right step: Algorithm 2

    // Shapes at the rank upper bounds: every step has at most 1024 columns and
    // keeps at most 256 (the limits of the TSQR and TSMM kernels); core sizes.
    std::vector<int64_t> rb(d + 1, 1), core_off(d + 1, 0);
    {
        int lo = 0, hi = d - 1;
        bool right = true;
        int64_t size = nbar;
        while (lo < hi) {
            const int64_t m = right ? dims[hi] * rb[hi + 1] : rb[lo] * dims[lo];
            const int64_t rows = size / m;
            const int64_t r = std::min<int64_t>(r_max, std::min(rows, m));
            if (m > 1024 || r > 256)
                return set_error(TTSVD_EUNSUPPORTED, "two_sided: step with %lld columns, rank %lld",
                                 (long long)m, (long long)r);
            if (right) rb[hi--] = r;
            else rb[++lo] = r;
            size = rows * r;
            right = !right;
        }
        for (int i = 0; i < d; ++i) core_off[i + 1] = core_off[i] + rb[i] * dims[i] * rb[i + 1];
    }
    const hipStream_t s = X->stream;
    memset(out, 0, sizeof(*out));
    TTPriv *priv = new TTPriv();
    out->priv = priv;
    out->d = d;
    for (int i = 0; i < d; ++i) out->dims[i] = dims[i];
    out->ranks[0] = out->ranks[d] = 1;
    priv->cores_dev = (double *)result_alloc((size_t)core_off[d] * 8);
    void *bufA = cache_acquire((size_t)nbar * es), *bufB = cache_acquire((size_t)nbar * es);
    StepState *state = (StepState *)cache_acquire(sizeof(StepState) * (size_t)d);
    StepState *hstate = (StepState *)pinned_stage(sizeof(StepState) + 1024 * 8);
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(s);
        cache_release(bufA);
        cache_release(bufB);
        cache_release(state);
    };
    auto fail = [&](int code) {
        cleanup();
        ttsvd_tt_free(out);
        return code;
    };
    if (!priv->cores_dev || !bufA || !bufB || !state || !hstate)
        return fail(set_error(TTSVD_ENOMEM, "two_sided: buffers"));
    if (hipMemsetAsync(state, 0, sizeof(StepState) * (size_t)d, s) != hipSuccess)
        return fail(set_error(TTSVD_EHIP, "two_sided: state"));
    double *sig_stage = (double *)(hstate + 1);

    const void *cur = X->data;  // input of the next step, tall-skinny, column-major
    int lo = 0, hi = d - 1;
    bool right = true;
    int64_t size = nbar;
    double disc = 0.0;
    while (lo < hi) {
        const int bond = right ? hi : lo + 1;
        const int64_t m = right ? dims[hi] * out->ranks[hi + 1] : out->ranks[lo] * dims[lo];
        const int64_t rows = size / m;
        const int64_t K = std::min(rows, m);
        const bool last = (right ? hi - 1 : lo + 1) == (right ? lo : hi);
        StepBufs sb;
        const size_t tq_bytes = tsqr_workspace_bytes(dt, rows, m);
        const size_t sv_bytes = std::max<size_t>(svd_scratch_bytes(K, m), 8);
        sb.p[0] = cache_acquire((size_t)(m * m) * 8);          // R
        sb.p[1] = cache_acquire(tq_bytes);                     // TSQR tree
        sb.p[2] = cache_acquire(sv_bytes);                     // SVD scratch
        sb.p[3] = cache_acquire((size_t)(K * m) * 8);          // V_r^T (r x m)
        sb.p[4] = cache_acquire((size_t)K * 8);                // sigma
        if (!sb.p[0] || !sb.p[1] || !sb.p[2] || !sb.p[3] || !sb.p[4])
            return fail(set_error(TTSVD_ENOMEM, "two_sided: step buffers"));
        double *R = (double *)sb.p[0], *Vt = (double *)sb.p[3], *sig = (double *)sb.p[4];
        int rc = tsqr_launch(cur, dt, rows, m, rows, R, m, sb.p[1], tq_bytes, s);
        if (rc != TTSVD_OK) return fail(rc);
        // V_r^T: for a right step directly the core (r, n_hi, r_{hi+1})
        double *core_rt = right ? priv->cores_dev + core_off[hi] : Vt;
        rc = svd_launch(R, m, K, m, sig, core_rt, r_max, tol, d - 1, bond == d - 1,
                        &state[bond], &state[d - 1], sb.p[2], sv_bytes, s);
        if (rc != TTSVD_OK) return fail(rc);
        if (hipMemcpyAsync(hstate, &state[bond], sizeof(StepState), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(sig_stage, sig, (size_t)K * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return fail(set_error(TTSVD_EHIP, "two_sided: step state"));
        const StepState hs = *hstate;
        if (hs.nonfinite) return fail(set_error(TTSVD_ENONFINITE, "two_sided: non-finite sigma"));
        const int64_t r = hs.rank;
        if (r < 1 || r > std::min(r_max, K))
            return fail(set_error(TTSVD_EHIP, "two_sided: device reported rank %lld", (long long)r));
        double *hsig = (double *)malloc(sizeof(double) * (size_t)K);
        if (!hsig) return fail(set_error(TTSVD_ENOMEM, "two_sided: host sigma"));
        memcpy(hsig, sig_stage, sizeof(double) * (size_t)K);
        priv->sigma_host.push_back(hsig);
        out->sigma[bond] = hsig;
        out->nsigma[bond] = K;
        out->discarded2[bond] = hs.discarded2;
        disc += hs.discarded2;
        out->ranks[bond] = r;
        if (bond == d - 1) {
            out->norm_sigma = std::sqrt(hs.norm2);
            out->delta = std::sqrt(hs.delta2);
        }
        if (!right) {
            // left core T^(lo) = reshape(V_r, (r_lo, n_lo, r)): V_r = (V_r^T)^T
            out->cores[lo] = priv->cores_dev + core_off[lo];
            rc = transpose_launch(Vt, out->cores[lo], r, m, 8, s);
            if (rc != TTSVD_OK) return fail(rc);
        } else {
            out->cores[hi] = priv->cores_dev + core_off[hi];
        }
        // Wbar = W V_r (rows x r); V(c, a) = V_r^T[a + r c]
        const double *Vsrc = right ? out->cores[hi] : Vt;
        if (last) {
            // the middle core: d even ends with a right step (core = Wbar),
            // d odd with a left step (core = Wbar^T)
            const int mid = right ? hi - 1 : lo + 1;
            out->cores[mid] = priv->cores_dev + core_off[mid];
            double *dst = right ? out->cores[mid] : (double *)bufA;
            rc = tsmm_launch(cur, dt, rows, m, rows, Vsrc, r, 1, r, 1, dst, TTSVD_F64, rows, s);
            if (rc == TTSVD_OK && !right) rc = transpose_launch(bufA, out->cores[mid], rows, r, 8, s);
            if (rc != TTSVD_OK) return fail(rc);
        } else {
            rc = tsmm_launch(cur, dt, rows, m, rows, Vsrc, r, 1, r, 1, bufA, dt, rows, s);
            if (rc != TTSVD_OK) return fail(rc);
            // reorder for the other side: after a right step the remainder
            // (r_lo n_lo) x rest becomes its transpose; after a left step the
            // rows x r matrix Wbar becomes r x rows
            if (right)
                rc = transpose_launch(bufA, bufB, out->ranks[lo] * dims[lo], rows * r /
                                      (out->ranks[lo] * dims[lo]), es, s);
            else
                rc = transpose_launch(bufA, bufB, rows, r, es, s);
            if (rc != TTSVD_OK) return fail(rc);
            cur = bufB;
        }
        if (hipStreamSynchronize(s) != hipSuccess)
            return fail(set_error(TTSVD_EHIP, "two_sided: step %d", bond));
        size = rows * r;
        if (right) --hi;
        else ++lo;
        right = !right;
    }
    out->err_bound = std::sqrt(disc);
    cleanup();
    return TTSVD_OK;
}

}  // extern "C"
