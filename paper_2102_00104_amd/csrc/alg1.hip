// Algorithm 1 (the original TT-SVD, Sec. 3.1.1) on the GPU, as an in-house
// comparator for the QR trick of Algorithm 2: every step takes the full SVD
// of the unfolding W^(i) itself -- rocSOLVER's GESVD with its QR
// preprocessing switched off (in-place mode), so no triangular factor is
// formed -- chooses the rank with delta = eps/sqrt(d-1) ||X||_F, and continues
// with W <- reshape(U_r Sigma_r).  Measurement infrastructure, not the
// product path (ttsvd_decompose).
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"
#include "driver.h"

namespace ttsvd {
namespace {

constexpr double kAlg1SigmaFloor = 1e-150;

// W(:, a) *= sigma[a] for a < r (rows x r, column-major, leading dimension ld).
__global__ void scale_columns(double *__restrict__ W, int64_t ld, int64_t rows, int64_t r,
                              const double *__restrict__ sigma) {
    const int64_t n = rows * r;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = i / rows, row = i - a * rows;
        W[row + ld * a] *= sigma[a];
    }
}

// The rank rule of Algorithm 1: r = min(r_max, r_delta) clamped to [1, K]
// with r_delta the smallest j such that the tail sigma_{j+1}^2 + ... is at
// most delta^2 (tails summed from the smallest value); tol = 0: min(r_max, K).
int64_t rank_rule(const double *s, int64_t K, int64_t r_max, double tol, double delta2,
                  double *discarded2) {
    int64_t r;
    if (tol == 0.0) {
        r = std::min<int64_t>(r_max, K);
    } else {
        int64_t r_delta = K;
        double acc = 0.0;
        for (int64_t i = K - 1; i >= 0; --i) {
            const double se = s[i] > kAlg1SigmaFloor ? s[i] : 0.0;
            acc = std::fma(se, se, acc);
            if (acc <= delta2)
                r_delta = i;
            else
                break;
        }
        r = std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(r_max, r_delta), K));
    }
    double disc = 0.0;
    for (int64_t i = K - 1; i >= r; --i) {
        const double se = s[i] > kAlg1SigmaFloor ? s[i] : 0.0;
        disc = std::fma(se, se, disc);
    }
    *discarded2 = disc;
    return r;
}

struct Alg1Buffers {
    void *A = nullptr, *Vt = nullptr, *S = nullptr, *E = nullptr, *info = nullptr;
    rocblas_handle h = nullptr;
    ~Alg1Buffers() {
        cache_release(A);
        cache_release(Vt);
        cache_release(S);
        cache_release(E);
        cache_release(info);
        if (h) (void)rocblas_destroy_handle(h);
    }
};

}  // namespace
}  // namespace ttsvd

using namespace ttsvd;

extern "C" {

int ttsvd_decompose_alg1(const ttsvd_tensor *X, const int64_t *dims, int d, int64_t r_max,
                         double tol, ttsvd_tt *out) {
    clear_error();
    if (!X || !X->data || !dims || !out) return set_error(TTSVD_EINVAL, "alg1: NULL pointer");
    if (d < 1 || d > TTSVD_MAX_D) return set_error(TTSVD_EINVAL, "alg1: d = %d", d);
    if (r_max < 1) return set_error(TTSVD_EINVAL, "alg1: r_max < 1");
    if (!(tol >= 0.0) || !std::isfinite(tol)) return set_error(TTSVD_EINVAL, "alg1: tol");
    if (X->dtype != TTSVD_F64) return set_error(TTSVD_EUNSUPPORTED, "alg1: FP64 tensors only");
    int64_t nbar = 1;
    for (int i = 0; i < d; ++i) {
        if (dims[i] < 1) return set_error(TTSVD_EINVAL, "alg1: dims[%d] < 1", i);
        if (nbar > (int64_t(1) << 62) / dims[i]) return set_error(TTSVD_EINVAL, "alg1: size overflow");
        nbar *= dims[i];
    }
    if (X->ld_last && X->ld_last != nbar / dims[d - 1])
        return set_error(TTSVD_EUNSUPPORTED, "alg1: padded last-mode stride");
    // every GESVD operand must be addressable with 32-bit rocSOLVER sizes
    {
        int64_t nb = nbar, rn = 1;
        for (int i = d - 1; i >= 1; --i) {
            const int64_t m = dims[i] * rn;
            const int64_t rows = nb / m;
            if (rows > INT32_MAX || m > 4096)
                return set_error(TTSVD_EUNSUPPORTED, "alg1: unfolding %lld x %lld too large",
                                 (long long)rows, (long long)m);
            rn = std::min<int64_t>(r_max, std::min(rows, m));
            nb = rows * rn;
        }
    }
    const hipStream_t s = X->stream;
    memset(out, 0, sizeof(*out));
    TTPriv *priv = new TTPriv();
    out->priv = priv;
    out->d = d;
    for (int i = 0; i < d; ++i) out->dims[i] = dims[i];
    out->ranks[0] = out->ranks[d] = 1;

    auto fail = [&](int code, const char *what) {
        (void)hipStreamSynchronize(s);
        ttsvd_tt_free(out);
        return set_error(code, "alg1: %s", what);
    };

    // Core storage for the rank upper bounds, and the work buffers.
    std::vector<int64_t> rb(d + 1, 1), core_off(d + 1, 0);
    size_t kmax = 1, mmax = 1;
    {
        int64_t nb = nbar;
        for (int i = d - 1; i >= 1; --i) {
            const int64_t m = dims[i] * rb[i + 1];
            const int64_t rows = nb / m;
            const int64_t K = std::min(rows, m);
            rb[i] = std::min<int64_t>(r_max, K);
            kmax = std::max<size_t>(kmax, (size_t)K);
            mmax = std::max<size_t>(mmax, (size_t)m);
            nb = rows * rb[i];
        }
        for (int i = 0; i < d; ++i) core_off[i + 1] = core_off[i] + rb[i] * dims[i] * rb[i + 1];
    }
    priv->cores_dev = (double *)result_alloc((size_t)core_off[d] * 8);
    if (!priv->cores_dev) return fail(TTSVD_ENOMEM, "cores");
    Alg1Buffers bf;
    bf.A = cache_acquire((size_t)nbar * 8);
    bf.Vt = cache_acquire(kmax * mmax * 8);
    bf.S = cache_acquire(kmax * 8);
    bf.E = cache_acquire(kmax * 8);
    bf.info = cache_acquire(sizeof(rocblas_int));
    if (!bf.A || !bf.Vt || !bf.S || !bf.E || !bf.info) return fail(TTSVD_ENOMEM, "work buffers");
    if (rocblas_create_handle(&bf.h) != rocblas_status_success ||
        rocblas_set_stream(bf.h, s) != rocblas_status_success)
        return fail(TTSVD_EHIP, "rocblas handle");
    double *A = (double *)bf.A;
    if (hipMemcpyAsync(A, X->data, (size_t)nbar * 8, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return fail(TTSVD_EHIP, "input copy");

    if (d == 1) {
        out->cores[0] = priv->cores_dev;
        if (hipMemcpyAsync(out->cores[0], A, (size_t)nbar * 8, hipMemcpyDeviceToDevice, s) !=
                hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return fail(TTSVD_EHIP, "d = 1 copy");
        return TTSVD_OK;
    }

    std::vector<double> hs(kmax);
    double delta2 = 0.0, disc_total = 0.0;
    int64_t nb = nbar;
    for (int i = d - 1; i >= 1; --i) {
        const int64_t rn = out->ranks[i + 1];
        const int64_t m = dims[i] * rn;
        const int64_t rows = nb / m;
        const int64_t K = std::min(rows, m);
        // full SVD of the unfolding W^(i) (rows x m, column-major in A):
        // U overwrites A's first K columns, V^T goes to Vt (K x m)
        const rocblas_status st = rocsolver_dgesvd(
            bf.h, rocblas_svect_overwrite, rocblas_svect_singular, (rocblas_int)rows,
            (rocblas_int)m, A, (rocblas_int)rows, (double *)bf.S, nullptr, 1, (double *)bf.Vt,
            (rocblas_int)K, (double *)bf.E, rocblas_inplace, (rocblas_int *)bf.info);
        if (st != rocblas_status_success) return fail(TTSVD_EHIP, "rocsolver_dgesvd");
        rocblas_int hinfo = 0;
        if (hipMemcpyAsync(hs.data(), bf.S, (size_t)K * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(&hinfo, bf.info, sizeof(hinfo), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return fail(TTSVD_EHIP, "singular values");
        if (hinfo != 0) return fail(TTSVD_EHIP, "GESVD did not converge");
        for (int64_t k = 0; k < K; ++k)
            if (!std::isfinite(hs[k])) return fail(TTSVD_ENONFINITE, "non-finite singular value");
        if (i == d - 1) {
            // ||X||_F^2 = the sum of sigma^2 of the first unfolding
            double n2 = 0.0;
            for (int64_t k = K - 1; k >= 0; --k) n2 = std::fma(hs[k], hs[k], n2);
            out->norm_sigma = std::sqrt(n2);
            delta2 = (tol * tol / (double)(d - 1)) * n2;
            out->delta = std::sqrt(delta2);
        }
        double disc = 0.0;
        const int64_t r = rank_rule(hs.data(), K, r_max, tol, delta2, &disc);
        out->ranks[i] = r;
        out->discarded2[i] = disc;
        disc_total += disc;
        double *sig = (double *)malloc(sizeof(double) * (size_t)K);
        if (!sig) return fail(TTSVD_ENOMEM, "host sigma");
        memcpy(sig, hs.data(), sizeof(double) * (size_t)K);
        priv->sigma_host.push_back(sig);
        out->sigma[i] = sig;
        out->nsigma[i] = K;
        // core T^(i) = reshape(V_{:,1:r}^T, (r, n_i, r_i)): rows 0..r-1 of V^T
        out->cores[i] = priv->cores_dev + core_off[i];
        if (hipMemcpy2DAsync(out->cores[i], (size_t)r * 8, bf.Vt, (size_t)K * 8, (size_t)r * 8,
                             (size_t)m, hipMemcpyDeviceToDevice, s) != hipSuccess)
            return fail(TTSVD_EHIP, "core copy");
        // W^(i-1) = reshape(U_r Sigma_r): the first r columns of A, scaled
        const unsigned blocks = (unsigned)std::min<int64_t>(4096, ceil_div(rows * r, 256));
        hipLaunchKernelGGL(scale_columns, dim3(blocks), dim3(256), 0, s, A, rows, rows, r,
                           (const double *)bf.S);
        if (hipGetLastError() != hipSuccess) return fail(TTSVD_EHIP, "scale kernel");
        nb = rows * r;
    }
    // T^(1) = reshape(W^(1), (1, n_1, r_1))
    out->cores[0] = priv->cores_dev + core_off[0];
    if (hipMemcpyAsync(out->cores[0], A, (size_t)dims[0] * out->ranks[1] * 8,
                       hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(TTSVD_EHIP, "last core");
    out->err_bound = std::sqrt(disc_total);
    return TTSVD_OK;
}

}  // extern "C"
