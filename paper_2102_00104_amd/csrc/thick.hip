// Thick-bounds TT-SVD (Algorithm 3 of arXiv 2102.00104): Algorithm 2 on the
// tensor with its k right-most modes combined into one of size m, then the
// combined core split by a TT-SVD of its own.  Host orchestration only: both
// decompositions are ttsvd_decompose calls on device data, and the result is
// assembled with device-to-device copies on the caller's stream.
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "common.h"
#include "driver.h"

using namespace ttsvd;

extern "C" {

int ttsvd_thick_bounds_k(const int64_t *dims, int d, int64_t m_min, double f1_min,
                         int64_t r_est, int *k, int64_t *m) {
    clear_error();
    if (!dims || !k || !m) return set_error(TTSVD_EINVAL, "thick: NULL pointer");
    if (d < 1 || d > TTSVD_MAX_D || m_min < 1 || !(f1_min > 0.0 && f1_min <= 1.0) || r_est < 1)
        return set_error(TTSVD_EINVAL, "thick: bad arguments");
    // the first step shrinks the work array by f_1 = r / m: f_1 <= f1_min
    // for r ~ r_est asks for m >= r_est / f1_min
    const double need = fmax((double)m_min, (double)r_est / f1_min);
    int64_t p = 1;
    for (int kk = 1; kk <= d; ++kk) {
        const int64_t n = dims[d - kk];
        if (n < 1) return set_error(TTSVD_EINVAL, "thick: dims[%d] = %lld", d - kk, (long long)n);
        if (p > INT64_MAX / n) return set_error(TTSVD_EINVAL, "thick: product of dims overflows");
        p *= n;
        if ((double)p >= need || kk == d) {
            *k = kk;
            *m = p;
            return TTSVD_OK;
        }
    }
    return set_error(TTSVD_EINVAL, "thick: no modes");  // not reached for d >= 1
}

int ttsvd_decompose_thick(const ttsvd_tensor *X, const int64_t *dims, int d, int64_t r_max,
                          double tol, int64_t m_min, double f1_min, ttsvd_tt *out) {
    clear_error();
    if (!X || !X->data || !dims || !out) return set_error(TTSVD_EINVAL, "thick: NULL pointer");
    int k = 0;
    int64_t m = 0;
    int rc = ttsvd_thick_bounds_k(dims, d, m_min, f1_min, r_max < 1 ? 1 : r_max, &k, &m);
    if (rc != TTSVD_OK) return rc;
    if (k <= 1 || k >= d) return ttsvd_decompose(X, dims, d, r_max, tol, out);
    // Combining the last k modes reinterprets X as (n_1 ... n_{d-k}) x m only
    // when the last mode is stored without padding.
    int64_t lead = 1;
    for (int i = 0; i < d - 1; ++i) lead *= dims[i];
    if (X->ld_last != 0 && X->ld_last != lead)
        return set_error(TTSVD_EUNSUPPORTED,
                         "thick: a padded last-mode stride (ld_last = %lld) cannot be combined",
                         (long long)X->ld_last);

    // 1. Algorithm 2 on (n_1, ..., n_{d-k}, m): the same memory in Fortran order
    const int da = d - k + 1;
    int64_t dims_a[TTSVD_MAX_D];
    for (int i = 0; i < d - k; ++i) dims_a[i] = dims[i];
    dims_a[d - k] = m;
    ttsvd_tt A;
    rc = ttsvd_decompose(X, dims_a, da, r_max, tol, &A);
    if (rc != TTSVD_OK) return rc;

    // 2. TT-SVD of the combined core Tbar (r, m, 1) read as (r n_{d-k+1}, ..., n_d)
    const int64_t r = A.ranks[d - k];
    ttsvd_tensor C;
    memset(&C, 0, sizeof(C));
    C.data = A.cores[d - k];
    C.dtype = TTSVD_F64;
    C.ld_last = 0;
    C.stream = X->stream;
    int64_t dims_b[TTSVD_MAX_D];
    dims_b[0] = r * dims[d - k];
    for (int j = 1; j < k; ++j) dims_b[j] = dims[d - k + j];
    ttsvd_tt B;
    rc = ttsvd_decompose(&C, dims_b, k, r_max, tol, &B);
    if (rc != TTSVD_OK) {
        ttsvd_tt_free(&A);
        return rc;
    }

    // 3. One d-mode result: cores 1..d-k of A, then the k cores of B (B's
    //    first core (1, r n, r') is the core (r, n, r'): the same memory).
    memset(out, 0, sizeof(*out));
    TTPriv *priv = new TTPriv();
    out->priv = priv;
    out->d = d;
    for (int i = 0; i < d; ++i) out->dims[i] = dims[i];
    for (int i = 0; i <= d - k; ++i) out->ranks[i] = A.ranks[i];
    for (int j = 1; j <= k; ++j) out->ranks[d - k + j] = B.ranks[j];
    std::vector<size_t> off(d + 1, 0);
    for (int i = 0; i < d; ++i)
        off[i + 1] = off[i] + (size_t)(out->ranks[i] * out->dims[i] * out->ranks[i + 1]);
    const hipStream_t s = X->stream;
    priv->cores_dev = (double *)result_alloc(std::max<size_t>(off[d], 1) * sizeof(double));
    hipError_t e = priv->cores_dev ? hipSuccess : hipErrorOutOfMemory;
    for (int i = 0; i < d && e == hipSuccess; ++i) {
        out->cores[i] = priv->cores_dev + off[i];
        const double *src = i < d - k ? A.cores[i] : B.cores[i - (d - k)];
        e = hipMemcpyAsync(out->cores[i], src, (off[i + 1] - off[i]) * sizeof(double),
                           hipMemcpyDeviceToDevice, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        ttsvd_tt_free(out);
        ttsvd_tt_free(&A);
        ttsvd_tt_free(&B);
        return set_error(e == hipErrorOutOfMemory ? TTSVD_ENOMEM : TTSVD_EHIP,
                         "thick: assembling the cores: %s", hipGetErrorString(e));
    }
    // host singular values: move ownership from A and B
    for (int i = 1; i <= d - k; ++i) {
        out->sigma[i] = A.sigma[i];
        out->nsigma[i] = A.nsigma[i];
        out->discarded2[i] = A.discarded2[i];
    }
    for (int j = 1; j < k; ++j) {
        out->sigma[d - k + j] = B.sigma[j];
        out->nsigma[d - k + j] = B.nsigma[j];
        out->discarded2[d - k + j] = B.discarded2[j];
    }
    TTPriv *pa = (TTPriv *)A.priv, *pb = (TTPriv *)B.priv;
    priv->sigma_host = pa->sigma_host;
    priv->sigma_host.insert(priv->sigma_host.end(), pb->sigma_host.begin(), pb->sigma_host.end());
    pa->sigma_host.clear();
    pb->sigma_host.clear();
    out->delta = A.delta;
    out->norm_sigma = A.norm_sigma;
    const double s1 = A.nsigma[d - k] > 0 ? A.sigma[d - k][0] : 0.0;
    out->err_bound = A.err_bound + s1 * B.err_bound;
    ttsvd_tt_free(&A);
    ttsvd_tt_free(&B);
    return TTSVD_OK;
}

}  // extern "C"
