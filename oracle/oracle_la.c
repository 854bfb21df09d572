/*
 * Plain CPU FP64 linear-algebra primitives for the TT-SVD oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the HIP path is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product library never links or calls it, and it shares no code with it.
 *
 * What it implements, and where the paper defines it (arXiv 2102.00104):
 *   - oracle_qr_r:       the triangular factor R of W = QR (Section 2.1.1,
 *                        "Matrix decompositions"), computed by textbook
 *                        Householder reflections (Householder 1958, cited in
 *                        Section 3.2).  Q is discarded, as in Algorithm 2,
 *                        which only needs R.
 *   - oracle_jacobi_svd: the SVD  A = U diag(sigma) V^T  (Section 2.1.1) by
 *                        the one-sided Jacobi method of Hestenes (1958), the
 *                        SVD used by both TT-SVD algorithms (Algorithm 1 step
 *                        "calculate SVD", Algorithm 2 "small SVD").
 *
 * Both routines are written for clarity, not speed: no blocking, no
 * reordering beyond what the definitions state.  The only concession is an
 * OpenMP pragma over independent columns in the QR update, so the oracle can
 * be timed on all host cores.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/*
 * Householder QR of W (rows x cols, column-major, leading dimension ld).
 * Writes the upper-trapezoidal R (K x cols, K = min(rows, cols)) to R,
 * column-major with leading dimension K.  W is not modified.
 *
 * For column j the reflector H = I - tau v v^T (v[0] = 1) maps x = A[j:, j]
 * to beta e_1 with beta = -sign(x_0) ||x||, sign(0) = +1 (LAPACK dlarfg
 * convention).  An exactly zero column is left alone (tau = 0, R_jj = 0).
 */
void oracle_qr_r(const double *W, int64_t rows, int64_t cols, int64_t ld,
                 double *R)
{
    int64_t K = rows < cols ? rows : cols;
    double *A = (double *)malloc((size_t)rows * (size_t)cols * sizeof(double));
    double *v = (double *)malloc((size_t)rows * sizeof(double));
    for (int64_t k = 0; k < cols; ++k)
        memcpy(A + k * rows, W + k * ld, (size_t)rows * sizeof(double));

    for (int64_t j = 0; j < K; ++j) {
        double *x = A + j * rows + j;
        int64_t len = rows - j;
        double norm2 = 0.0;
        for (int64_t i = 0; i < len; ++i) norm2 += x[i] * x[i];
        double normx = sqrt(norm2);
        if (normx == 0.0) continue;                 /* tau = 0 */
        double x0 = x[0];
        double beta = (x0 >= 0.0) ? -normx : normx;
        double scale = 1.0 / (x0 - beta);
        v[0] = 1.0;
        for (int64_t i = 1; i < len; ++i) v[i] = x[i] * scale;
        double tau = (beta - x0) / beta;
        x[0] = beta;
        for (int64_t i = 1; i < len; ++i) x[i] = 0.0;
        #pragma omp parallel for schedule(static)
        for (int64_t k = j + 1; k < cols; ++k) {
            double *y = A + k * rows + j;
            double w = 0.0;
            for (int64_t i = 0; i < len; ++i) w += v[i] * y[i];
            w *= tau;
            for (int64_t i = 0; i < len; ++i) y[i] -= w * v[i];
        }
    }
    for (int64_t k = 0; k < cols; ++k)
        for (int64_t i = 0; i < K; ++i)
            R[i + k * K] = (i <= k) ? A[i + k * rows] : 0.0;
    free(v);
    free(A);
}

/*
 * One-sided Jacobi SVD (Hestenes) of A (rows x n, column-major, lda).
 *
 * Plane rotations J_pq are applied to the columns of a working copy B = A
 * (and accumulated in V = I) until every column pair is orthogonal to
 * working precision:  |b_p^T b_q| <= tol * ||b_p|| ||b_q||,
 * tol = sqrt(rows) * 2^-52 (cyclic by rows p < q, at most max_sweeps sweeps).
 * Then sigma_k = ||b_k||, sorted in decreasing order (stable), V's columns
 * permuted alike, and U[:, k] = b_k (the rotated column, i.e. U_k sigma_k);
 * callers divide by sigma_k themselves if they need unit vectors.
 *
 * Outputs: sigma (n values), V (n x n, column-major), US (rows x n,
 * column-major, may be NULL).  Returns the number of sweeps used, or -1 if
 * it did not converge within max_sweeps.
 */
int oracle_jacobi_svd(const double *A, int64_t rows, int64_t n, int64_t lda,
                      int max_sweeps, double *sigma, double *V, double *US)
{
    double *B = (double *)malloc((size_t)rows * (size_t)n * sizeof(double));
    double *Vw = (double *)malloc((size_t)n * (size_t)n * sizeof(double));
    double *nrm = (double *)malloc((size_t)n * sizeof(double));
    int64_t *order = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    for (int64_t k = 0; k < n; ++k)
        memcpy(B + k * rows, A + k * lda, (size_t)rows * sizeof(double));
    for (int64_t k = 0; k < n * n; ++k) Vw[k] = 0.0;
    for (int64_t k = 0; k < n; ++k) Vw[k + k * n] = 1.0;

    const double tol = sqrt((double)(rows > 0 ? rows : 1)) * ldexp(1.0, -52);
    int sweeps = 0, converged = 0;
    while (sweeps < max_sweeps) {
        int64_t rotated = 0;
        for (int64_t p = 0; p + 1 < n; ++p) {
            for (int64_t q = p + 1; q < n; ++q) {
                double *bp = B + p * rows, *bq = B + q * rows;
                double alpha = 0.0, beta = 0.0, gamma = 0.0;
                for (int64_t i = 0; i < rows; ++i) {
                    alpha += bp[i] * bp[i];
                    beta += bq[i] * bq[i];
                    gamma += bp[i] * bq[i];
                }
                if (alpha == 0.0 || beta == 0.0) continue;
                if (fabs(gamma) <= tol * sqrt(alpha) * sqrt(beta)) continue;
                ++rotated;
                /* Rotation that zeroes the (p, q) entry of B^T B. */
                double zeta = (beta - alpha) / (2.0 * gamma);
                double t;
                if (fabs(zeta) > 1e150)
                    t = 0.5 / zeta;
                else
                    t = (zeta >= 0.0 ? 1.0 : -1.0) /
                        (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                double c = 1.0 / sqrt(1.0 + t * t);
                double s = c * t;
                for (int64_t i = 0; i < rows; ++i) {
                    double a = bp[i], b = bq[i];
                    bp[i] = c * a - s * b;
                    bq[i] = s * a + c * b;
                }
                double *vp = Vw + p * n, *vq = Vw + q * n;
                for (int64_t i = 0; i < n; ++i) {
                    double a = vp[i], b = vq[i];
                    vp[i] = c * a - s * b;
                    vq[i] = s * a + c * b;
                }
            }
        }
        ++sweeps;
        if (rotated == 0) { converged = 1; break; }
    }

    for (int64_t k = 0; k < n; ++k) {
        double s2 = 0.0;
        for (int64_t i = 0; i < rows; ++i) s2 += B[i + k * rows] * B[i + k * rows];
        nrm[k] = sqrt(s2);
        order[k] = k;
    }
    /* Stable insertion sort by decreasing norm. */
    for (int64_t a = 1; a < n; ++a) {
        int64_t key = order[a];
        int64_t b = a - 1;
        while (b >= 0 && nrm[order[b]] < nrm[key]) {
            order[b + 1] = order[b];
            --b;
        }
        order[b + 1] = key;
    }
    for (int64_t k = 0; k < n; ++k) {
        int64_t src = order[k];
        sigma[k] = nrm[src];
        memcpy(V + k * n, Vw + src * n, (size_t)n * sizeof(double));
        if (US) memcpy(US + k * rows, B + src * rows, (size_t)rows * sizeof(double));
    }
    free(order);
    free(nrm);
    free(Vw);
    free(B);
    return converged ? sweeps : -1;
}
