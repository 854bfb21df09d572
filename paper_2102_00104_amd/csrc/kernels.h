// Internal launcher interface between the C ABI and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace ttsvd {

// ---------------------------------------------------------------- TSQR
// Q-less TSQR: R (m x m, FP64, column-major, ldr) of W (rows x m, dtype).
// ws must hold tsqr_workspace_bytes(dtype, rows, m) bytes.
size_t tsqr_workspace_bytes(int dtype, int64_t rows, int64_t m);
int tsqr_launch(const void *W, int dtype, int64_t rows, int64_t m, int64_t ld,
                double *R, int64_t ldr, void *ws, size_t ws_bytes,
                hipStream_t s);

// Levels 1.. of the TSQR of a rows x m unfolding whose level 0 was written by
// tsmm_qr_launch into the same workspace (nothing to do if it was the only
// level: R is then written already).
int tsqr_launch_after_first(int dtype, int64_t rows, int64_t m, double *R, int64_t ldr,
                            void *ws, size_t ws_bytes, hipStream_t s);

// ---------------------------------------------------------------- TSMM
// Y = reshape(W V, (rows/n_next, n_next k)), V(c, a) = V[c*svc + a*sva] (FP64).
// W has element type dtype; Y has element type ydtype (equal to dtype, or
// FP64 for the last TT core).
int tsmm_launch(const void *W, int dtype, int64_t rows, int64_t m, int64_t ld,
                const double *V, int64_t svc, int64_t sva, int64_t k,
                int64_t n_next, void *Y, int ydtype, int64_t ld_y,
                hipStream_t s);

// The product of tsmm_launch (ydtype = dtype, ld_y = rows / n_next) fused
// with level 0 of the TSQR of Y, for the shapes tsmm_qr_applies accepts
// (n_next in {2, 4}, Y taller than wide with n_next k <= 8 columns and W
// with m <= 8, or n_next k <= 32 and m <= 32): writes Y and level 0's factors (R itself, ldr, if that is the only
// level; else the stacked factors at the start of ws, which holds
// tsqr_workspace_bytes(dtype, rows / n_next, n_next k) bytes), and sets
// *levels_done = 1.  Y and the factors equal those of tsmm_launch followed
// by tsqr_launch.
bool tsmm_qr_applies(int dtype, int64_t rows, int64_t m, int64_t k, int64_t n_next);
int tsmm_qr_launch(const void *W, int dtype, int64_t rows, int64_t m, int64_t ld,
                   const double *V, int64_t svc, int64_t sva, int64_t k, int64_t n_next, void *Y,
                   double *R, int64_t ldr, void *ws, size_t ws_bytes, hipStream_t s,
                   int *levels_done);

// ---------------------------------------------------------------- SVD
// Device state shared by the steps of one decomposition.
struct StepState {
    double delta2;      // delta^2, set by the first step
    double norm2;       // ||Sigma||_F^2 of the first step
    int64_t rank;       // rank chosen by the last step
    double discarded2;  // sum of discarded sigma^2 of the last step
    int64_t sweeps;     // Jacobi sweeps of the last step
    int64_t nonfinite;  // set if the triangular factor was not finite
};

// Small SVD of the first K rows of R (m columns, column-major, ldr) by
// one-sided Jacobi on those rows, followed by the truncation rule and the
// core T = reshape(V_{:,1:r}^T, (r, m)).  scratch holds scratch_bytes >=
// svd_scratch_bytes(K, m) (checked).
//   sigma_out: K sorted singular values (device)
//   core_out : r x m FP64 (device), r = chosen rank, T[a + r*c] = V(c, a)
//   first    : this is the first step (sets delta from ||Sigma||_F)
//   state    : this step's rank / discarded energy; state0: the first step's
//              state, which holds delta^2 for every later step
//   tol, dm1 : tolerance and d - 1;  r_max: maximal rank
size_t svd_scratch_bytes(int64_t K, int64_t m);
int svd_launch(const double *R, int64_t ldr, int64_t K, int64_t m,
               double *sigma_out, double *core_out,
               int64_t r_max, double tol, int dm1, int first,
               StepState *state, StepState *state0, void *scratch, size_t scratch_bytes,
               hipStream_t s);

}  // namespace ttsvd
