"""GPU parity against the CPU FP64 oracle on the shapes where the kernels
loop: TSQR slices that span several row tiles (the triangular factor carried
from tile to tile), the grid-stride loop of the FP64 MFMA product, the
K = 512 block Jacobi SVD, and a padded last-mode stride.  Same tolerances as
test_gpu_parity.py (R to 1e-12 ||W||_F after row-sign normalisation, Gram
identity to 1e-12 ||W||_F^2, bit-exact products on small-integer data, TT
results to 1e-10 / 1e-12).
"""
import sys

import numpy as np
import pytest

import oracle
import ttcheck
from paper_2102_00104_amd import model, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU host
    pytest.skip("no GPU", allow_module_level=True)

import paper_2102_00104_amd as tt  # noqa: E402

DEV = torch.device("cuda:0")


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def sign_rows(R):
    K = min(R.shape)
    s = np.sign(np.diag(R[:K, :K]))
    s[s == 0] = 1
    out = R.copy()
    out[:K] *= s[:, None]
    return out


# Tall shapes whose first tree level has more row tiles per slice than one
# (the planner caps the slice count; each slice then reduces several tiles
# with its factor carried along): m = 2 and 8 (single-wave slices of
# 512-row tiles, 2 and 3 tiles), m = 16, 32, 64 and 100 (cooperative
# workgroups, 2 to 5 tiles); m = 144 takes the blocked kernel.
TSQR_TALL = [(1_200_000, 2), (3_000_000, 8), (600_000, 16), (1_000_000, 32),
             (700_000, 64), (300_000, 100),
             # blocked kernel: more 1024-row tiles than workgroups (each
             # workgroup reduces several tiles in turn), three tree levels
             (300_000, 144)]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("rows,cols", TSQR_TALL)
def test_tsqr_r_multi_tile_slices(rows, cols):
    log("tsqr tall %dx%d" % (rows, cols))
    W = np.random.default_rng(rows + 13 * cols).standard_normal((rows, cols))
    ld = rows + 5
    buf = np.zeros((ld, cols))
    buf[:rows] = W
    Wd = ttcheck.dev_from_fortran(buf, torch.float64, DEV)
    del buf
    R = torch.full((cols * cols,), np.nan, dtype=torch.float64, device=DEV)
    tt.ttsvd_tsqr_r(Wd, tt.TTSVD_F64, rows, cols, ld, R, cols)
    torch.cuda.synchronize()
    Rg = R.cpu().numpy().reshape(cols, cols, order="F")
    del Wd
    Ro = oracle.qr_r(W)
    nW = np.linalg.norm(W)
    assert np.all(np.isfinite(Rg))
    assert np.all(np.tril(Rg, -1) == 0.0)
    assert np.max(np.abs(sign_rows(Rg) - sign_rows(Ro))) <= 1e-12 * nW
    G = W.T @ W
    assert np.max(np.abs(Rg.T @ Rg - G)) <= 1e-12 * nW * nW


# FP64 products with m <= 64 and 16 < k <= 32 take the MFMA kernel, whose
# grid is capped: more than 524,288 rows make every workgroup loop.
GEMM_TALL = [(2_000_002, 64, 32, 2), (1_048_580, 48, 17, 4)]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("rows,cols,k,n_next", GEMM_TALL)
def test_gemm_reshape_grid_stride_bit_exact(rows, cols, k, n_next):
    log("gemm tall %s" % ((rows, cols, k, n_next),))
    rng = np.random.default_rng(rows + cols + k)
    W = rng.integers(-8, 9, size=(rows, cols)).astype(np.float64)
    V = rng.integers(-8, 9, size=(cols, k)).astype(np.float64)
    rn = rows // n_next
    Y = torch.full((rn * n_next * k,), np.nan, dtype=torch.float64, device=DEV)
    tt.ttsvd_gemm_reshape(ttcheck.dev_from_fortran(W, torch.float64, DEV), tt.TTSVD_F64, rows,
                          cols, rows, ttcheck.dev_from_fortran(V, torch.float64, DEV), cols, k,
                          n_next, Y, rn)
    torch.cuda.synchronize()
    Yh = Y.cpu().numpy().reshape(rn, n_next * k, order="F")
    P = W @ V  # exact: small integers
    # reshape(P, (rows/n_next, n_next k)) column-major: row i = i0 + rn b of P
    # lands in row i0, column b + n_next a
    expect = P.reshape(n_next, rn, k).transpose(1, 2, 0).reshape(rn, k * n_next)
    assert np.array_equal(Yh, expect)


@pytest.mark.timeout(900)
def test_block_svd_k512_matches_oracle():
    # d = 6, n = 16, r_max = 32: steps with m = 16, 256, 512 (4096 rows, so
    # K = 512: the 512 x 512 block Jacobi), 512 (K = 256) and 512 (K = 16)
    dims = [16] * 6
    log("uniform %s (K = 512 block SVD)" % (dims,))
    X = synth.uniform(dims, seed=71)
    g = tt.ttsvd_decompose(ttcheck.dev_from_fortran(X, torch.float64, DEV), dims, 32, 0.0)
    steps = model.steps(dims, g.ranks)
    assert any(m == 512 and min(rows, m) == 512 for _, rows, m, _ in steps)
    o = oracle.ttsvd(X, dims, 32, 0.0)
    ttcheck.compare_tt(g, o, X, tt.core_array)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("dims,r_max,tol,pad", [
    ([4, 4, 4, 4, 4, 6], 10, 0.0, 7),
    ([2] * 16 + [8], 32, 0.0, 129),
    ([3, 5, 7, 9], 8, 1e-3, 1),
])
def test_padded_last_mode_stride(dims, r_max, tol, pad):
    """X with ld_last > n_1...n_{d-1}: the padding (NaN here) is never read and
    the result equals the oracle's on the dense tensor."""
    log("ld_last %s pad %d" % (dims, pad))
    if tol > 0:
        X = synth.exact_tt(dims, 3, seed=81, noise=1e-6, noise_seed=82)
    else:
        X = synth.uniform(dims, seed=81)
    lead = synth.prod(dims[:-1])
    n_d = dims[-1]
    buf = np.full((lead + pad, n_d), np.nan)
    buf[:lead] = X.reshape(lead, n_d, order="F")
    Xd = ttcheck.dev_from_fortran(buf, torch.float64, DEV)
    g = tt.ttsvd_decompose(Xd, dims, r_max, tol, ld_last=lead + pad)
    o = oracle.ttsvd(X, dims, r_max, tol)
    if tol > 0:
        assert min(o.margins[1:]) > 1e-3
    ttcheck.compare_tt(g, o, X, tt.core_array)
    # the caller-workspace entry point on the same padded input: equal bits
    ws = torch.empty(tt.ttsvd_workspace_size(dims, r_max, tt.TTSVD_F64), dtype=torch.uint8,
                     device=DEV)
    cores = torch.empty(tt.ttsvd_cores_size(dims, r_max), dtype=torch.float64, device=DEV)
    h = tt.ttsvd_decompose_ws(Xd, dims, r_max, tol, ws, cores, ld_last=lead + pad)
    assert h.ranks == g.ranks
    for a, b in zip(h.cores, g.cores):
        assert torch.equal(a, b)
    for j in range(1, len(dims)):
        assert h.sigma[j] == g.sigma[j]
