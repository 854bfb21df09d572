"""The allocation-free TSQR entry point (ttsvd_tsqr_r_noalloc) against
ttsvd_tsqr_r on the same input: same kernels and reduction tree, so the
triangular factors must agree bit for bit.  Two calls in a row on one GPU
(the second with a smaller input, so stale tree factors of the first call sit
in the shared scratch), and a shape whose tree needs more than the fixed
scratch, which the host rejects before any launch.
"""
import sys

import numpy as np
import pytest

import ttcheck

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU host
    pytest.skip("no GPU", allow_module_level=True)

import paper_2102_00104_amd as tt  # noqa: E402

DEV = torch.device("cuda:0")


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def both(W, rows, cols, ld, dtype, tdt):
    Wd = ttcheck.dev_from_fortran(W, tdt, DEV)
    need = tt.ttsvd_tsqr_workspace_size(dtype, rows, cols)
    assert 0 < need <= tt.NOALLOC_SCRATCH_BYTES
    ws = torch.empty(need, dtype=torch.uint8, device=DEV)
    R_ws = torch.full((cols * cols,), 7.0, dtype=torch.float64, device=DEV)
    R_na = torch.full((cols * cols,), -7.0, dtype=torch.float64, device=DEV)
    tt.ttsvd_tsqr_r(Wd, dtype, rows, cols, ld, R_ws, cols, ws, need)
    tt.ttsvd_tsqr_r_noalloc(Wd, dtype, rows, cols, ld, R_na, cols)
    torch.cuda.synchronize()
    a = R_ws.cpu().numpy().reshape(cols, cols, order="F")
    b = R_na.cpu().numpy().reshape(cols, cols, order="F")
    return a, b


@pytest.mark.parametrize("dtype_name", ["f64", "f32"])
def test_noalloc_matches_workspace_form_two_calls(dtype_name):
    dtype, tdt = {"f64": (tt.TTSVD_F64, torch.float64),
                  "f32": (tt.TTSVD_F32, torch.float32)}[dtype_name]
    # first call: 700,000 x 64 (several row tiles per slice, two tree levels);
    # second call: a smaller, ragged 50,001 x 40 input on the same scratch
    for rows, cols, seed in ((700_000, 64, 1), (50_001, 40, 2)):
        log("noalloc %s %dx%d" % (dtype_name, rows, cols))
        ld = rows + 3
        W = np.zeros((ld, cols))
        W[:rows] = np.random.default_rng(seed).standard_normal((rows, cols))
        a, b = both(W, rows, cols, ld, dtype, tdt)
        assert np.array_equal(a, b), np.max(np.abs(a - b))
        # and the result is a triangular factor of W (Gram identity)
        Wt = W[:rows].astype(np.float32).astype(np.float64) if dtype_name == "f32" else W[:rows]
        G = Wt.T @ Wt
        tol = (1e-12 if dtype_name == "f64" else 1e-5) * np.linalg.norm(Wt) ** 2
        assert np.max(np.abs(b.T @ b - G)) <= tol
        assert np.all(np.tril(b, -1) == 0)


def test_noalloc_blocked_kernel_two_calls():
    # 128 < m <= 512 takes the blocked TSQR, whose tile regions (and the
    # flags of tiles shared by several workgroups) then live in the scratch:
    # 20,000 x 200 (20 tiles, three levels), then a smaller 3,000 x 144
    for rows, cols, seed in ((20_000, 200, 3), (3_000, 144, 4)):
        log("noalloc blocked %dx%d" % (rows, cols))
        ld = rows + 1
        W = np.zeros((ld, cols))
        W[:rows] = np.random.default_rng(seed).standard_normal((rows, cols))
        a, b = both(W, rows, cols, ld, tt.TTSVD_F64, torch.float64)
        assert np.array_equal(a, b), np.max(np.abs(a - b))
        G = W[:rows].T @ W[:rows]
        assert np.max(np.abs(b.T @ b - G)) <= 1e-12 * np.linalg.norm(W[:rows]) ** 2


def test_noalloc_rejects_shapes_beyond_the_scratch():
    rows, cols = 1 << 20, 256
    assert tt.ttsvd_tsqr_workspace_size(tt.TTSVD_F64, rows, cols) > tt.NOALLOC_SCRATCH_BYTES
    W = torch.empty(1, dtype=torch.float64, device=DEV)   # never read: rejected on the host
    R = torch.empty(1, dtype=torch.float64, device=DEV)
    with pytest.raises(tt.TTSVDError) as e:
        tt.ttsvd_tsqr_r_noalloc(W, tt.TTSVD_F64, rows, cols, rows, R, cols)
    assert e.value.code == -1 and "scratch" in str(e.value)
