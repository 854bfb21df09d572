"""GPU tests of the precision forms: FP32 / BF16 storage, FP32 block-local
accumulation, FP64 reduction tree and SVD of R.

Bounds (u = 2^-24, FP32 unit roundoff; the stored values themselves are exact
inputs, so the algorithmic error is that of FP32 accumulation):
  * TSQR: ||R^T R - W^T W|| <= 1e-5 ||W||_F^2 for W as stored;
  * gemm_reshape: bit-exact on small integers (exact in FP32); BF16 output is
    the round-to-nearest-even of the exact value;
  * TT-SVD: the work matrices W^(i) are stored in the input type, so every
    step adds a storage rounding of at most u_s ||W^(i)||_F (u_s = 2^-24 for
    FP32, 2^-8 for BF16) on top of FP32 accumulation.  With c = (d - 1) u_s +
    1e-5: kept singular values within c sigma_1 of the FP64 oracle on the
    upcast stored tensor (Weyl), relative reconstruction error within c of the
    oracle's; against the original FP64 tensor one more u_s (input rounding).
"""
import numpy as np
import pytest

import oracle
from paper_2102_00104_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU host
    pytest.skip("no GPU", allow_module_level=True)

import paper_2102_00104_amd as tt  # noqa: E402

DEV = torch.device("cuda:0")
DTYPES = {"f32": torch.float32, "bf16": torch.bfloat16}


def to_dev(flat_f64, dtype):
    return torch.from_numpy(np.ascontiguousarray(flat_f64)).to(DEV).to(dtype)


def stored_f64(t):
    return t.to(torch.float64).cpu().numpy()


def bf16_rne(x):
    """Round float64 values (exact in FP32) to bfloat16, nearest-even."""
    f = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((f >> 16) & 1) + 0x7FFF
    out = ((f + r) >> 16).astype(np.uint32) << 16
    return out.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("name", ["f32", "bf16"])
@pytest.mark.parametrize("rows,cols", [(100000, 2), (50000, 8), (40000, 16), (30000, 32),
                                       (20000, 64), (5000, 100)])
def test_tsqr_low_precision(name, rows, cols):
    W = np.random.default_rng(rows + cols).random((rows, cols))
    Wd = to_dev(W.reshape(-1, order="F"), DTYPES[name])
    Ws = stored_f64(Wd).reshape(rows, cols, order="F")
    R = torch.zeros(cols * cols, dtype=torch.float64, device=DEV)
    tt.ttsvd_tsqr_r(Wd, tt.dtype_code(Wd), rows, cols, rows, R, cols)
    torch.cuda.synchronize()
    Rg = R.cpu().numpy().reshape(cols, cols, order="F")
    G = Ws.T @ Ws
    assert np.all(np.isfinite(Rg))
    assert np.max(np.abs(Rg.T @ Rg - G)) <= 1e-5 * np.linalg.norm(Ws) ** 2


@pytest.mark.parametrize("name", ["f32", "bf16"])
@pytest.mark.parametrize("rows,cols,k,n_next", [
    (8192, 16, 16, 4),      # two rows per lane (even rows, ld, rows/n_next, ld_y)
    (65536, 64, 32, 2),     # the d = 28 shape, k bucket 32
    (1000, 7, 5, 5),        # k bucket 8, several chunks of rows per block
    (8190, 16, 16, 2),      # rows/n_next odd: one row per lane
    (999, 3, 2, 3),         # odd rows
])
def test_gemm_reshape_low_precision_exact(name, rows, cols, k, n_next):
    rng = np.random.default_rng(7)
    W = rng.integers(-4, 5, size=(rows, cols)).astype(np.float64)
    V = rng.integers(-4, 5, size=(cols, k)).astype(np.float64)
    Wd = to_dev(W.reshape(-1, order="F"), DTYPES[name])
    Vd = torch.from_numpy(V.reshape(-1, order="F").copy()).to(DEV)
    rn = rows // n_next
    Y = torch.zeros(rn * n_next * k, dtype=DTYPES[name], device=DEV)
    tt.ttsvd_gemm_reshape(Wd, tt.dtype_code(Wd), rows, cols, rows, Vd, cols, k, n_next, Y, rn)
    torch.cuda.synchronize()
    Yh = stored_f64(Y).reshape(rn, n_next * k, order="F")
    P = W @ V
    if name == "bf16":
        P = bf16_rne(P)
    expect = np.empty((rn, n_next * k))
    for a in range(k):
        expect[:, n_next * a:n_next * (a + 1)] = P[:, a].reshape(rn, n_next, order="F")
    assert np.array_equal(Yh, expect)


@pytest.mark.parametrize("name", ["f32", "bf16"])
def test_exact_tt_with_noise_low_precision(name):
    # the precision workload at small scale: exact TT, ranks 16, unit-variance
    # cores, relative noise 1e-4; r_max = 32, no tolerance
    dims = [2] * 18
    X = synth.exact_tt(dims, 16, seed=61, noise=1e-4, noise_seed=62, unit_variance=True,
                       relative_noise=True)
    Xd = to_dev(X, DTYPES[name])
    Xs = stored_f64(Xd)
    g = tt.ttsvd_decompose(Xd, dims, 32, 0.0)
    o_s = oracle.ttsvd(Xs, dims, 32, 0.0)          # oracle on the stored values
    assert g.ranks == o_s.ranks
    u_s = 2.0 ** -24 if name == "f32" else 2.0 ** -8
    c = (len(dims) - 1) * u_s + 1e-5
    worst = 0.0
    for j in range(1, len(dims)):
        sg, so = np.asarray(g.sigma[j]), o_s.sigma[j]
        r = o_s.ranks[j]
        dev = np.max(np.abs(sg[:r] - so[:r])) / so[0]
        worst = max(worst, dev)
        assert dev <= c, (j, dev)
    cores = [tt.core_array(c_, (g.ranks[j], dims[j], g.ranks[j + 1])) for j, c_ in enumerate(g.cores)]
    Xg = oracle.tt_full(cores)
    e_s = oracle.rel_error(Xs, Xg)
    e_os = oracle.rel_error(Xs, oracle.tt_full(o_s.cores))
    assert abs(e_s - e_os) <= c
    # against the original FP64 tensor: the input rounding adds <= u_s ||X||
    e_x = oracle.rel_error(X, Xg)
    o_x = oracle.ttsvd(X, dims, 32, 0.0)
    e_ox = oracle.rel_error(X, oracle.tt_full(o_x.cores))
    assert e_x <= e_ox + u_s + c
    print("%s: max sigma deviation %.2e sigma_1, rel. error %.3e (FP64 oracle %.3e)"
          % (name, worst, e_x, e_ox))
