"""GPU tests of the thick-bounds TT-SVD (``ttsvd_decompose_thick``,
Algorithm 3) through the C ABI, against the FP64 oracle's Algorithm 3 and
against the plain path."""
import numpy as np
import pytest

import oracle
from paper_2102_00104_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU host
    pytest.skip("no GPU", allow_module_level=True)

import paper_2102_00104_amd as tt  # noqa: E402
import ttcheck  # noqa: E402

DEV = torch.device("cuda:0")


def log(msg):
    print("[thick] %s" % msg, flush=True)


def _dev(X):
    return ttcheck.dev_from_fortran(X, torch.float64, DEV)


def _check(g, th, X, kept_rel=1e-10, err_abs=1e-12):
    o = th.tt
    d = len(o.dims)
    assert g.ranks == o.ranks, (g.ranks, o.ranks)
    for j in range(1, d):
        sg, so = np.asarray(g.sigma[j]), o.sigma[j]
        assert len(sg) == len(so)
        r = o.ranks[j]
        assert np.all(np.abs(sg[:r] - so[:r]) <= kept_rel * so[:r]), j
        assert np.max(np.abs(sg - so)) <= kept_rel * max(so[0], 1e-300), j
    cores = ttcheck.host_cores(g, tt.core_array)
    Xg = oracle.tt_full(cores)
    eg, eo = oracle.rel_error(X, Xg), oracle.rel_error(X, oracle.tt_full(o.cores))
    assert abs(eg - eo) <= err_abs, (eg, eo)
    # ||X - X~|| within the stated bound, which matches the oracle's
    assert np.linalg.norm(X - Xg) <= g.err_bound * (1 + 1e-10) + 1e-12
    # (the bound is a sum of discarded sigma^2: the kept_rel sigma_1 accuracy
    # of small discarded values leaves it about 1e-7 relative)
    assert abs(g.err_bound - th.err_bound) <= 1e-6 * max(th.err_bound, 1e-300) + 1e-12
    # cores right of the first one keep orthonormal rows, except the first
    # core of the split block (a product with the block's left factor)
    for j in range(1, d):
        if j == d - th.k and th.rec is not None:
            continue
        r, n, rn = cores[j].shape
        M = cores[j].reshape(r, n * rn, order="F")
        assert np.max(np.abs(M @ M.T - np.eye(r))) <= 1e-12
    return Xg


@pytest.mark.parametrize("dims,r_max,tol,m_min", [
    ([2] * 12, 16, 0.0, 16),          # k = 5: no rank cut inside the block
    ([2] * 16, 32, 0.0, 64),          # k = 6: the d = 28 workload's split at 2^16
    ([3, 4, 5, 6, 2], 2, 0.0, 16),    # ranks cut inside the block
    ([4] * 5, 50, 0.3, 16),           # tolerance decides the ranks
    ([16] * 4, 32, 0.0, 64),          # k = 2, m = 256: column-group TSQR
])
def test_thick_matches_oracle(dims, r_max, tol, m_min):
    log("thick %s r=%d tol=%g m_min=%d" % (dims, r_max, tol, m_min))
    X = synth.uniform(dims, seed=37)
    th = oracle.ttsvd_thick(X, dims, r_max, tol, m_min, 0.5)
    assert 1 < th.k < len(dims)
    if tol > 0:
        assert min(th.main.margins[1:] + th.rec.margins[1:]) > 1e-3
    g = tt.ttsvd_decompose_thick(_dev(X), dims, r_max, tol, m_min=m_min, f1_min=0.5)
    _check(g, th, X)


def test_thick_equals_plain_without_inner_truncation():
    dims, r_max = [2] * 14, 32
    X = synth.uniform(dims, seed=41)
    Xd = _dev(X)
    g = tt.ttsvd_decompose_thick(Xd, dims, r_max, 0.0, m_min=64, f1_min=0.5)
    p = tt.ttsvd_decompose(Xd, dims, r_max, 0.0)
    assert g.ranks == p.ranks
    k, _ = tt.thick_bounds_k(dims, 64, 0.5, r_max)
    d = len(dims)
    for j in range(1, d - k + 1):
        assert np.allclose(g.sigma[j], p.sigma[j], rtol=1e-11, atol=1e-11 * p.sigma[j][0])
    Xg = oracle.tt_full(ttcheck.host_cores(g, tt.core_array))
    Xp = oracle.tt_full(ttcheck.host_cores(p, tt.core_array))
    assert np.linalg.norm(Xg - Xp) <= 1e-12 * np.linalg.norm(X)


@pytest.mark.parametrize("dims,m_min", [([3, 100], 16), ([2, 2, 2], 64)])
def test_thick_without_split_is_plain(dims, m_min):
    # k = 1 or k = d: ttsvd_decompose itself, bit for bit
    X = synth.uniform(dims, seed=43)
    Xd = _dev(X)
    g = tt.ttsvd_decompose_thick(Xd, dims, 4, 0.0, m_min=m_min, f1_min=0.5)
    p = tt.ttsvd_decompose(Xd, dims, 4, 0.0)
    assert g.ranks == p.ranks
    for a, b in zip(g.cores, p.cores):
        assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())


def test_thick_rejects_padded_last_mode():
    # [2]*8 with m_min 16 combines 4 modes; a padded last-mode stride is not
    # a reinterpretation of the combined modes
    import ctypes
    dims = [2] * 8
    X = torch.zeros(2 * 160, dtype=torch.float64, device=DEV)
    xs = tt.TensorStruct(X.data_ptr(), tt.TTSVD_F64, 160, 0)
    arr = (ctypes.c_int64 * 8)(*dims)
    out = tt.TTStruct()
    rc = tt.lib().ttsvd_decompose_thick(ctypes.byref(xs), arr, 8, 4, 0.0, 16, 0.5, ctypes.byref(out))
    assert rc == -5  # TTSVD_EUNSUPPORTED
    assert out.priv is None


def test_thick_errors():
    X = torch.zeros(16, dtype=torch.float64, device=DEV)
    with pytest.raises(tt.TTSVDError) as e:
        tt.ttsvd_decompose_thick(X, [4, 4], 2, 0.0, m_min=0, f1_min=0.5)
    assert e.value.code == -1
    with pytest.raises(tt.TTSVDError) as e:
        tt.ttsvd_decompose_thick(X, [4, 4], 2, 0.0, m_min=4, f1_min=1.5)
    assert e.value.code == -1
