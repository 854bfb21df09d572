"""GPU parity of the two-sided TSQR TT-SVD (Algorithm 4,
``ttsvd_decompose_two_sided``) against the oracle's ``ttsvd_two_sided``.

FP64 tolerances as for Algorithm 2: identical ranks, kept singular values of
every step to 1e-10 relative and all of them to 1e-10 sigma_1, relative
reconstruction errors equal to 1e-12; cores left of the middle have
orthonormal columns, cores right of it orthonormal rows (1e-12); the norm
identity ||T_mid||^2 + sum of discarded sigma^2 = ||X||^2.  FP32 storage: the
bound c = (d - 1) 2^-24 + 1e-5 of the precision tests against the oracle on
the stored values.
"""
import sys

import numpy as np
import pytest

import oracle
import ttcheck
from paper_2102_00104_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU host
    pytest.skip("no GPU", allow_module_level=True)

import paper_2102_00104_amd as tt  # noqa: E402

DEV = torch.device("cuda:0")


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


CASES = [
    ([2] * 10, 5, 0.0, "uniform"),
    ([3, 4, 5, 6, 2], 4, 0.0, "uniform"),
    ([4] * 6, 16, 0.0, "uniform"),
    ([2, 3, 2, 3, 2, 3], 3, 0.0, "uniform"),
    ([6, 5, 4], 30, 0.0, "uniform"),          # no truncation
    ([2] * 13, 32, 0.0, "uniform"),           # odd d, steps of up to 64 columns
    ([2] * 12, 16, 1e-6, "exact4"),
    ([3, 4, 5, 2, 3], 50, 1e-12, "exact2"),
    ([16, 16, 16, 16], 32, 0.0, "uniform"),   # 256-column left and right steps
    ([40, 30], 6, 0.0, "uniform"),            # d = 2: Algorithm 2
]


def make(dims, kind, seed):
    if kind == "uniform":
        return synth.uniform(dims, seed=seed)
    if kind == "exact4":
        return synth.exact_tt(dims, 4, seed=seed, noise=1e-9, noise_seed=seed + 1)
    return synth.exact_tt(dims, 2, seed=seed)


def check_cores(g, dims):
    d = len(dims)
    mid = d // 2 - 1 if d % 2 == 0 else (d - 1) // 2
    cores = [tt.core_array(c, (g.ranks[j], dims[j], g.ranks[j + 1])) for j, c in enumerate(g.cores)]
    for j, c in enumerate(cores):
        r, n, rn = c.shape
        if j < mid:
            M = c.reshape(r * n, rn, order="F")
            assert np.max(np.abs(M.T @ M - np.eye(rn))) <= 1e-12, j
        elif j > mid:
            M = c.reshape(r, n * rn, order="F")
            assert np.max(np.abs(M @ M.T - np.eye(r))) <= 1e-12, j
    return cores, mid


@pytest.mark.parametrize("case", range(len(CASES)))
def test_two_sided_matches_oracle(case):
    dims, r_max, tol, kind = CASES[case]
    log("two-sided %s r_max=%d tol=%g" % (dims, r_max, tol))
    X = make(dims, kind, 500 + case)
    o = oracle.ttsvd_two_sided(X, dims, r_max, tol)
    if tol > 0:
        assert min(o.margins[1:]) > 1e-3
    g = tt.ttsvd_decompose_two_sided(ttcheck.dev_from_fortran(X, torch.float64, DEV), dims,
                                     r_max, tol)
    assert g.ranks == o.ranks
    d = len(dims)
    for j in range(1, d):
        sg, so = np.asarray(g.sigma[j]), o.sigma[j]
        assert len(sg) == len(so), j
        r = o.ranks[j]
        assert np.all(np.abs(sg[:r] - so[:r]) <= 1e-10 * so[:r]), j
        assert np.max(np.abs(sg - so)) <= 1e-10 * so[0], j
    cores, mid = check_cores(g, dims)
    eg = oracle.rel_error(X, oracle.tt_full(cores))
    eo = oracle.rel_error(X, oracle.tt_full(o.cores))
    assert abs(eg - eo) <= 1e-12, (eg, eo)
    nx2 = float(np.sum(X * X))
    assert abs(float(np.sum(cores[mid] ** 2)) + sum(g.discarded2[1:]) - nx2) <= 1e-10 * nx2


def test_two_sided_fp32_storage_within_bound():
    dims = [2] * 16
    X = synth.exact_tt(dims, 6, seed=71, noise=1e-6, noise_seed=72, unit_variance=True,
                       relative_noise=True)
    Xd = ttcheck.dev_from_fortran(X, torch.float32, DEV)
    Xs = Xd.to(torch.float64).cpu().numpy()
    o = oracle.ttsvd_two_sided(Xs, dims, 16, 1e-4)
    assert min(o.margins[1:]) > 1e-2
    g = tt.ttsvd_decompose_two_sided(Xd, dims, 16, 1e-4)
    assert g.ranks == o.ranks
    c = (len(dims) - 1) * 2.0 ** -24 + 1e-5
    for j in range(1, len(dims)):
        r = o.ranks[j]
        assert np.max(np.abs(np.asarray(g.sigma[j])[:r] - o.sigma[j][:r])) <= c * o.sigma[j][0]
    cores, _ = check_cores(g, dims)
    assert abs(oracle.rel_error(Xs, oracle.tt_full(cores)) -
               oracle.rel_error(Xs, oracle.tt_full(o.cores))) <= c


def test_two_sided_errors():
    X = torch.zeros(16 ** 3, dtype=torch.float64, device=DEV)
    with pytest.raises(tt.TTSVDError) as e:
        tt.ttsvd_decompose_two_sided(X, [16, 16, 16], 0, 0.0)
    assert e.value.code == -1
    g = tt.ttsvd_decompose_two_sided(X, [16, 16, 16], 4, 0.0)   # zero tensor: no NaN
    assert all(torch.isfinite(c).all() for c in g.cores)
