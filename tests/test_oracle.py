"""Pins of the CPU FP64 oracle against what the paper and the mathematics fix.

None of these checks retypes the oracle's formulas: they test closed forms,
invariants, library special cases (numpy's LAPACK-backed QR and SVD), brute
force (Algorithm 1 against Algorithm 2) and the values printed in the paper's
Table 2.
"""
import math
import os

import numpy as np
import pytest

import oracle
from paper_2102_00104_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _sign_normalise_rows(R):
    s = np.sign(np.diag(R[:, :R.shape[0]]))
    s[s == 0] = 1.0
    return R * s[:, None]


# ---------------------------------------------------------------- QR ------

def test_qr_single_column_is_norm():
    w = np.random.default_rng(3).standard_normal((57, 1))
    R = oracle.qr_r(w)
    assert R.shape == (1, 1)
    assert abs(abs(R[0, 0]) - math.sqrt(math.fsum(w[:, 0] ** 2))) < 1e-13


def test_qr_gram_identity_and_triangular():
    W = np.random.default_rng(4).standard_normal((300, 9))
    R = oracle.qr_r(W)
    assert np.all(np.tril(R, -1) == 0.0)
    G = W.T @ W
    assert np.max(np.abs(R.T @ R - G)) <= 1e-12 * np.max(np.abs(G))


def test_qr_matches_lapack_up_to_row_signs():
    W = np.random.default_rng(5).random((200, 12))
    R = oracle.qr_r(W)
    Rl = np.linalg.qr(W, mode="r")
    assert np.allclose(_sign_normalise_rows(R), _sign_normalise_rows(Rl),
                       rtol=0, atol=1e-12 * np.abs(Rl).max())


def test_qr_wide_matrix():
    W = np.random.default_rng(6).standard_normal((4, 7))
    R = oracle.qr_r(W)
    assert R.shape == (4, 7)
    assert np.max(np.abs(R.T @ R - W.T @ W)) < 1e-12


def test_qr_rank_deficient_keeps_rank():
    rng = np.random.default_rng(7)
    W = rng.standard_normal((100, 2)) @ rng.standard_normal((2, 6))
    R = oracle.qr_r(W)
    s = np.linalg.svd(R, compute_uv=False)
    assert s[1] > 1e-3 * s[0]
    assert s[2] < 1e-13 * s[0]


def test_qr_zero_matrix_no_nan():
    R = oracle.qr_r(np.zeros((10, 3)))
    assert np.all(R == 0.0)


# ---------------------------------------------------------------- SVD -----

@pytest.mark.parametrize("shape", [(40, 8), (8, 8), (5, 9), (1, 4), (30, 1)])
def test_jacobi_svd_matches_lapack(shape):
    A = np.random.default_rng(8).standard_normal(shape)
    sigma, V = oracle.jacobi_svd(A)
    s_ref = np.linalg.svd(A, compute_uv=False)
    k = len(s_ref)
    assert np.allclose(sigma[:k], s_ref, rtol=0, atol=1e-13 * s_ref[0])
    assert np.all(sigma[k:] <= 1e-13 * s_ref[0])
    assert np.max(np.abs(V.T @ V - np.eye(shape[1]))) < 1e-13


def test_jacobi_svd_decomposition_identity():
    A = np.random.default_rng(9).standard_normal((25, 6))
    sigma, V, US = oracle.jacobi_svd(A, want_u=True)
    assert np.max(np.abs(A @ V - US)) < 1e-13
    U = US / sigma
    assert np.max(np.abs(U.T @ U - np.eye(6))) < 1e-13
    assert np.all(np.diff(sigma) <= 0)


def test_jacobi_svd_diagonal_closed_form():
    d = np.array([0.5, -3.0, 2.0, 0.0, 1.0])
    sigma, V = oracle.jacobi_svd(np.diag(d))
    assert np.array_equal(sigma, np.array([3.0, 2.0, 1.0, 0.5, 0.0]))


def test_jacobi_svd_2x2_closed_form():
    a, b, c = 3.0, 4.0, 2.0
    sigma, _ = oracle.jacobi_svd(np.array([[a, b], [0.0, c]]))
    # sigma1 sigma2 = |det|, sigma1^2 + sigma2^2 = ||A||_F^2
    assert abs(sigma[0] * sigma[1] - abs(a * c)) < 1e-13
    assert abs(sigma[0] ** 2 + sigma[1] ** 2 - (a * a + b * b + c * c)) < 1e-12


# ---------------------------------------------------------- rank rule -----

def test_rank_rule_hand_built_sigma():
    s = np.array([3.0, 2.0, 1.0, 0.5])
    # tails: 14.25, 5.25, 1.25, 0.25, 0 ; '<=' is inclusive
    assert oracle.rank_rule(s, math.sqrt(1.25), 10, 1.0) == 2
    assert oracle.rank_rule(s, math.sqrt(1.2), 10, 1.0) == 3
    assert oracle.rank_rule(s, math.sqrt(1.25), 1, 1.0) == 1
    # delta >= ||Sigma||_F: r_delta = 0, clamped to 1
    assert oracle.rank_rule(s, 10.0, 10, 1.0) == 1
    # no tolerance: min(r_max, K)
    assert oracle.rank_rule(s, 0.0, 3, 0.0) == 3
    assert oracle.rank_rule(s, 0.0, 9, 0.0) == 4


# ------------------------------------------------------------- TT-SVD -----

def _orthonormal_rows(core):
    r, n, rn = core.shape
    M = core.reshape(r, n * rn, order="F")
    return np.max(np.abs(M @ M.T - np.eye(r)))


@pytest.mark.parametrize("dims,rank", [([3, 4, 5, 2, 3], 2), ([2] * 9, 3),
                                       ([4, 3, 4, 3], 5)])
def test_exact_tt_ranks_recovered(dims, rank):
    X = synth.exact_tt(dims, rank, seed=11)
    tt = oracle.ttsvd(X, dims, r_max=50, tol=1e-12)
    assert tt.ranks == synth.capped_ranks(dims, rank)
    assert oracle.rel_error(X, oracle.tt_full(tt.cores)) <= 1e-13
    for j in range(1, len(dims)):
        assert _orthonormal_rows(tt.cores[j]) <= 1e-13


@pytest.mark.parametrize("dims,r_max", [([2] * 10, 5), ([3, 4, 5, 6], 4),
                                        ([16, 16, 16], 7)])
def test_oseledets_error_identity(dims, r_max):
    # right-to-left sequential truncation: the per-step errors are mutually
    # orthogonal, so ||X - X~||^2 equals the sum of discarded sigma^2
    X = synth.uniform(dims, seed=12)
    tt = oracle.ttsvd(X, dims, r_max=r_max, tol=0.0)
    err2 = float(np.sum((X - oracle.tt_full(tt.cores)) ** 2))
    bound2 = math.fsum(tt.discarded2)
    assert abs(err2 - bound2) <= 1e-10 * float(np.sum(X * X))
    assert err2 > 0


@pytest.mark.parametrize("eps", [1e-1, 1e-2, 3e-3])
def test_tolerance_guarantee(eps):
    # ENSURE clause: ||X - X~||_F <= eps ||X||_F when r_max >= r_delta
    dims = [4, 4, 4, 4, 4]
    X = synth.exact_tt(dims, 3, seed=13, noise=0.02, noise_seed=14)
    tt = oracle.ttsvd(X, dims, r_max=1000, tol=eps)
    assert oracle.rel_error(X, oracle.tt_full(tt.cores)) <= eps * (1 + 1e-12)


@pytest.mark.parametrize("dims", [[2] * 8, [3] * 5, [4] * 4, [2, 3, 4, 5]])
def test_algorithm2_equals_algorithm1_brute_force(dims):
    X = synth.uniform(dims, seed=15)
    for r_max, tol in [(3, 0.0), (100, 0.05)]:
        a2 = oracle.ttsvd(X, dims, r_max, tol, variant="alg2")
        a1 = oracle.ttsvd(X, dims, r_max, tol, variant="alg1")
        assert a1.ranks == a2.ranks
        for j in range(1, len(dims)):
            s1, s2 = a1.sigma[j], a2.sigma[j]
            assert np.allclose(s1, s2, rtol=0, atol=1e-12 * s1[0])
        x1 = oracle.tt_full(a1.cores)
        x2 = oracle.tt_full(a2.cores)
        assert np.max(np.abs(x1 - x2)) <= 1e-12 * np.max(np.abs(X))


def test_two_dims_is_truncated_svd():
    dims = [30, 20]
    X = synth.uniform(dims, seed=16)
    tt = oracle.ttsvd(X, dims, r_max=6, tol=0.0)
    M = X.reshape(30, 20, order="F")
    s = np.linalg.svd(M, compute_uv=False)
    err = np.linalg.norm(M - oracle.tt_full(tt.cores).reshape(30, 20, order="F"))
    assert abs(err - math.sqrt(np.sum(s[6:] ** 2))) < 1e-12 * s[0]
    assert np.allclose(tt.sigma[1], s, rtol=0, atol=1e-13 * s[0])


def test_rank_one_outer_product():
    rng = np.random.default_rng(17)
    vs = [rng.standard_normal(n) for n in (3, 4, 2, 5)]
    X = vs[0]
    for v in vs[1:]:
        X = np.multiply.outer(X, v)
    X = np.asfortranarray(X).reshape(-1, order="F")
    tt = oracle.ttsvd(X, [3, 4, 2, 5], r_max=10, tol=1e-10)
    assert tt.ranks == [1, 1, 1, 1, 1]
    assert oracle.rel_error(X, oracle.tt_full(tt.cores)) < 1e-14


def test_zero_tensor():
    dims = [2, 3, 4]
    tt = oracle.ttsvd(np.zeros(24), dims, r_max=5, tol=1e-8)
    assert tt.ranks == [1, 1, 1, 1]
    assert all(np.all(np.isfinite(c)) for c in tt.cores)
    assert np.all(oracle.tt_full(tt.cores) == 0.0)


def test_single_mode_is_identity():
    X = synth.uniform([7], seed=18)
    tt = oracle.ttsvd(X, [7], r_max=3, tol=0.1)
    assert tt.ranks == [1, 1]
    assert np.array_equal(tt.cores[0].reshape(-1), X)


def _read_table2():
    rows = []
    with open(os.path.join(GOLDEN, "table2_plain_ranks.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            r_max, ranks, fs = [p.strip() for p in line.split("|")]
            fr = []
            for t in fs.split():
                num, _, den = t.partition("/")
                fr.append(float(num) / float(den or 1))
            rows.append((int(r_max), [int(x) for x in ranks.split()], fr))
    return rows


@pytest.mark.parametrize("r_max,ranks,fs", _read_table2())
def test_table2_rank_sequences(r_max, ranks, fs):
    d = 11
    dims = [2] * d
    X = synth.uniform(dims, seed=19)
    tt = oracle.ttsvd(X, dims, r_max=r_max, tol=0.0)
    # right-most inner ranks r_{d-len}..r_{d-1}
    assert tt.ranks[d - len(ranks):d] == ranks
    # reduction factors f_j = r_{i-1} / (n_i r_i), i = d, d-1, ...
    got = [tt.ranks[i - 1] / (dims[i - 1] * tt.ranks[i]) for i in range(d, d - len(fs), -1)]
    assert np.allclose(got, fs)


def test_small_workload_ranks_and_margin():
    dims, X, r_max, tol = synth.small_exact_tt_workload()
    tt = oracle.ttsvd(X, dims, r_max, tol)
    assert tt.ranks == synth.capped_ranks(dims, 4)
    assert min(tt.margins[1:]) > 1e-3          # well-posed rank decisions
    assert oracle.rel_error(X, oracle.tt_full(tt.cores)) < 1e-10


# ------------------------------------------------------ Table 3 (model) ---

def test_table3_byte_and_flop_model():
    from paper_2102_00104_amd import model
    with open(os.path.join(GOLDEN, "table3_model.txt")) as f:
        rows = [l.split("|") for l in f if l.strip() and not l.startswith("#")]
    for case, d, n, r_max, gflop, gbyte in rows:
        dims = [int(n)] * int(d)
        ranks = model.no_tol_ranks(dims, int(r_max))
        assert round(model.flops(dims, ranks) / 1e9) == int(gflop)
        assert round(model.algorithmic_bytes(dims, ranks, 8) / 1e9) == int(gbyte)


def test_model_matches_oracle_shapes():
    from paper_2102_00104_amd import model
    dims = [2] * 11
    X = synth.uniform(dims, seed=20)
    tt = oracle.ttsvd(X, dims, r_max=5, tol=0.0)
    assert model.no_tol_ranks(dims, 5) == tt.ranks


# --------------------------------------------------------------- Algorithm 3

def _read_table2_thick():
    rows = []
    with open(os.path.join(GOLDEN, "table2_thick_bounds.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            r_max, m, ranks, fs = [p.strip() for p in line.split("|")]
            fr = []
            for t in fs.split():
                num, _, den = t.partition("/")
                fr.append(float(num) / float(den or 1))
            rows.append((int(r_max), int(m), [int(x) for x in ranks.split()], fr))
    return rows


@pytest.mark.parametrize("r_max,m,ranks,fs", _read_table2_thick())
def test_table2_thick_bounds(r_max, m, ranks, fs):
    # Table 2, thick-bounds rows: m_min = 16, f_1^min = 1/2 on a 2^d tensor
    d = 11
    dims = [2] * d
    X = synth.uniform(dims, seed=19)
    th = oracle.ttsvd_thick(X, dims, r_max=r_max, tol=0.0, m_min=16, f1_min=0.5)
    assert th.m == m and 2 ** th.k == m
    dw = [2] * (d - th.k) + [m]
    dd = len(dw)
    assert th.main.ranks[dd - len(ranks):dd] == ranks
    got = [th.main.ranks[i - 1] / (dw[i - 1] * th.main.ranks[i]) for i in range(dd, dd - len(fs), -1)]
    assert np.allclose(got, fs)


def test_thick_k_extremes():
    # one mode already wide enough: nothing is combined
    assert oracle.thick_k([3, 100], 16, 0.5, 4) == (1, 100)
    # no k qualifies: every mode is combined
    assert oracle.thick_k([2, 2, 2], 64, 0.5, 4) == (3, 8)
    for dims in ([3, 100], [2, 2, 2]):
        X = synth.uniform(dims, seed=23)
        th = oracle.ttsvd_thick(X, dims, r_max=4, tol=0.0, m_min=64 if dims == [2, 2, 2] else 16,
                                f1_min=0.5)
        tt = oracle.ttsvd(X, dims, r_max=4, tol=0.0)
        assert th.rec is None and th.tt.ranks == tt.ranks
        for a, b in zip(th.tt.cores, tt.cores):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("dims,r_max", [([2] * 12, 16), ([2] * 10, 8), ([3, 4, 2, 2, 2, 2], 8)])
def test_thick_equals_plain_without_inner_truncation(dims, r_max):
    # When r_max does not cut any rank inside the combined block, Algorithm 3
    # truncates the same unfolding as Algorithm 2 at the block boundary and
    # splits the combined core exactly: same ranks, same singular values at
    # and left of the boundary, same approximation.
    X = synth.uniform(dims, seed=29)
    th = oracle.ttsvd_thick(X, dims, r_max=r_max, tol=0.0, m_min=16, f1_min=0.5)
    tt = oracle.ttsvd(X, dims, r_max=r_max, tol=0.0)
    d = len(dims)
    k = th.k
    assert 1 < k < d
    # no rank inside the block is cut: the exact ranks fit under r_max
    assert all(oracle._prod(dims[j:]) <= min(r_max, oracle._prod(dims[:j]))
               for j in range(d - k + 1, d))
    assert th.tt.ranks == tt.ranks
    for j in range(1, d - k + 1):
        assert np.allclose(th.tt.sigma[j], tt.sigma[j], rtol=1e-12, atol=1e-12 * tt.sigma[j][0])
    Xa, Xb = oracle.tt_full(th.tt.cores), oracle.tt_full(tt.cores)
    assert np.linalg.norm(Xa - Xb) <= 1e-12 * np.linalg.norm(X)


@pytest.mark.parametrize("dims,r_max,tol", [([3, 4, 5, 6, 2], 2, 0.0), ([2] * 10, 3, 0.0),
                                            ([4, 4, 4, 4, 4], 50, 0.3)])
def test_thick_error_bound_with_inner_truncation(dims, r_max, tol):
    # ranks cut inside the combined block: the result differs from
    # Algorithm 2, but ||X - X~|| stays below e_main + sigma_1 e_rec and the
    # cores right of the block boundary keep orthonormal rows
    X = synth.uniform(dims, seed=31)
    th = oracle.ttsvd_thick(X, dims, r_max=r_max, tol=tol, m_min=16, f1_min=0.5)
    d = len(dims)
    assert 1 < th.k < d
    assert sum(th.rec.discarded2[1:]) > 0                # something was cut inside
    err = np.linalg.norm(X - oracle.tt_full(th.tt.cores))
    assert err <= th.err_bound * (1 + 1e-12) + 1e-12
    for j in list(range(1, d - th.k)) + list(range(d - th.k + 1, d)):
        r, n, rn = th.tt.cores[j].shape
        M = th.tt.cores[j].reshape(r, n * rn, order="F")
        assert np.max(np.abs(M @ M.T - np.eye(r))) <= 1e-12
