"""Pins of the oracle's two-sided TT-SVD (Algorithm 4, ``oracle.ttsvd_two_sided``)
against facts that do not depend on it:

* d = 2 is a single right step, i.e. Algorithm 2 itself;
* without truncation the TT reproduces X exactly, and exact TT tensors
  (TT ranks are unique) get their ranks back;
* every step truncates the remainder by an orthogonal projection on one
  side, so ||X - X~||^2 equals the sum of the discarded sigma^2, and with a
  tolerance the ENSURE bound ||X - X~|| <= eps ||X|| holds;
* cores left of the middle have orthonormal columns as (r n) x r', cores right
  of it orthonormal rows as r x (n r');
* brute force: the same left/right order with numpy's SVD of the unfoldings
  themselves (the left singular vectors of the short-wide left unfolding, no
  QR of a transpose) gives the same singular values and the same TT tensor.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2102_00104_amd import synth


def two_sided_by_svd(X, dims, r_max):
    """Algorithm 4's step order with full SVDs of the unfoldings (no tol)."""
    d = len(dims)
    ranks = [1] * (d + 1)
    cores = [None] * d
    sig = [None] * d
    Y = np.asarray(X, dtype=np.float64).reshape(-1, order="F")
    lo, hi, right = 0, d - 1, True
    while lo < hi:
        if right:
            m = dims[hi] * ranks[hi + 1]
            W = Y.reshape(-1, m, order="F")
            U, s, Vt = np.linalg.svd(W, full_matrices=False)
            r = min(r_max, len(s))
            ranks[hi], sig[hi] = r, s
            cores[hi] = Vt[:r].reshape(r, dims[hi], ranks[hi + 1], order="F")
            Y = (U[:, :r] * s[:r]).reshape(-1, order="F")
            hi -= 1
        else:
            P = ranks[lo] * dims[lo]
            L = Y.reshape(P, -1, order="F")
            U, s, Vt = np.linalg.svd(L, full_matrices=False)
            r = min(r_max, len(s))
            ranks[lo + 1], sig[lo + 1] = r, s
            cores[lo] = U[:, :r].reshape(ranks[lo], dims[lo], r, order="F")
            Y = (s[:r, None] * Vt[:r]).reshape(-1, order="F")
            lo += 1
        right = not right
    cores[lo] = Y.reshape(ranks[lo], dims[lo], ranks[lo + 1], order="F")
    return ranks, cores, sig


SHAPES = [[2] * 8, [3, 4, 5, 6, 2], [4] * 5, [2, 3, 2, 3, 2, 3], [6, 5, 4]]


def test_d2_is_algorithm_2():
    X = synth.uniform([40, 30], seed=3)
    a = oracle.ttsvd_two_sided(X, [40, 30], 7, 0.0)
    b = oracle.ttsvd(X, [40, 30], 7, 0.0)
    assert a.ranks == b.ranks
    assert np.array_equal(a.sigma[1], b.sigma[1])
    for ca, cb in zip(a.cores, b.cores):
        assert np.array_equal(ca, cb)


@pytest.mark.parametrize("dims", SHAPES)
def test_no_truncation_is_exact(dims):
    X = synth.uniform(dims, seed=11)
    o = oracle.ttsvd_two_sided(X, dims, 10 ** 6, 0.0)
    assert oracle.rel_error(X, oracle.tt_full(o.cores)) <= 1e-13


@pytest.mark.parametrize("dims,rank", [([2] * 10, 3), ([3, 4, 5, 3, 4], 2), ([4] * 6, 5)])
def test_exact_tt_ranks_recovered(dims, rank):
    X = synth.exact_tt(dims, rank, seed=21)
    o = oracle.ttsvd_two_sided(X, dims, 50, 1e-12)
    d = len(dims)
    expect = [1] + [min(rank, synth.prod(dims[:k]), synth.prod(dims[k:])) for k in range(1, d)] + [1]
    assert o.ranks == expect
    assert oracle.rel_error(X, oracle.tt_full(o.cores)) <= 1e-13


@pytest.mark.parametrize("dims", SHAPES)
@pytest.mark.parametrize("r_max", [1, 2, 3])
def test_error_equals_discarded_energy(dims, r_max):
    X = synth.uniform(dims, seed=31)
    o = oracle.ttsvd_two_sided(X, dims, r_max, 0.0)
    err2 = float(np.sum((X - oracle.tt_full(o.cores)) ** 2))
    assert abs(err2 - sum(o.discarded2[1:])) <= 1e-10 * float(np.sum(X * X))


@pytest.mark.parametrize("tol", [0.05, 0.2, 0.5])
def test_tolerance_bound(tol):
    dims = [3, 4, 5, 6, 2]
    X = synth.uniform(dims, seed=41)
    o = oracle.ttsvd_two_sided(X, dims, 10 ** 6, tol)
    assert oracle.rel_error(X, oracle.tt_full(o.cores)) <= tol * (1 + 1e-12)


@pytest.mark.parametrize("dims", SHAPES)
def test_core_orthonormality(dims):
    X = synth.uniform(dims, seed=51)
    o = oracle.ttsvd_two_sided(X, dims, 3, 0.0)
    d = len(dims)
    mid = d // 2 - 1 if d % 2 == 0 else (d - 1) // 2   # 0-based index of the middle core
    for j, c in enumerate(o.cores):
        r, n, rn = c.shape
        if j < mid:
            M = c.reshape(r * n, rn, order="F")
            assert np.max(np.abs(M.T @ M - np.eye(rn))) <= 1e-13
        elif j > mid:
            M = c.reshape(r, n * rn, order="F")
            assert np.max(np.abs(M @ M.T - np.eye(r))) <= 1e-13


@pytest.mark.parametrize("dims", SHAPES)
@pytest.mark.parametrize("r_max", [2, 4])
def test_brute_force_full_svd_of_unfoldings(dims, r_max):
    X = synth.uniform(dims, seed=61)
    o = oracle.ttsvd_two_sided(X, dims, r_max, 0.0)
    ranks, cores, sig = two_sided_by_svd(X, dims, r_max)
    assert o.ranks == ranks
    for j in range(1, len(dims)):
        K = len(o.sigma[j])
        assert np.max(np.abs(o.sigma[j] - sig[j][:K])) <= 1e-12 * sig[j][0]
    nx = math.sqrt(float(np.sum(X * X)))
    assert np.linalg.norm(oracle.tt_full(o.cores) - oracle.tt_full(cores)) <= 1e-12 * nx
