"""Seeded synthetic inputs for the TT-SVD (shared by the HIP path and the oracle).

This module only draws random numbers and assembles input tensors; it holds
none of the decomposition's arithmetic.  Every tensor is a flat float64 numpy
array in Fortran order (first mode fastest), the layout the decomposition
reads (Sec. 3.1.2 of arXiv 2102.00104, "Memory layout").

Workloads (sizes and distributions follow the paper's experiments, which use
uniformly random data with prescribed dimensions or TT ranks, Sec. 5):

* ``uniform``  -- i.i.d. U[0, 1) entries: a full-rank, worst-case tensor.
* ``exact_tt`` -- contraction of random Gaussian cores with prescribed ranks
  (an exact TT tensor), optionally plus i.i.d. Gaussian noise.
"""
from __future__ import annotations

from typing import List, Optional, Sequence

import numpy as np


def prod(xs: Sequence[int]) -> int:
    p = 1
    for x in xs:
        p *= int(x)
    return p


def capped_ranks(dims: Sequence[int], rank: int | Sequence[int]) -> List[int]:
    """Bond ranks r_0..r_d (r_0 = r_d = 1), each capped at
    min(prod(n_1..n_k), prod(n_{k+1}..n_d)) so the TT tensor can have them."""
    d = len(dims)
    if isinstance(rank, (int, np.integer)):
        inner = [int(rank)] * (d - 1)
    else:
        inner = [int(r) for r in rank]
        if len(inner) != d - 1:
            raise ValueError("need d-1 inner ranks")
    r = [1] + inner + [1]
    for k in range(1, d):
        left = prod(dims[:k])
        right = prod(dims[k:])
        r[k] = max(1, min(r[k], left, right))
    return r


def uniform(dims: Sequence[int], seed: int = 0) -> np.ndarray:
    """i.i.d. U[0, 1) entries, ``default_rng(seed).random``."""
    return np.random.default_rng(seed).random(prod(dims))


def gaussian_cores(dims: Sequence[int], ranks: Sequence[int], seed: int,
                   unit_variance: bool = False) -> List[np.ndarray]:
    """Cores G^(k) ~ N(0, 1) of shape (r_{k-1}, n_k, r_k), Fortran order.

    ``unit_variance`` scales core k >= 2 by 1/sqrt(r_{k-1}) so that the
    entries of the contracted tensor have unit variance.
    """
    rng = np.random.default_rng(seed)
    cores = []
    for k, n in enumerate(dims):
        shape = (int(ranks[k]), int(n), int(ranks[k + 1]))
        g = rng.standard_normal(prod(shape)).reshape(shape, order="F")
        if unit_variance and k >= 1:
            g = g / np.sqrt(ranks[k])
        cores.append(np.asfortranarray(g))
    return cores


def contract(cores: Sequence[np.ndarray]) -> np.ndarray:
    """Dense Fortran-ordered tensor of a TT given by its cores (einsum form)."""
    P = np.asarray(cores[0])[0]                      # (n_1, r_1)
    for G in cores[1:]:
        N = P.shape[0]
        Q = np.einsum("Ia,aib->Iib", P, G, optimize=True)   # (N, n, r')
        P = Q.reshape(N * G.shape[1], G.shape[2], order="F")
    return np.ascontiguousarray(P.reshape(-1, order="F"))


def exact_tt(dims: Sequence[int], rank: int | Sequence[int], seed: int,
             noise: float = 0.0, noise_seed: Optional[int] = None,
             unit_variance: bool = False, relative_noise: bool = False) -> np.ndarray:
    """Exact random TT tensor (Gaussian cores, ranks capped) plus noise.

    ``noise`` is the standard deviation of i.i.d. Gaussian noise drawn with
    ``default_rng(noise_seed)``; with ``relative_noise`` it is scaled by the
    RMS of the noise-free tensor.
    """
    ranks = capped_ranks(dims, rank)
    X = contract(gaussian_cores(dims, ranks, seed, unit_variance))
    if noise > 0:
        rng = np.random.default_rng(seed + 1 if noise_seed is None else noise_seed)
        scale = noise
        if relative_noise:
            scale *= float(np.sqrt(np.mean(X * X)))
        X = X + scale * rng.standard_normal(X.size)
    return X


def small_exact_tt_workload():
    """The small parity workload: d = 12, n_i = 2 (4096 elements), exact TT
    with all ranks 4 (Gaussian cores, seed 0) plus N(0, 1e-8^2) noise
    (seed 1); decomposed with r_max = 8, tol = 1e-10."""
    dims = [2] * 12
    X = exact_tt(dims, 4, seed=0, noise=1e-8, noise_seed=1)
    return dims, X, 8, 1e-10


def full_rank_workloads():
    """The two 2 GiB FP64 shapes of the full-rank workload: 2^28 i.i.d.
    U[0, 1) values (seed 0) viewed as d = 7, n_i = 16 and d = 28, n_i = 2,
    r_max = 32, no tolerance."""
    return [([16] * 7, 32, 0.0), ([2] * 28, 32, 0.0)]
