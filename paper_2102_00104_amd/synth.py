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
* ``batch_specs`` / ``exact_tt_device`` -- the many-tensor workloads (mixed
  shapes and ranks), assembled on the GPU because the batch is gigabytes.
* ``serving_trace`` -- a Poisson stream of requests of log-uniform sizes.
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


def batch_specs(count: int = 512, seed: int = 3, min_bytes: int = 4096,
                max_bytes: int = 64 << 20, elem_bytes: int = 4):
    """Shapes and bond ranks of the batched workload, ``default_rng(seed)``:
    per tensor d ~ U{6..20} and n_i ~ U{2, 4, 8}, rejected unless
    min_bytes <= elem_bytes * prod(n) <= max_bytes; then d - 1 bond ranks
    ~ U{2..16}, capped.  Returns [(dims, ranks r_0..r_d)]."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        d = int(rng.integers(6, 21))
        dims = [int(x) for x in rng.choice([2, 4, 8], size=d)]
        size = elem_bytes * prod(dims)
        if not (min_bytes <= size <= max_bytes):
            continue
        inner = [int(r) for r in rng.integers(2, 17, size=d - 1)]
        out.append((dims, capped_ranks(dims, inner)))
    return out


def exact_tt_device(dims: Sequence[int], ranks: Sequence[int], seed: int, noise: float,
                    noise_seed: int, device, dtype=None):
    """``exact_tt`` with unit-variance cores and relative noise, assembled on
    a torch device: the cores come from ``gaussian_cores(..., seed,
    unit_variance=True)``, the contraction runs in FP64 on the device and the
    noise is drawn by a device generator seeded with noise_seed.  Returns the
    flat Fortran-ordered tensor in dtype (default FP64)."""
    import torch
    cores = gaussian_cores(dims, ranks, seed, unit_variance=True)
    # A Fortran (N, r) matrix is held as the row-major (r, N) tensor T.
    T = torch.from_numpy(np.ascontiguousarray(cores[0][0].T)).to(device)
    for G in cores[1:]:
        r0, n, r1 = G.shape
        Gt = torch.from_numpy(np.ascontiguousarray(G.reshape(r0, n * r1, order="F").T)).to(device)
        T = (Gt @ T).reshape(r1, -1)
    X = T.reshape(-1)
    if noise > 0:
        g = torch.Generator(device=device)
        g.manual_seed(int(noise_seed))
        # the scale stays a device scalar: no host synchronisation, so a
        # producer can enqueue several tensors ahead of their use
        scale = noise * torch.sqrt(torch.mean(X * X))
        X = X + scale * torch.randn(X.numel(), generator=g, device=device, dtype=X.dtype)
    return X if dtype is None else X.to(dtype)


def serving_cores_device(dims: Sequence[int], ranks: Sequence[int], seed: int, device):
    """The cores of ``exact_tt_device`` (unit variance, ``default_rng(seed)``)
    as FP32 device matrices for ``serving_tensor``: the first as the row-major
    (r_1, n_1) tensor, core k as (row-major (n_k r_k, r_{k-1}) tensor, r_k).
    Building them ahead keeps host work and host-to-device copies out of a
    replay loop."""
    import torch
    cores = gaussian_cores(dims, ranks, seed, unit_variance=True)
    first = torch.from_numpy(np.ascontiguousarray(cores[0][0].T)).to(device, torch.float32)
    rest = []
    for G in cores[1:]:
        r0, n, r1 = G.shape
        Gt = torch.from_numpy(np.ascontiguousarray(G.reshape(r0, n * r1, order="F").T))
        rest.append((Gt.to(device, torch.float32), int(r1)))
    return first, rest


def serving_tensor(cores_dev, noise: float, noise_seed: int, device):
    """FP32 serving request tensor: the TT of ``cores_dev`` (from
    ``serving_cores_device``) contracted in FP32 on the device, plus i.i.d.
    Gaussian noise of `noise` times its RMS drawn by an FP32 device generator
    seeded with noise_seed.  Nothing synchronises with the host, so a
    producer can enqueue tensors ahead of their arrival.  Returns the flat
    Fortran-ordered tensor."""
    import torch
    first, rest = cores_dev
    T = first
    for Gt, r1 in rest:
        T = (Gt @ T).reshape(r1, -1)
    X = T.reshape(-1)
    if noise > 0:
        g = torch.Generator(device=device)
        g.manual_seed(int(noise_seed))
        scale = noise * torch.sqrt(torch.mean(X * X))
        X.addcmul_(torch.randn(X.numel(), generator=g, device=device, dtype=X.dtype), scale)
    return X


def serving_trace(duration_s: float = 10.0, rate: float = 200.0, seed: int = 4,
                  min_exp: int = 18, max_exp: int = 30):
    """Request trace of the serving workload, ``default_rng(seed)``: Poisson
    arrivals at `rate` per second over `duration_s`; per request 2^e elements
    with e ~ U{min_exp..max_exp}, split over modes with log2 n_i ~ U{1..4}
    (drawn until they sum to e, the last one cut to fit); r_max ~ U{4..64};
    tol log-uniform in [1e-5, 1e-2]; content bond ranks ~ U{2..16}, capped.
    Returns [{t, dims, ranks, r_max, tol}] in arrival order."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t > duration_s:
            break
        e = int(rng.integers(min_exp, max_exp + 1))
        logs = []
        while sum(logs) < e:
            logs.append(min(int(rng.integers(1, 5)), e - sum(logs)))
        dims = [2 ** l for l in logs]
        r_max = int(rng.integers(4, 65))
        tol = float(10.0 ** rng.uniform(-5.0, -2.0))
        inner = [int(x) for x in rng.integers(2, 17, size=len(dims) - 1)]
        out.append(dict(t=t, dims=dims, ranks=capped_ranks(dims, inner), r_max=r_max, tol=tol))
    return out
