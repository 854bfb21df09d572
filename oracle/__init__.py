"""CPU FP64 oracle for the TT-SVD of arXiv 2102.00104.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference that the HIP path is checked against.  Only ``tests/``, the smoke
check in ``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  It shares no code with the product library and never imports it.

Contents and the passages they follow (section / algorithm / equation numbers
of the paper):

* ``qr_r``        -- triangular factor R of W = QR (Sec. 2.1.1), textbook
                     Householder, in C (``oracle_la.c``).
* ``jacobi_svd``  -- SVD by one-sided Jacobi (Sec. 2.1.1), in C.
* ``rank_rule``   -- the truncation rank  r = min(r_max, r_delta)  with
                     r_delta = min{j : sigma_{j+1}^2 + sigma_{j+2}^2 + ... <= delta^2}
                     (Algorithm 1 and Algorithm 2, "choose rank").
* ``ttsvd``       -- Algorithm 2 (optimized TSQR TT-SVD): R from a QR of each
                     unfolding, SVD of R, delta from the first step's Sigma,
                     W <- reshape(W V_r).  ``variant="alg1"`` runs Algorithm 1
                     instead: full SVD of each unfolding, delta from ||X||_F,
                     W <- U_r Sigma_r.
* ``thick_k``     -- the number k of right-most modes Algorithm 3 combines:
                     the smallest k with m = n_{d-k+1} ... n_d >=
                     max(m_min, r_est / f_1^min) (k = d if none).
* ``ttsvd_thick`` -- Algorithm 3 (thick-bounds TT-SVD): Algorithm 2 on the
                     tensor with its k right-most modes combined, then the
                     combined core split by a TT-SVD of its own.
* ``ttsvd_two_sided`` -- Algorithm 4 (two-sided TSQR TT-SVD): steps on the
                     right-most and the left-most remaining mode in turn; a
                     left step takes the QR of the transposed left unfolding.
* ``tt_full``     -- contraction of the TT cores back to a dense tensor
                     (the TT format, Sec. 2.1.2).

Conventions (the paper leaves them open; the same readings are listed with the
design notes): tensors are flat float64 arrays in Fortran order (i_1 fastest,
Sec. 3.1.2 "Memory layout"); core T^(j) has shape (r_{j-1}, n_j, r_j) in
Fortran order; tol = 0 means "no tolerance", i.e. r = min(r_max, K); the rank
is clamped to 1 <= r <= K, K = min(rows, cols) of the unfolding.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle_la.c")
_LIB = os.path.join(_HERE, "liboracle_la.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``oracle_la.c`` into ``liboracle_la.so`` with gcc."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
             "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        lib.oracle_qr_r.argtypes = [dp, i64, i64, i64, dp]
        lib.oracle_qr_r.restype = None
        lib.oracle_jacobi_svd.argtypes = [dp, i64, i64, i64, ctypes.c_int,
                                          dp, dp, dp]
        lib.oracle_jacobi_svd.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def qr_r(W: np.ndarray) -> np.ndarray:
    """R (K x cols, upper trapezoidal, K = min(rows, cols)) of W = QR.

    Textbook Householder (Sec. 2.1.1, QR decomposition); W is not modified.
    Row signs follow LAPACK's dlarfg convention (R_jj = -sign(x_0)||x||).
    """
    W = np.asfortranarray(W, dtype=np.float64)
    rows, cols = W.shape
    K = min(rows, cols)
    R = np.zeros((K, cols), dtype=np.float64, order="F")
    if K == 0:
        return R
    _load().oracle_qr_r(_dp(W), rows, cols, max(rows, 1), _dp(R))
    return R


def jacobi_svd(A: np.ndarray, max_sweeps: int = 60, want_u: bool = False):
    """One-sided Jacobi SVD of A (rows x n): returns (sigma, V[, U*sigma]).

    sigma has n entries in decreasing order; V is n x n orthogonal with
    A V = U diag(sigma) (Sec. 2.1.1).  With ``want_u`` the rotated columns
    U diag(sigma) are returned too.
    """
    A = np.asfortranarray(A, dtype=np.float64)
    rows, n = A.shape
    sigma = np.zeros(n, dtype=np.float64)
    V = np.zeros((n, n), dtype=np.float64, order="F")
    US = np.zeros((rows, n), dtype=np.float64, order="F") if want_u else None
    if n == 0:
        return (sigma, V, US) if want_u else (sigma, V)
    sweeps = _load().oracle_jacobi_svd(
        _dp(A), rows, n, max(rows, 1), max_sweeps, _dp(sigma), _dp(V),
        _dp(US) if want_u else ctypes.POINTER(ctypes.c_double)())
    if sweeps < 0:
        raise RuntimeError("oracle Jacobi SVD did not converge")
    return (sigma, V, US) if want_u else (sigma, V)


def tails(sigma: np.ndarray) -> np.ndarray:
    """tails[i] = sigma_i^2 + sigma_{i+1}^2 + ... (0-based), tails[K] = 0.

    Summed from the smallest value upward in FP64.
    """
    K = len(sigma)
    t = np.zeros(K + 1, dtype=np.float64)
    acc = 0.0
    for i in range(K - 1, -1, -1):
        acc += float(sigma[i]) * float(sigma[i])
        t[i] = acc
    return t


def rank_rule(sigma: np.ndarray, delta: float, r_max: int, tol: float) -> int:
    """r = min(r_max, r_delta), clamped to [1, K] (Algorithms 1 and 2).

    r_delta is the smallest j with sigma_{j+1}^2 + sigma_{j+2}^2 + ... <= delta^2
    (1-based sigma), i.e. the smallest 0-based count i with tails[i] <= delta^2.
    tol == 0 means no tolerance: r = min(r_max, K).
    """
    K = len(sigma)
    if tol == 0.0:
        return max(1, min(r_max, K))
    t = tails(sigma)
    d2 = delta * delta
    r_delta = K
    for i in range(K + 1):
        if t[i] <= d2:
            r_delta = i
            break
    return max(1, min(r_max, r_delta, K))


@dataclass
class OracleTT:
    """Result of the oracle TT-SVD.

    ranks[0..d] with ranks[0] = ranks[d] = 1; cores[j] has shape
    (ranks[j], dims[j], ranks[j+1]) (0-based j); sigma[j] holds all K singular
    values of the step that produced core j (j = 1..d-1, None for j = 0);
    discarded2[j] the sum of the discarded sigma^2 of that step; margins[j]
    the relative distance of the two tail sums around the chosen rank from
    delta^2 (inf where no tolerance decided the rank).
    """
    dims: List[int]
    ranks: List[int]
    cores: List[np.ndarray]
    sigma: List[Optional[np.ndarray]]
    discarded2: List[float]
    delta: float
    norm_sigma: float
    margins: List[float] = field(default_factory=list)


def _prod(xs: Sequence[int]) -> int:
    p = 1
    for x in xs:
        p *= int(x)
    return p


def ttsvd(X: np.ndarray, dims: Sequence[int], r_max: int, tol: float,
          variant: str = "alg2") -> OracleTT:
    """TT-SVD of the Fortran-ordered tensor X (Algorithm 2, or Algorithm 1).

    ``variant="alg2"``: optimized TSQR TT-SVD (Algorithm 2):
      for i = d..2: R <- QR(W^(i)); (Sigma, V) <- SVD(R); in the first
      iteration delta <- eps / sqrt(d-1) * ||Sigma||_F; r_{i-1} <- rank rule;
      T^(i) <- reshape(V_{:,1:r}^T, (r_{i-1}, n_i, r_i));
      W^(i-1) <- reshape(W^(i) V_{:,1:r}, ...); finally T^(1) <- W^(1).
    ``variant="alg1"``: original TT-SVD (Algorithm 1): delta from ||X||_F, the
      SVD of the whole unfolding, W <- U_r Sigma_r.
    """
    dims = [int(n) for n in dims]
    d = len(dims)
    if d < 1 or any(n < 1 for n in dims) or r_max < 1 or tol < 0:
        raise ValueError("invalid TT-SVD arguments")
    nbar = _prod(dims)
    X = np.asarray(X, dtype=np.float64).reshape(-1, order="F")
    if X.size != nbar:
        raise ValueError("X has %d elements, dims need %d" % (X.size, nbar))
    if d == 1:
        core = X.reshape(1, dims[0], 1, order="F").copy(order="F")
        return OracleTT(dims, [1, 1], [core], [None], [0.0], 0.0,
                        float(np.sqrt(np.sum(X * X))), [math.inf])
    ranks = [1] * (d + 1)
    cores: List[Optional[np.ndarray]] = [None] * d
    sigmas: List[Optional[np.ndarray]] = [None] * d
    disc = [0.0] * d
    margins = [math.inf] * d
    delta = 0.0
    norm_sigma = 0.0
    if variant == "alg1":
        delta = tol / math.sqrt(d - 1) * float(np.sqrt(np.sum(X * X)))
    W = X.copy()
    for i in range(d - 1, 0, -1):          # 0-based core index (paper's i+1)
        m = dims[i] * ranks[i + 1]
        rows = nbar // m
        K = min(rows, m)
        Wm = W.reshape(rows, m, order="F")
        if variant == "alg2":
            R = qr_r(Wm)                                   # QR, keep R only
            sigma, V = jacobi_svd(R)                       # SVD of R
            sigma = sigma[:K].copy()
            US = None
        elif variant == "alg1":
            sigma, V, US = jacobi_svd(Wm, want_u=True)     # SVD of W itself
            sigma = sigma[:K].copy()
        else:
            raise ValueError("variant must be 'alg1' or 'alg2'")
        if i == d - 1:
            norm_sigma = float(np.sqrt(np.sum(sigma * sigma)))
            if variant == "alg2":
                delta = tol / math.sqrt(d - 1) * norm_sigma
        r = rank_rule(sigma, delta, r_max, tol)
        t = tails(sigma)
        disc[i] = float(t[r])
        if tol > 0:
            d2 = delta * delta
            cand = [abs(t[r] - d2) / d2 if d2 > 0 else math.inf]
            if r >= 1:
                cand.append(abs(t[r - 1] - d2) / d2 if d2 > 0 else math.inf)
            margins[i] = min(cand)
        sigmas[i] = sigma
        cores[i] = V[:, :r].T.reshape(r, dims[i], ranks[i + 1], order="F").copy(order="F")
        if variant == "alg2":
            Wn = Wm @ V[:, :r]                              # W^(i) V_{:,1:r}
        else:
            Wn = US[:, :r]                                  # U_r Sigma_r
        nbar = rows * r
        ranks[i] = r
        W = np.asfortranarray(Wn).reshape(-1, order="F")
    cores[0] = W.reshape(1, dims[0], ranks[1], order="F").copy(order="F")
    return OracleTT(dims, ranks, cores, sigmas, disc, delta, norm_sigma, margins)


def ttsvd_two_sided(X: np.ndarray, dims: Sequence[int], r_max: int, tol: float) -> OracleTT:
    """Two-sided TSQR TT-SVD (Algorithm 4).

    The remaining tensor Y has modes lo..hi (0-based) with bond ranks
    r_lo on its left and r_{hi+1} on its right, Fortran-ordered.  Steps
    alternate, starting on the right (the paper's i = d, 1, d-1, 2, ...):

    * right step on mode hi: W = reshape(Y, (rest, n_hi r_{hi+1})); R from the
      QR of W; SVD of R; r_hi by the rank rule; T^(hi) = reshape(V_r^T);
      Y <- W V_r;
    * left step on mode lo: L = reshape(Y, (r_lo n_lo, rest)) is short and
      wide, so the QR is taken of its transpose L^T (the reordering of
      Algorithm 4); SVD of R = U S V^T gives L = V S (Q U)^T, so
      T^(lo) = reshape(V_r, (r_lo, n_lo, r_{lo+1})) and the remainder is
      (L^T V_r)^T.

    delta comes from the first step's ||Sigma||_F as in Algorithm 2.  The last
    remaining mode is the middle core.  sigma[j] and discarded2[j] belong to
    the step that chose ranks[j] (j = 1..d-1), as for ``ttsvd``.
    """
    dims = [int(n) for n in dims]
    d = len(dims)
    if d < 1 or any(n < 1 for n in dims) or r_max < 1 or tol < 0:
        raise ValueError("invalid TT-SVD arguments")
    X = np.asarray(X, dtype=np.float64).reshape(-1, order="F")
    if X.size != _prod(dims):
        raise ValueError("X has %d elements, dims need %d" % (X.size, _prod(dims)))
    if d == 1:
        return ttsvd(X, dims, r_max, tol)
    ranks = [1] * (d + 1)
    cores: List[Optional[np.ndarray]] = [None] * d
    sigmas: List[Optional[np.ndarray]] = [None] * d
    disc = [0.0] * d
    margins = [math.inf] * d
    delta = 0.0
    norm_sigma = 0.0
    first = True
    Y = X.copy()
    lo, hi = 0, d - 1
    right = True
    while lo < hi:
        if right:
            m = dims[hi] * ranks[hi + 1]
            rows = Y.size // m
            W = Y.reshape(rows, m, order="F")
            bond = hi
        else:
            P = ranks[lo] * dims[lo]
            Q = Y.size // P
            W = np.asfortranarray(Y.reshape(P, Q, order="F").T)      # L^T, Q x P
            rows, m = Q, P
            bond = lo + 1
        K = min(rows, m)
        R = qr_r(W)
        sigma, V = jacobi_svd(R)
        sigma = sigma[:K].copy()
        if first:
            norm_sigma = float(np.sqrt(np.sum(sigma * sigma)))
            delta = tol / math.sqrt(d - 1) * norm_sigma
            first = False
        r = rank_rule(sigma, delta, r_max, tol)
        t = tails(sigma)
        disc[bond] = float(t[r])
        if tol > 0:
            d2 = delta * delta
            cand = [abs(t[r] - d2) / d2 if d2 > 0 else math.inf]
            if r >= 1:
                cand.append(abs(t[r - 1] - d2) / d2 if d2 > 0 else math.inf)
            margins[bond] = min(cand)
        sigmas[bond] = sigma
        ranks[bond] = r
        Wbar = W @ V[:, :r]                                          # rows x r
        if right:
            cores[hi] = V[:, :r].T.reshape(r, dims[hi], ranks[hi + 1], order="F").copy(order="F")
            Y = np.asfortranarray(Wbar).reshape(-1, order="F")
            hi -= 1
        else:
            cores[lo] = V[:, :r].reshape(ranks[lo], dims[lo], r, order="F").copy(order="F")
            Y = np.asfortranarray(Wbar.T).reshape(-1, order="F")
            lo += 1
        right = not right
    cores[lo] = Y.reshape(ranks[lo], dims[lo], ranks[lo + 1], order="F").copy(order="F")
    return OracleTT(dims, ranks, cores, sigmas, disc, delta, norm_sigma, margins)


def tt_full(cores: Sequence[np.ndarray]) -> np.ndarray:
    """Dense Fortran-ordered tensor (flat) from TT cores (Sec. 2.1.2).

    P_1 = T^(1) as n_1 x r_1; P_{k+1} = reshape(P_k T^(k+1)_{(r_k, n r)}),
    which in Fortran order is a reinterpretation of the same memory.
    """
    P = np.asarray(cores[0], dtype=np.float64)
    r0, n0, r1 = P.shape
    P = P.reshape(n0, r1, order="F")
    for T in cores[1:]:
        r, n, rn = T.shape
        Q = P @ np.asarray(T, dtype=np.float64).reshape(r, n * rn, order="F")
        P = Q.reshape(Q.shape[0] * n, rn, order="F")
    return P.reshape(-1, order="F")


def rel_error(X: np.ndarray, Xt: np.ndarray) -> float:
    """||X - X~||_F / ||X||_F (0 for X = 0 and X~ = 0)."""
    X = np.asarray(X, dtype=np.float64).reshape(-1)
    Xt = np.asarray(Xt, dtype=np.float64).reshape(-1)
    nx = math.sqrt(math.fsum(float(v) * float(v) for v in X)) if X.size < 1 << 16 \
        else float(np.sqrt(np.sum(X * X)))
    diff = X - Xt
    nd = float(np.sqrt(np.sum(diff * diff)))
    return nd / nx if nx > 0 else nd


def thick_k(dims: Sequence[int], m_min: int, f1_min: float, r_est: int):
    """Number k of right-most modes that Algorithm 3 combines, and their
    product m: the smallest k in 1..d with m >= max(m_min, r_est / f1_min).

    The first step of Algorithm 2 on the combined tensor shrinks the work
    array by f_1 = r / m; asking for f_1 <= f1_min with r ~ r_est gives
    m >= r_est / f1_min (the reading that reproduces Table 2).  Where no k
    qualifies, all d modes are combined (k = d).
    """
    dims = [int(n) for n in dims]
    if not dims or m_min < 1 or not (0.0 < f1_min <= 1.0) or r_est < 1:
        raise ValueError("invalid thick-bounds arguments")
    need = max(float(m_min), float(r_est) / float(f1_min))
    m = 1
    for k in range(1, len(dims) + 1):
        m *= dims[len(dims) - k]
        if m >= need:
            return k, m
    return len(dims), m


@dataclass
class OracleThick:
    """Result of Algorithm 3: ``tt`` the d-mode TT decomposition, ``k`` and
    ``m`` the combined modes and their product, ``main`` Algorithm 2 on the
    combined tensor, ``rec`` the TT-SVD of its combined core (None if k <= 1
    or k >= d), and ``err_bound`` an upper bound of ||X - X~||_F."""
    tt: OracleTT
    k: int
    m: int
    main: OracleTT
    rec: Optional[OracleTT]
    err_bound: float


def ttsvd_thick(X: np.ndarray, dims: Sequence[int], r_max: int, tol: float,
                m_min: int, f1_min: float, r_est: Optional[int] = None) -> OracleThick:
    """Thick-bounds TT-SVD (Algorithm 3).

    1. k, m <- thick_k(dims, m_min, f1_min, r_est or r_max);
    2. W <- reshape(X, (n_1, ..., n_{d-k}, m)) (a reinterpretation in
       Fortran order);
    3. T^(1), ..., T^(d-k), Tbar <- TT-SVD(W) (Algorithm 2, r_max, tol);
    4. the k cores of the combined modes from the TT-SVD of Tbar, read as the
       tensor (r_{d-k} n_{d-k+1}, n_{d-k+2}, ..., n_d) with the same r_max
       and tol; its first core (1, r n, r') is the core (r, n, r').
    k <= 1 or k >= d is Algorithm 2 on X itself.  Since X = L Tbar with
    ||L||_2 = sigma_1 of the combined step, ||X - X~|| <= e_main + sigma_1 e_rec,
    e = sqrt(sum of discarded sigma^2) of each TT-SVD.
    """
    dims = [int(n) for n in dims]
    d = len(dims)
    k, m = thick_k(dims, m_min, f1_min, r_est if r_est is not None else r_max)
    if k <= 1 or k >= d:
        tt = ttsvd(X, dims, r_max, tol)
        e = math.sqrt(sum(tt.discarded2[1:]))
        return OracleThick(tt, k, m, tt, None, e)
    dims_w = dims[:d - k] + [m]
    main = ttsvd(X, dims_w, r_max, tol)
    r = main.ranks[d - k]
    Tbar = main.cores[d - k].reshape(-1, order="F")             # (r, m, 1)
    dims_b = [r * dims[d - k]] + dims[d - k + 1:]
    rec = ttsvd(Tbar, dims_b, r_max, tol)
    ranks = main.ranks[:d - k + 1] + rec.ranks[1:]
    cores = main.cores[:d - k] + \
        [rec.cores[0].reshape(r, dims[d - k], rec.ranks[1], order="F").copy(order="F")] + \
        rec.cores[1:]
    sigma = main.sigma[:d - k + 1] + rec.sigma[1:]
    disc = main.discarded2[:d - k + 1] + rec.discarded2[1:]
    margins = main.margins[:d - k + 1] + rec.margins[1:]
    tt = OracleTT(dims, ranks, cores, sigma, disc, main.delta, main.norm_sigma, margins)
    s1 = float(main.sigma[d - k][0]) if main.sigma[d - k] is not None and len(main.sigma[d - k]) else 0.0
    e = math.sqrt(sum(main.discarded2[1:])) + s1 * math.sqrt(sum(rec.discarded2[1:]))
    return OracleThick(tt, k, m, main, rec, e)
