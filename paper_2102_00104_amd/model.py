"""Data-volume and operation model of the TSQR TT-SVD (Sec. 4 of arXiv 2102.00104).

Per step (unfolding W of rows x m, next rank k):
  * TSQR reads W once:                     e * rows * m bytes,  2 rows m^2 flops
  * TSMM reads W again and writes W V:     e * rows * (m + k),  2 rows m k flops
so a step moves 2 e n + e f n bytes with n = rows m elements and f = k / m
(the eq. "TT-SVD data volume" of Sec. 4.2: read twice, write the reduced
matrix once).  These are the method's algorithmic bytes: what the paper's
roofline counts, independent of how an implementation moves them.
"""
from __future__ import annotations

from typing import List, Sequence


def no_tol_ranks(dims: Sequence[int], r_max: int) -> List[int]:
    """Ranks r_0..r_d of the plain algorithm without tolerance:
    r_{i-1} = min(r_max, rows_i, m_i) (the shapes of Table 2)."""
    d = len(dims)
    r = [1] * (d + 1)
    nbar = 1
    for n in dims:
        nbar *= int(n)
    for i in range(d - 1, 0, -1):
        m = dims[i] * r[i + 1]
        rows = nbar // m
        r[i] = min(r_max, rows, m)
        nbar = rows * r[i]
    return r


def steps(dims: Sequence[int], ranks: Sequence[int]):
    """[(i, rows, m, k)] for i = d-1 .. 1 (0-based core index i)."""
    d = len(dims)
    nbar = 1
    for n in dims:
        nbar *= int(n)
    out = []
    for i in range(d - 1, 0, -1):
        m = dims[i] * ranks[i + 1]
        rows = nbar // m
        k = ranks[i]
        out.append((i, rows, m, k))
        nbar = rows * k
    return out


def algorithmic_bytes(dims, ranks, elem_bytes: int = 8) -> float:
    return float(sum(elem_bytes * (2 * rows * m + rows * k) for _, rows, m, k in steps(dims, ranks)))


def flops(dims, ranks) -> float:
    return float(sum(2 * rows * m * m + 2 * rows * m * k for _, rows, m, k in steps(dims, ranks)))


def per_step(dims, ranks, elem_bytes: int = 8):
    return [dict(core=i, rows=rows, m=m, k=k,
                 tsqr_bytes=elem_bytes * rows * m, tsqr_flops=2 * rows * m * m,
                 tsmm_bytes=elem_bytes * rows * (m + k), tsmm_flops=2 * rows * m * k)
            for i, rows, m, k in steps(dims, ranks)]
