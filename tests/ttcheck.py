"""Comparison helpers shared by the GPU parity tests (no GPU needed to import)."""
import numpy as np

import oracle


def dev_from_fortran(a, dtype, device):
    """Flat device copy of a Fortran-ordered array."""
    import torch
    flat = np.asfortranarray(a).reshape(-1, order="F")
    return torch.from_numpy(np.ascontiguousarray(flat)).to(device, dtype=dtype)


def host_cores(g, core_array):
    return [core_array(c, (g.ranks[j], g.dims[j], g.ranks[j + 1])) for j, c in enumerate(g.cores)]


def compare_tt(g, o, X, core_array, kept_rel=1e-10, err_abs=1e-12, recon=None, orth=1e-12):
    """A GPU TT result against the oracle's on the same input X:
    identical ranks; kept singular values to kept_rel relative and all of them
    to kept_rel sigma_1; relative reconstruction errors equal to err_abs;
    optionally reconstructions equal to recon ||X||_F; orthonormal cores."""
    assert g.ranks == o.ranks, (g.ranks, o.ranks)
    d = len(o.dims)
    for j in range(1, d):
        sg = np.asarray(g.sigma[j])
        so = o.sigma[j]
        assert len(sg) == len(so)
        r = o.ranks[j]
        assert np.all(np.abs(sg[:r] - so[:r]) <= kept_rel * so[:r]), j
        assert np.max(np.abs(sg - so)) <= kept_rel * max(so[0], 1e-300), j
    cores = host_cores(g, core_array)
    Xg = oracle.tt_full(cores)
    Xo = oracle.tt_full(o.cores)
    eg, eo = oracle.rel_error(X, Xg), oracle.rel_error(X, Xo)
    assert abs(eg - eo) <= err_abs, (eg, eo)
    if recon is not None:
        assert np.linalg.norm(Xg - Xo) <= recon * np.linalg.norm(X)
    for j in range(1, d):
        r, n, rn = cores[j].shape
        M = cores[j].reshape(r, n * rn, order="F")
        assert np.max(np.abs(M @ M.T - np.eye(r))) <= orth
    return cores, Xg
