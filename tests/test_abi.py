"""CPU checks of the C ABI: the library loads and exports every declared symbol.

No compute call is made here (there is no GPU on this host).
"""
import ctypes
import os
import re

import pytest

import paper_2102_00104_amd as tt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ttsvd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ttsvd_[a-z0-9_]+)\s*\(", src)))


def test_header_matches_binding_list():
    assert _declared() == sorted(tt.EXPORTED)


@pytest.mark.skipif(not os.path.exists(tt.LIB_PATH), reason="libttsvd.so not built")
def test_library_exports_every_symbol():
    L = ctypes.CDLL(tt.LIB_PATH)
    for name in _declared():
        assert hasattr(L, name), name


@pytest.mark.skipif(not os.path.exists(tt.LIB_PATH), reason="libttsvd.so not built")
def test_host_only_entry_points():
    L = tt.lib()
    assert L.ttsvd_version().decode().startswith("libttsvd")
    assert L.ttsvd_strerror(-1).decode() == "invalid argument"
    assert L.ttsvd_strerror(0).decode() == "success"
    # workspace and footprint queries are pure host computations
    assert tt.ttsvd_tsqr_workspace_size(tt.TTSVD_F64, 1 << 20, 16) > 0
    assert tt.ttsvd_tsqr_workspace_size(tt.TTSVD_F64, 100, 2000) == 0
    fp = tt.ttsvd_footprint_bytes([2] * 28, 32, tt.TTSVD_F64)
    # two ping-pong work matrices of the size of X dominate (f = 1 steps)
    assert 2 * 8 * 2 ** 28 <= fp <= 3 * 8 * 2 ** 28
    assert tt.ttsvd_footprint_bytes([2] * 28, 0, tt.TTSVD_F64) == 0
    # caller-buffer sizes: cores at the no-tolerance ranks, and the footprint
    # is the workspace plus the (256-byte aligned) cores
    from paper_2102_00104_amd import model
    for dims, r_max in (([2] * 28, 32), ([16] * 7, 32), ([3, 5, 7, 9], 4), ([9], 3)):
        rk = model.no_tol_ranks(dims, r_max)
        nc = sum(rk[j] * dims[j] * rk[j + 1] for j in range(len(dims)))
        assert tt.ttsvd_cores_size(dims, r_max) == nc
        ws = tt.ttsvd_workspace_size(dims, r_max, tt.TTSVD_F64)
        assert ws > 0 and ws % 256 == 0
        assert tt.ttsvd_footprint_bytes(dims, r_max, tt.TTSVD_F64) == ws + (nc * 8 + 255) // 256 * 256
    assert tt.ttsvd_workspace_size([2] * 28, 32, 7) == 0
    assert tt.ttsvd_cores_size([2, 0, 2], 4) == 0


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(tt, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(tt, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        tt.lib()


def test_thick_bounds_k_host_logic():
    # host-only entry point (no GPU work): the Table 2 thick-bounds rows and
    # the oracle's choice on a few other shapes
    import oracle
    from paper_2102_00104_amd import thick_bounds_k
    for r_max, m in ((1, 16), (5, 16), (16, 32)):
        assert thick_bounds_k([2] * 11, 16, 0.5, r_max) == (m.bit_length() - 1, m)
    for dims, m_min, f1, r in (([2] * 28, 64, 0.5, 32), ([16] * 7, 64, 0.5, 32),
                               ([3, 100], 16, 0.5, 4), ([2, 2, 2], 64, 0.5, 4),
                               ([5, 3, 7, 2], 10, 1.0 / 3, 6)):
        assert thick_bounds_k(dims, m_min, f1, r) == oracle.thick_k(dims, m_min, f1, r)
    with pytest.raises(Exception):
        thick_bounds_k([2, 2], 0, 0.5, 4)
    with pytest.raises(Exception):
        thick_bounds_k([2, 2], 4, 0.0, 4)
