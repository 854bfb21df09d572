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
    return sorted(set(re.findall(r"\b(ttsvd_[a-z_]+)\s*\(", src)))


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


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(tt, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(tt, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        tt.lib()
