"""The C ABI library loads and exports every entry point include/gsr.h
declares; host-only argument checks work without a GPU (no compute calls)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gsr.h")
LIB = os.path.join(ROOT, "paper_2607_14481_amd", "libgsr.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gsr_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("gsr_rasterize_forward", "gsr_rasterize_backward", "gsr_workspace_bytes",
                     "gsr_query_pairs", "gsr_version", "gsr_status_string", "gsr_last_error"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = C.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name
    from paper_2607_14481_amd import gsr
    assert sorted(gsr.EXPORTED) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_host_side_argument_checks():
    from paper_2607_14481_amd import gsr
    from paper_2607_14481_amd import scenes as S
    assert gsr.version() == 2
    assert gsr.status_string(gsr.GSR_ERR_CAPACITY) == "GSR_ERR_CAPACITY"
    cam = S.pinhole(128, 96, S.look_at([0, 0, -3]))
    nb1 = gsr.workspace_bytes(1000, [cam], 10_000)
    nb2 = gsr.workspace_bytes(1000, [cam], 20_000)
    assert nb2 > nb1 > 0 and nb1 % 256 == 0
    assert gsr.workspace_bytes(0, [cam], 1) > 0
    with pytest.raises(gsr.GsrError):
        gsr.workspace_bytes(1000, [cam], 0)
    with pytest.raises(gsr.GsrError):
        gsr.workspace_bytes(-1, [cam], 100)
    with pytest.raises(gsr.GsrError):
        gsr.workspace_bytes(10, [cam] * (gsr.GSR_MAX_VIEWS + 1), 100)
    bad = S.pinhole(0, 96, S.look_at([0, 0, -3]))
    with pytest.raises(gsr.GsrError):
        gsr.workspace_bytes(10, [bad], 100)
    # workspace sizing reports failure as 0 bytes plus a message
    with pytest.raises(gsr.GsrError):
        gsr.workspace_bytes(10, [cam], 100, gsr.launch_config(tile_h=12))
    assert "tile_h" in gsr.last_error()
