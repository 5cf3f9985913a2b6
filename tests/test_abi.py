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
    assert gsr.version() == 3
    assert C.sizeof(gsr.gsr_launch_config) == 32
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


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_bundle_adjustment_host_checks():
    """Sizing and the structure checks of the plan run on the host before any
    device call, so they work without a GPU."""
    import numpy as np
    from paper_2607_14481_amd import gsr
    n1 = gsr.ba_workspace_bytes(20, 16, 10_000, 8)
    n2 = gsr.ba_workspace_bytes(20, 16, 20_000, 8)
    assert n2 > n1 > 0 and n1 % 256 == 0
    for bad in ((20, 21, 100, 8), (20, 16, 0, 8), (20, 16, 100, 9), (20, 16, 100, 1), (0, 0, 100, 2)):
        with pytest.raises(gsr.GsrError):
            gsr.ba_workspace_bytes(*bad)
    L = gsr.lib()
    fake_ws = C.c_void_p(1 << 20)   # never dereferenced: every case fails its checks first

    def create(free_slot, obs_cam, ws_bytes=1 << 40):
        fs = np.ascontiguousarray(free_slot, np.int32)
        oc = np.ascontiguousarray(obs_cam, np.int32)
        h = C.c_void_p()
        rc = L.gsr_ba_plan_create(len(fs), fs.ctypes.data_as(C.c_void_p), oc.shape[0], oc.shape[1],
                                  oc.ctypes.data_as(C.c_void_p), fake_ws, ws_bytes, None, C.byref(h))
        return rc, gsr.last_error(), h.value

    ok_fs = [0, -1, 1, 2]
    cases = [
        (ok_fs, [[0, 0, -1], [1, 2, -1]], "twice"),            # a keyframe twice in one landmark
        (ok_fs, [[0, -1, -1], [1, 2, 3]], "observations"),     # one observation only
        (ok_fs, [[0, -1, 1], [1, 2, 3]], "come first"),        # a gap before a valid slot
        (ok_fs, [[0, 4, -1], [1, 2, 3]], "keyframe indices"),  # keyframe out of range
        ([0, 0, 1, 2], [[0, 1, -1], [1, 2, 3]], "one-to-one"),  # two keyframes in one slot
        ([0, 5, 1, 2], [[0, 1, -1], [1, 2, 3]], "one-to-one"),  # slot out of range
        (list(range(21)), [[0, 1, -1]], "free keyframes"),     # more free keyframes than supported
    ]
    for fs, oc, msg in cases:
        rc, err, h = create(fs, oc)
        assert rc != gsr.GSR_OK and h is None and msg in err, (fs, oc, err)
    rc, err, _ = create(ok_fs, [[0, 1, -1], [1, 2, 3]], ws_bytes=1024)
    assert rc == gsr.GSR_ERR_WORKSPACE_TOO_SMALL
    assert L.gsr_ba_plan_destroy(None) == gsr.GSR_OK


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_hierarchy_cut_host_checks():
    """The cut needs somewhere to put its size (host and/or device); checked
    before any device call."""
    from paper_2607_14481_amd import gsr
    from paper_2607_14481_amd import scenes as S
    L = gsr.lib()
    g = gsr.gsr_gaussians()
    g.n, g.sh_degree = 10, 0
    cams = gsr.cameras([S.pinhole(64, 48, S.look_at([0, 0, -3]))])
    rc = L.gsr_hierarchy_cut(C.byref(g), None, None, cams, None, 1.5, None, 0, None, None, None, None)
    assert rc == gsr.GSR_ERR_INVALID_ARGUMENT and "n_cut" in gsr.last_error()
    n_cut = C.c_int64(-1)
    g.n = 0  # an empty hierarchy has an empty cut
    assert L.gsr_hierarchy_cut(C.byref(g), None, None, cams, None, 1.5, None, 0, None, None, C.byref(n_cut),
                               None) == gsr.GSR_OK
    assert n_cut.value == 0


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_hierarchy_layout_host_only():
    """The node layout of a device-built hierarchy (host arithmetic only)
    matches the host builder's levels, including ragged last groups and the
    early stop at a single root."""
    import numpy as np
    from paper_2607_14481_amd import gsr
    from paper_2607_14481_amd import hierarchy as H
    from paper_2607_14481_amd import scenes as S
    rng = np.random.default_rng(0)
    for n, levels in ((1, 3), (8, 2), (9, 2), (1000, 7), (4097, 3)):
        leaves = S._gaussian_body(rng, rng.uniform(-1, 1, (n, 3)), 0)
        h = H.build(leaves, levels)
        np.testing.assert_array_equal(gsr.hierarchy_layout(n, levels, 8), h.level_start)
    assert list(gsr.hierarchy_layout(10, 0, 8)) == [0, 10]
    assert list(gsr.hierarchy_layout(19, 5, 4)) == [0, 19, 24, 26, 27]
    for bad in ((0, 3, 8), (10, -1, 8), (10, 3, 1), (10, 31, 8)):
        with pytest.raises(gsr.GsrError):
            gsr.hierarchy_layout(*bad)
