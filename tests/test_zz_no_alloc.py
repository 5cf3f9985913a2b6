"""The scratch-free level-of-detail cut (gsr_hierarchy_cut_static), called
through the C ABI, against the cut with caller-provided scratch
(gsr_hierarchy_cut): identical node lists and counts (index work: bit-exact)
on two calls in a row, the second on a smaller hierarchy than the first, in
the blocking form and in the form that leaves the count on the device; and
the size limit of its static scratch."""
import ctypes as C

import numpy as np
import pytest

from paper_2607_14481_amd import hierarchy as H
from paper_2607_14481_amd import scenes as S

from ._util import log, params_to_device

pytestmark = pytest.mark.gpu


def _street_tree(seed, n_leaves, levels, deg=1):
    rng = np.random.default_rng(seed)
    means = np.c_[rng.uniform(0, 400, n_leaves), rng.uniform(-4, 4, n_leaves), rng.uniform(0, 3, n_leaves)]
    return H.build(S._gaussian_body(rng, means, deg), levels=levels)


def _both_cuts(h, cam, tau, label):
    import torch
    from paper_2607_14481_amd import gsr
    deg = h.nodes.sh_degree
    nodes = params_to_device(h.nodes)
    parent = torch.tensor(h.parent.astype(np.int32), device="cuda")
    counts = torch.tensor(h.child_count.astype(np.int32), device="cuda")
    w2c = torch.tensor(np.asarray(cam.world_to_cam, np.float32), device="cuda")
    n = h.nodes.n
    ref = gsr.hierarchy_cut(nodes, deg, parent, counts, cam, w2c, tau)  # caller-provided scratch
    m_ref = int(ref.numel())
    out = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    m = gsr.hierarchy_cut_static(nodes, deg, parent, counts, cam, w2c, tau, out)
    log(f"{label}: {n} nodes, cut {m} (with caller scratch {m_ref})")
    assert m == m_ref
    assert torch.equal(out[:m], ref)
    # the device-count form: nothing read back, the count stays on the device
    out2 = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    cnt = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    assert gsr.hierarchy_cut_static(nodes, deg, parent, counts, cam, w2c, tau, out2, count=cnt) is None
    torch.cuda.synchronize()
    assert int(cnt.item()) == m_ref
    assert torch.equal(out2[:m_ref], ref)
    per_level = np.bincount(h.level_of(ref.cpu().numpy()), minlength=h.levels)
    log(f"{label}: cut per level {per_level.tolist()}")
    return per_level


def test_static_cut_matches_the_scratch_cut_on_two_calls():
    eye = np.array([-1.0, 0.0, 1.5])
    cam = S.pinhole(320, 180, S.look_at(eye, eye + np.array([1.0, 0.02, 0.0])))
    big = _street_tree(41, 120_000, 6)
    small = _street_tree(42, 4_000, 4)
    lv = _both_cuts(big, cam, 1.5, "first call (120k leaves)")
    assert lv[1:].sum() > 0  # the cut mixes levels
    _both_cuts(small, cam, 1.5, "second call (4k leaves)")
    _both_cuts(big, cam, 3.0, "third call (120k leaves, coarser threshold)")


def test_static_cut_size_limit_and_arguments():
    from paper_2607_14481_amd import gsr
    L = gsr.lib()
    cams = gsr.cameras([S.pinhole(64, 48, S.look_at([0, 0, -3]))])
    g = gsr.gsr_gaussians()
    g.sh_degree = 0
    g.n = gsr.HIERARCHY_CUT_STATIC_MAX_NODES + 1
    n_cut = C.c_int64(-1)
    rc = L.gsr_hierarchy_cut_static(C.byref(g), None, None, cams, None, 1.5, None, None, C.byref(n_cut), None)
    assert rc == gsr.GSR_ERR_UNSUPPORTED and "exceeds" in gsr.last_error()
    g.n = 10
    rc = L.gsr_hierarchy_cut_static(C.byref(g), None, None, cams, None, 1.5, None, None, None, None)
    assert rc == gsr.GSR_ERR_INVALID_ARGUMENT and "n_cut" in gsr.last_error()
    g.n = 0
    assert L.gsr_hierarchy_cut_static(C.byref(g), None, None, cams, None, 1.5, None, None, C.byref(n_cut),
                                      None) == gsr.GSR_OK
    assert n_cut.value == 0
