"""Pins of the FP64 level-of-detail cut reference (oracle/hierarchy_cut.py):
a hand-built tree, and the per-node characterisation (in the cut iff it stops
while all its ancestors descend) written out separately on random trees."""
import numpy as np

from oracle import hierarchy_cut as HC
from paper_2607_14481_amd import hierarchy as H
from paper_2607_14481_amd import scenes as S


def test_hand_built_tree():
    # camera at the origin looking down +z (identity pose), focal 100:
    # S = 100 * scale / distance.
    #   0 root   (scale 1.0 at 10 m: S = 10)   -> descends
    #   1 child  (scale 0.1 at 20 m: S = 0.5)  -> stops: in the cut, its leaves 4, 5 are not
    #   2 child  (scale 0.5 at 10 m: S = 5)    -> descends to leaves 6, 7
    #   3 leaf   (scale 1.0 at 10 m: S = 10)   -> leaf: in the cut
    #   8 root   (scale 0.001 at 10 m: S = 0.01, leaf count 0) -> in the cut
    parent = np.array([-1, 0, 0, 0, 1, 1, 2, 2, -1])
    means = np.array([[0, 0, 10], [0, 0, 20], [0, 0, 10], [0, 0, 10], [0, 0, 20], [0, 0, 20],
                      [0, 0, 10], [0, 0, 10], [0, 0, 10]], float)
    scales = np.array([1.0, 0.1, 0.5, 1.0, 0.05, 0.05, 0.2, 0.2, 0.001])
    ls = np.log(np.repeat(scales[:, None], 3, 1))
    got = HC.cut(means, ls, parent, np.eye(4), 100.0, 1.5)
    np.testing.assert_array_equal(got, [1, 3, 6, 7, 8])


def _brute(means, ls, parent, counts, w2c, f, tau):
    S_ = HC.screen_size(means, ls, w2c, f)
    out = []
    for i in range(len(parent)):
        if counts[i] > 0 and S_[i] >= tau:
            continue
        a, ok = parent[i], True
        while a >= 0:
            if not (counts[a] > 0 and S_[a] >= tau):
                ok = False
                break
            a = parent[a]
        if ok:
            out.append(i)
    return np.array(out)


def test_cut_equals_the_per_node_characterisation():
    rng = np.random.default_rng(3)
    for trial in range(4):
        n = int(rng.integers(200, 1200))
        means = np.c_[rng.uniform(0, 300, n), rng.uniform(-3, 3, n), rng.uniform(0, 3, n)]
        h = H.build(S._gaussian_body(rng, means, 0), levels=4)
        cam = S.pinhole(160, 120, S.look_at([-1, 0, 1.5], [10, rng.uniform(-1, 1), 1.5]))
        nodes = h.nodes
        parent = h.parent
        counts = h.child_count
        got = HC.cut(nodes.means, nodes.log_scales, parent, cam.world_to_cam, cam.fx, 1.5)
        ref = _brute(nodes.means, nodes.log_scales, parent, counts, cam.world_to_cam, cam.fx, 1.5)
        np.testing.assert_array_equal(got, ref)
        # every leaf has exactly one node of the cut on its way to the root
        in_cut = np.zeros(len(parent), bool)
        in_cut[got] = True
        for leaf in range(h.level_start[1]):
            a, hits = leaf, 0
            while a >= 0:
                hits += in_cut[a]
                a = parent[a]
            assert hits == 1
