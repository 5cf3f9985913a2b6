"""Host-side level-of-detail hierarchy (the hierarchical workload's input
preparation): merge, factorisation, Morton order and the per-view cut, each
checked against mathematics that does not reuse the code under test."""
import numpy as np

from paper_2607_14481_amd import hierarchy as H
from paper_2607_14481_amd import scenes as S


def _random_children(rng, n, k=4):
    mu = rng.normal(0, 1, (n, 3))
    a = rng.normal(0, 0.3, (n, 3, 3))
    cov = a @ a.transpose(0, 2, 1) + 0.01 * np.eye(3)
    opac = rng.uniform(0.05, 0.95, n)
    sh = rng.normal(0, 1, (n, k, 3))
    return mu, cov, opac, sh


def test_spread_bits_and_morton_order():
    assert int(H._spread_bits(np.array([0b111]))[0]) == 0b1001001
    assert int(H._spread_bits(np.array([0x1FFFFF]))[0]) == int("001" * 21, 2)
    # along one axis the codes increase with the coordinate
    p = np.zeros((50, 3))
    p[:, 0] = np.linspace(0, 1, 50)
    c = H.morton_codes(p)
    assert np.all(np.diff(c.astype(np.float64)) > 0)
    # interleaving order: x is bit 0, y bit 1, z bit 2 of each triple
    q = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 1]], np.float64)
    c = H.morton_codes(q)
    top = np.uint64(7) << np.uint64(60)
    assert [int((x & top) >> np.uint64(60)) for x in c] == [0, 1, 2, 4, 7]


def test_merge_of_identical_children_is_the_child():
    rng = np.random.default_rng(0)
    mu, cov, opac, sh = _random_children(rng, 1)
    k = 8
    mp, cp, op, sp = H.merge_groups(np.repeat(mu, k, 0), np.repeat(cov, k, 0), np.repeat(opac, k, 0),
                                    np.repeat(sh, k, 0), np.array([0]))
    np.testing.assert_allclose(mp[0], mu[0], atol=1e-12)
    np.testing.assert_allclose(cp[0], cov[0], atol=1e-12)
    np.testing.assert_allclose(sp[0], sh[0], atol=1e-12)
    np.testing.assert_allclose(op[0], 1 - (1 - opac[0]) ** k, rtol=1e-12)


def test_merge_matches_sampled_mixture_moments():
    # the parent must carry the mean and covariance of the opacity-weighted
    # mixture of its children: checked against samples drawn from that mixture
    rng = np.random.default_rng(1)
    mu, cov, opac, sh = _random_children(rng, 5)
    mp, cp, _, _ = H.merge_groups(mu, cov, opac, sh, np.array([0]))
    m = 400_000
    comp = rng.choice(5, size=m, p=opac / opac.sum())
    chol = np.linalg.cholesky(cov)
    x = mu[comp] + np.einsum("nij,nj->ni", chol[comp], rng.standard_normal((m, 3)))
    np.testing.assert_allclose(mp[0], x.mean(0), atol=0.01)
    np.testing.assert_allclose(cp[0], np.cov(x.T), atol=0.02)


def test_merge_groups_are_independent_and_ragged():
    rng = np.random.default_rng(2)
    mu, cov, opac, sh = _random_children(rng, 19)
    starts = np.array([0, 8, 16])
    mp, cp, op, sp = H.merge_groups(mu, cov, opac, sh, starts)
    for g, (a, b) in enumerate(((0, 8), (8, 16), (16, 19))):
        m1, c1, o1, s1 = H.merge_groups(mu[a:b], cov[a:b], opac[a:b], sh[a:b], np.array([0]))
        np.testing.assert_allclose(mp[g], m1[0], rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(cp[g], c1[0], rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(op[g], o1[0], rtol=1e-12)


def test_quaternion_round_trip_and_covariance_factorisation():
    rng = np.random.default_rng(3)
    q = rng.standard_normal((500, 4))
    r = H.quat_to_rotation(q)
    # proper rotations
    np.testing.assert_allclose(r @ r.transpose(0, 2, 1), np.broadcast_to(np.eye(3), r.shape), atol=1e-12)
    np.testing.assert_allclose(np.linalg.det(r), 1.0, atol=1e-12)
    # 90 degrees about z: (w, x, y, z) = (cos 45, 0, 0, sin 45) maps x to y
    rz = H.quat_to_rotation(np.array([[np.cos(np.pi / 4), 0, 0, np.sin(np.pi / 4)]]))[0]
    np.testing.assert_allclose(rz @ [1, 0, 0], [0, 1, 0], atol=1e-12)
    q2 = H.rotation_to_quat(r)
    np.testing.assert_allclose(H.quat_to_rotation(q2), r, atol=1e-12)
    qn = q / np.linalg.norm(q, axis=1, keepdims=True)
    np.testing.assert_allclose(np.abs(np.sum(q2 * qn, 1)), 1.0, atol=1e-12)  # same up to sign
    _, cov, _, _ = _random_children(rng, 300)
    ls, qq = H.factor_covariance(cov.copy())
    np.testing.assert_allclose(H.covariance(ls, qq), cov, rtol=1e-9, atol=1e-12)


def _small_hierarchy(n=3000, levels=4):
    # a sparse 600 m street, so that coarse nodes fall under the threshold far away
    rng = np.random.default_rng(5)
    means = np.c_[rng.uniform(0, 600, n), rng.uniform(-3, 3, n), rng.uniform(0, 3, n)]
    leaves = S._gaussian_body(rng, means, 1)
    return leaves, H.build(leaves, levels)


def test_build_structure():
    leaves, h = _small_hierarchy()
    sizes = np.diff(h.level_start)
    expect = [3000]
    for _ in range(4):
        expect.append(-(-expect[-1] // 8))
    assert sizes.tolist() == expect
    # leaves are a permutation of the input
    a = np.lexsort(leaves.means.T)
    b = np.lexsort(h.nodes.means[:3000].T)
    np.testing.assert_array_equal(leaves.means[a], h.nodes.means[:3000][b])
    # children ranges tile each level exactly once and point back to their parent
    for l in range(1, h.levels):
        nodes = np.arange(h.level_start[l], h.level_start[l + 1])
        cs, cc = h.child_start[nodes], h.child_count[nodes]
        assert cs[0] == h.level_start[l - 1]
        np.testing.assert_array_equal(cs[1:], cs[:-1] + cc[:-1])
        assert cs[-1] + cc[-1] == h.level_start[l]
        for p, s0, c in zip(nodes, cs, cc):
            assert np.all(h.parent[s0:s0 + c] == p)
    assert np.all(h.parent[h.roots] == -1)


def test_cut_covers_every_leaf_once_and_respects_the_threshold():
    leaves, h = _small_hierarchy()
    cam = S.pinhole(160, 120, S.look_at([-1, 0, 1.5], [10, 0.5, 1.5]))
    tau = 1.5
    cut = H.select_cut(h, cam, tau)
    in_cut = np.zeros(h.level_start[-1], bool)
    in_cut[cut] = True
    # walk every leaf to its root: exactly one node on the way is in the cut
    node = np.arange(3000)
    hits = in_cut[node].astype(np.int64)
    alive = np.ones(3000, bool)
    for _ in range(h.levels):
        up = np.where(alive, h.parent[node], -1)
        alive = up >= 0
        node = np.where(alive, up, node)
        hits += alive & in_cut[node]
    assert not alive.any()
    assert np.all(hits == 1)
    s = H.screen_size(h, cut, cam)
    leaf = h.child_count[cut] == 0
    assert np.all(leaf | (s < tau))
    par = h.parent[cut]
    par = par[par >= 0]
    assert np.all(H.screen_size(h, par, cam) >= tau)
    lv = np.bincount(h.level_of(cut), minlength=h.levels)
    assert lv[0] > 0 and lv[1] > 0 and lv[2] > 0  # the cut mixes levels on this street
