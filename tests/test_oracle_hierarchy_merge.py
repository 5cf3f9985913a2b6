"""Pins of the FP64 hierarchy merge reference (oracle/hierarchy_merge.py)
against what the mathematics fixes: identical children, a two-child closed
form, the mixture's sampled moments, the KL(mixture || single) minimum, the
factorisation, scipy's rotations, and ragged groups."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import hierarchy_merge as M


def _random_children(rng, k, K=4):
    means = rng.normal(0, 1.0, (k, 3))
    ls = rng.normal(-1.0, 0.4, (k, 3))
    q = rng.normal(size=(k, 4))
    o = rng.uniform(0.05, 0.95, k)
    sh = rng.normal(size=(k, K, 3))
    return means, ls, q, o, sh


def test_covariance_uses_the_rotation_of_the_quaternion():
    rng = np.random.default_rng(0)
    for _ in range(10):
        q = rng.normal(size=4)
        s = rng.normal(size=3)
        R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()  # scipy: scalar last
        np.testing.assert_allclose(M.rotation(q), R, atol=1e-14)
        np.testing.assert_allclose(M.covariance(s, q), R @ np.diag(np.exp(2 * s)) @ R.T, rtol=1e-12, atol=1e-14)


def test_identical_children_merge_to_themselves():
    rng = np.random.default_rng(1)
    m, s, q, o, sh = _random_children(rng, 1)
    for k in (1, 2, 5, 8):
        r = M.merge_group(np.repeat(m, k, 0), np.repeat(s, k, 0), np.repeat(q, k, 0), np.repeat(o, k), np.repeat(sh, k, 0))
        np.testing.assert_allclose(r["mean"], m[0], rtol=1e-14)
        np.testing.assert_allclose(r["cov"], M.covariance(s[0], q[0]), rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(r["sh"], sh[0], rtol=1e-13)
        assert r["opacity"] == pytest.approx(1 - (1 - o[0]) ** k, rel=1e-14)


def test_two_isotropic_children_closed_form():
    a, rad, o = 0.7, 0.2, 0.4
    means = np.array([[-a, 0, 0], [a, 0, 0]])
    ls = np.full((2, 3), np.log(rad))
    q = np.array([[1.0, 0, 0, 0], [0.3, -0.2, 0.5, 0.1]])  # isotropic: the rotation is irrelevant
    sh = np.array([[[1.0, 2.0, 3.0]], [[3.0, 2.0, 1.0]]])
    r = M.merge_group(means, ls, q, [o, o], sh)
    np.testing.assert_allclose(r["mean"], 0.0, atol=1e-15)
    np.testing.assert_allclose(r["cov"], np.diag([rad ** 2 + a ** 2, rad ** 2, rad ** 2]), atol=1e-14)
    assert r["opacity"] == pytest.approx(1 - (1 - o) ** 2)
    np.testing.assert_allclose(r["sh"], [[2.0, 2.0, 2.0]], rtol=1e-14)
    # unequal opacities shift the mean towards the more opaque child
    r2 = M.merge_group(means, ls, q, [0.2, 0.6], sh)
    np.testing.assert_allclose(r2["mean"], [a * (0.6 - 0.2) / 0.8, 0, 0], atol=1e-15)
    np.testing.assert_allclose(r2["sh"], [[0.25 * 1 + 0.75 * 3, 2.0, 0.25 * 3 + 0.75 * 1]], rtol=1e-14)


def test_moments_of_samples_from_the_mixture():
    rng = np.random.default_rng(2)
    m, s, q, o, sh = _random_children(rng, 6)
    r = M.merge_group(m, s, q, o, sh)
    n = 400_000
    w = o / o.sum()
    comp = rng.choice(len(o), n, p=w)
    z = rng.standard_normal((n, 3))
    x = np.empty((n, 3))
    for i in range(len(o)):
        L = np.linalg.cholesky(M.covariance(s[i], q[i]))
        sel = comp == i
        x[sel] = m[i] + z[sel] @ L.T
    mean = x.mean(0)
    cov = np.cov(x.T)
    se_mean = np.sqrt(np.diag(r["cov"]) / n)
    assert np.all(np.abs(mean - r["mean"]) < 5 * se_mean)
    # sampling error of a covariance entry ~ sqrt((S_aa S_bb + S_ab^2) / n), plus the mixture's extra kurtosis
    d = np.sqrt(np.diag(r["cov"]))
    tol = 8 * np.outer(d, d) / np.sqrt(n)
    assert np.all(np.abs(cov - r["cov"]) < tol)


def test_the_merge_minimises_the_kl_divergence():
    """KL(mixture || q) = cross-entropy(q) - entropy(mixture): the merged
    Gaussian must have the lowest cross-entropy among perturbed ones."""
    rng = np.random.default_rng(3)
    for _ in range(5):
        m, s, q, o, sh = _random_children(rng, 8)
        covs = [M.covariance(a, b) for a, b in zip(s, q)]
        r = M.merge_group(m, s, q, o, sh)
        best = M.cross_entropy(m, covs, o, r["mean"], r["cov"])
        for _ in range(50):
            dmu = rng.normal(0, 0.05, 3)
            A = rng.normal(0, 0.05, (3, 3))
            cov2 = r["cov"] + (A + A.T) / 2
            if np.linalg.eigvalsh(cov2).min() <= 0:
                continue
            assert M.cross_entropy(m, covs, o, r["mean"] + dmu, r["cov"]) > best
            assert M.cross_entropy(m, covs, o, r["mean"], cov2) > best
        # uniform weights (ignoring opacity) give a worse fit to the opacity-weighted mixture
        r_u = M.merge_group(m, s, q, np.ones_like(o), sh)
        assert M.cross_entropy(m, covs, o, r_u["mean"], r_u["cov"]) > best


def test_factorisation_reconstructs_the_covariance():
    rng = np.random.default_rng(4)
    for _ in range(20):
        m, s, q, o, sh = _random_children(rng, int(rng.integers(1, 9)))
        r = M.merge_group(m, s, q, o, sh)
        R, ls = r["rot"], r["log_scales"]
        assert np.linalg.det(R) == pytest.approx(1.0, abs=1e-12)
        np.testing.assert_allclose(R.T @ R, np.eye(3), atol=1e-12)
        assert np.all(np.diff(ls) >= 0)
        np.testing.assert_allclose(R @ np.diag(np.exp(2 * ls)) @ R.T, r["cov"], rtol=1e-10, atol=1e-14)
        qq = M.quat_of(R)
        assert qq[0] >= 0 and np.linalg.norm(qq) == pytest.approx(1.0)
        ref = Rotation.from_matrix(R).as_quat()  # (x, y, z, w)
        ref = np.array([ref[3], ref[0], ref[1], ref[2]])
        np.testing.assert_allclose(qq, ref * np.sign(ref[0]), atol=1e-9)
        np.testing.assert_allclose(M.covariance(ls, qq), r["cov"], rtol=1e-8, atol=1e-14)


def test_ragged_levels():
    rng = np.random.default_rng(5)
    m, s, q, o, sh = _random_children(rng, 19)
    lv = M.build_levels(m, s, q, o, sh, levels=5)
    assert [len(x) for x in lv] == [19, 3, 1]
    last = M.merge_group(m[16:], s[16:], q[16:], o[16:], sh[16:])  # the short last group
    np.testing.assert_allclose(lv[1][2]["mean"], last["mean"], rtol=1e-14)
    assert lv[1][2]["opacity"] == pytest.approx(1 - np.prod(1 - o[16:]))
    root = lv[2][0]
    kids = lv[1]
    exp = M.merge_group([k["mean"] for k in kids], [k["log_scales"] for k in kids], [k["quat"] for k in kids],
                        [k["opacity"] for k in kids], [k["sh"] for k in kids])
    np.testing.assert_allclose(root["cov"], exp["cov"], rtol=1e-12)
    assert root["opacity"] == pytest.approx(1 - np.prod(1 - o))
