"""Pins of the FP64 oracle against mathematics that does not come from the
oracle itself: library routines (scipy rotations, scipy spherical harmonics,
scipy's matrix exponential), closed forms, exact invariances, brute force and
finite differences.  CPU only.

The paper prints no worked rasterizer example (its renderer is one sentence in
Sec. 5.2), so every pin here is mathematical.
"""
import math

import numpy as np
import pytest
from scipy.linalg import expm
from scipy.spatial.transform import Rotation
from scipy.special import sph_harm_y

from oracle import dense as D
from oracle import oracle as O
from paper_2607_14481_amd import scenes as S

C0 = 1.0 / (2.0 * math.sqrt(math.pi))


def _cam(w, h, f, cx=None, cy=None, pose=None, near=0.2):
    return S.Camera(w, h, f, f, w / 2.0 if cx is None else cx, h / 2.0 if cy is None else cy,
                    np.eye(4, dtype=np.float64) if pose is None else np.asarray(pose, np.float64), near)


def _scene(means, log_scales, quats, opac, sh, deg):
    return S.Scene(np.asarray(means, np.float64), np.asarray(log_scales, np.float64),
                   np.asarray(quats, np.float64), np.asarray(opac, np.float64),
                   np.asarray(sh, np.float64), deg)


# ---------------------------------------------------------------------------
# Rotation
# ---------------------------------------------------------------------------

def test_quaternion_matches_scipy_rotation():
    rng = np.random.default_rng(0)
    for _ in range(50):
        q = rng.standard_normal(4) * rng.uniform(0.1, 5.0)
        ref = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()  # scalar-last
        np.testing.assert_allclose(O.quat_to_rot(q), ref, atol=1e-13)
        np.testing.assert_allclose(O.quat_to_rot(-q), ref, atol=1e-13)


def test_quaternion_known_rotations():
    s = math.sqrt(0.5)
    # 90 degrees about x maps y -> z
    Rx = O.quat_to_rot([s, s, 0, 0])
    np.testing.assert_allclose(Rx @ [0, 1, 0], [0, 0, 1], atol=1e-15)
    Ry = O.quat_to_rot([s, 0, s, 0])
    np.testing.assert_allclose(Ry @ [0, 0, 1], [1, 0, 0], atol=1e-15)
    Rz = O.quat_to_rot([s, 0, 0, s])
    np.testing.assert_allclose(Rz @ [1, 0, 0], [0, 1, 0], atol=1e-15)
    R = O.quat_to_rot([0.3, -1.2, 0.7, 2.0])
    np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-14)
    assert abs(np.linalg.det(R) - 1.0) < 1e-14


# ---------------------------------------------------------------------------
# Spherical harmonics
# ---------------------------------------------------------------------------

def _real_sh_scipy(deg, dirs):
    """Real SH from scipy's complex SH (Condon-Shortley phase included):
    m < 0: sqrt(2) Im Y_l^|m|, m = 0: Y_l^0, m > 0: sqrt(2) Re Y_l^m; m = -l..l."""
    x, y, z = dirs[:, 0], dirs[:, 1], dirs[:, 2]
    theta = np.arccos(np.clip(z, -1, 1))
    phi = np.arctan2(y, x)
    cols = []
    for l in range(deg + 1):
        for m in range(-l, l + 1):
            Y = sph_harm_y(l, abs(m), theta, phi)
            if m < 0:
                cols.append(math.sqrt(2) * Y.imag)
            elif m == 0:
                cols.append(Y.real)
            else:
                cols.append(math.sqrt(2) * Y.real)
    return np.stack(cols, 1)


def test_sh_basis_matches_scipy():
    rng = np.random.default_rng(1)
    d = rng.standard_normal((200, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    for deg in range(4):
        np.testing.assert_allclose(O.sh_basis(deg, d), _real_sh_scipy(deg, d), atol=1e-12)


def test_sh_basis_orthonormal_by_quadrature():
    # Gauss-Legendre in cos(theta) x uniform phi: exact for the degree-6
    # polynomials that products of two degree-3 harmonics are.
    mu, wmu = np.polynomial.legendre.leggauss(12)
    phi = np.arange(24) * (2 * np.pi / 24)
    M, P = np.meshgrid(mu, phi, indexing="ij")
    W = np.outer(wmu, np.full(24, 2 * np.pi / 24)).reshape(-1)
    st = np.sqrt(1 - M ** 2)
    dirs = np.stack([st * np.cos(P), st * np.sin(P), M], -1).reshape(-1, 3)
    Y = O.sh_basis(3, dirs)
    gram = (Y * W[:, None]).T @ Y
    np.testing.assert_allclose(gram, np.eye(16), atol=1e-12)


# ---------------------------------------------------------------------------
# Projection: EWA covariance, centre, colour, tile box
# ---------------------------------------------------------------------------

def _random_pose(rng, dist=6.0):
    d = rng.standard_normal(3)
    d /= np.linalg.norm(d)
    return S.look_at(d * dist, target=rng.uniform(-0.3, 0.3, 3))


def test_projection_matches_pinhole_jacobian_and_library_pieces():
    rng = np.random.default_rng(2)
    n = 300
    cam = _cam(160, 120, 150.0, pose=_random_pose(rng))
    sc = _scene(rng.uniform(-1, 1, (n, 3)), rng.normal(-2.5, 0.5, (n, 3)), rng.standard_normal((n, 4)),
                rng.uniform(0.05, 0.95, n), rng.normal(0, 0.3, (n, 16, 3)), 3)
    pr = O.project(sc, cam)
    W = cam.world_to_cam[:3, :3]
    t = cam.world_to_cam[:3, 3]
    camc = -W.T @ t
    fx, fy, cx, cy = cam.fx, cam.fy, cam.cx, cam.cy

    def pin(p):
        return np.array([fx * p[0] / p[2] + cx, fy * p[1] / p[2] + cy])

    checked = 0
    for i in range(n):
        p = W @ sc.means[i] + t
        if p[2] <= cam.near:
            continue
        if abs(p[0] / p[2]) > 1.2 * cam.width / (2 * fx) or abs(p[1] / p[2]) > 1.2 * cam.height / (2 * fy):
            continue  # the Jacobian clamp is pinned separately
        # numerical Jacobian of the pinhole map
        J = np.zeros((2, 3))
        h = 1e-6
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            J[:, k] = (pin(p + e) - pin(p - e)) / (2 * h)
        R = Rotation.from_quat(np.roll(sc.quats[i], -1)).as_matrix()
        Sig = R @ np.diag(np.exp(2 * sc.log_scales[i])) @ R.T
        cov = J @ W @ Sig @ W.T @ J.T + 0.3 * np.eye(2)
        np.testing.assert_allclose(pr["cov"][i], [cov[0, 0], cov[0, 1], cov[1, 1]], rtol=1e-7, atol=1e-9)
        con = np.linalg.inv(cov)
        np.testing.assert_allclose(pr["conic"][i], [con[0, 0], con[0, 1], con[1, 1]], rtol=1e-7, atol=1e-9)
        np.testing.assert_allclose([pr["u"][i], pr["v"][i]], pin(p), rtol=1e-12)
        assert pr["z"][i] == pytest.approx(p[2], rel=1e-13)
        dvec = sc.means[i] - camc
        Y = _real_sh_scipy(3, (dvec / np.linalg.norm(dvec))[None])[0]
        rgb = np.maximum(Y @ sc.sh[i] + 0.5, 0.0)
        np.testing.assert_allclose(pr["rgb"][i], rgb, atol=1e-12)
        checked += 1
    assert checked > 100


def test_jacobian_clamp_outside_fov():
    # A Gaussian far to the side: the Jacobian is evaluated at x/z clamped to
    # 1.3 x the half-FOV tangent; y is unclamped.
    cam = _cam(64, 48, 60.0)
    lim = 1.3 * 64 / (2 * 60.0)
    mu = np.array([[3.0, 0.1, 2.0]])  # x/z = 1.5 > lim
    sc = _scene(mu, [[-0.5, -1.0, -0.7]], [[1.0, 0.2, -0.1, 0.3]], [0.9], np.zeros((1, 1, 3)), 0)
    pr = O.project(sc, cam)
    z = 2.0
    J = np.array([[60.0 / z, 0, -60.0 * lim / z], [0, 60.0 / z, -60.0 * 0.05 / z]])
    R = Rotation.from_quat(np.roll(sc.quats[0] / np.linalg.norm(sc.quats[0]), -1)).as_matrix()
    Sig = R @ np.diag(np.exp(2 * sc.log_scales[0])) @ R.T
    cov = J @ Sig @ J.T + 0.3 * np.eye(2)
    np.testing.assert_allclose(pr["cov"][0], [cov[0, 0], cov[0, 1], cov[1, 1]], rtol=1e-12)


def test_tile_box_is_exact_box_of_alpha_threshold_ellipse():
    rng = np.random.default_rng(3)
    n = 200
    cam = _cam(96, 80, 90.0)
    sc = _scene(np.c_[rng.uniform(-1, 1, (n, 2)), rng.uniform(2, 4, n)], rng.normal(-2.5, 0.6, (n, 3)),
                rng.standard_normal((n, 4)), rng.uniform(0.01, 0.99, n), np.zeros((n, 1, 3)), 0)
    pr = O.project(sc, cam)
    ys = np.linspace(-60, 60, 40001)
    for i in np.nonzero(pr["visible"])[0]:
        a, b, c = pr["cov"][i]
        Q = np.linalg.inv(np.array([[a, b], [b, c]]))
        o = pr["opacity"][i]
        u, v = pr["u"][i], pr["v"][i]

        def max_alpha_on_column(xc):
            dx = xc - u
            dy = ys + (v - 0)  # dy sampled around the centre
            dy = ys
            s = 0.5 * (Q[0, 0] * dx * dx + 2 * Q[0, 1] * dx * dy + Q[1, 1] * dy * dy)
            return o * np.exp(-s.min())

        x0, y0, x1, y1 = pr["rect"][i]
        thr = 1.0 / 255.0
        # the box reaches the ellipse on its first/last column, and the column
        # beyond it (unless clipped by the image) lies outside the ellipse
        assert max_alpha_on_column(x0 + 0.5) >= thr * (1 - 1e-6) or x0 == 0
        assert max_alpha_on_column(x1 + 0.5) >= thr * (1 - 1e-6) or x1 == cam.width - 1
        if x0 > 0:
            assert max_alpha_on_column(x0 - 0.5) < thr * (1 + 1e-6)
        if x1 < cam.width - 1:
            assert max_alpha_on_column(x1 + 1.5) < thr * (1 + 1e-6)
        # every pixel centre with alpha >= 1/255 is inside the box
        X, Y = np.meshgrid(np.arange(cam.width) + 0.5, np.arange(cam.height) + 0.5)
        dx, dy = X - u, Y - v
        s = 0.5 * (Q[0, 0] * dx * dx + 2 * Q[0, 1] * dx * dy + Q[1, 1] * dy * dy)
        hit = o * np.exp(-s) >= thr
        yy, xx = np.nonzero(hit)
        if len(xx):
            assert xx.min() >= x0 and xx.max() <= x1 and yy.min() >= y0 and yy.max() <= y1
        assert tuple(pr["trect"][i]) == (x0 // 16, y0 // 16, x1 // 16, y1 // 16)


# ---------------------------------------------------------------------------
# Binning and sort order
# ---------------------------------------------------------------------------

def test_binning_order_and_membership():
    wl = S.small_view(seed=11, n=400, width=100, height=75)
    cam = wl.cameras[0]
    pr = O.project(wl.scene, cam)
    tx, ty = O.tile_grid(cam)
    tiles, gids, ranges = O.bin_pairs(pr["visible"], pr["trect"], pr["zbits"], tx, ty)
    triples = [(int(t), int(pr["zbits"][g]), int(g)) for t, g in zip(tiles, gids)]
    assert triples == sorted(triples)
    # membership: exactly the tiles of each visible Gaussian's tile box
    want = set()
    for g in np.nonzero(pr["visible"])[0]:
        a, b, c, d = pr["trect"][g]
        for yy in range(b, d + 1):
            for xx in range(a, c + 1):
                want.add((yy * tx + xx, int(g)))
    assert set(zip(tiles.tolist(), gids.tolist())) == want
    assert len(want) == len(tiles)
    for t in range(tx * ty):
        s0, s1 = ranges[t]
        assert np.all(tiles[s0:s1] == t)
    assert ranges[:, 1].max() == len(tiles)


# ---------------------------------------------------------------------------
# Closed forms
# ---------------------------------------------------------------------------

def test_single_isotropic_gaussian_closed_form():
    W = H = 33
    f, z, r, o = 40.0, 3.0, 0.05, 0.7
    rgb = np.array([0.6, 0.3, 0.9])
    bg = np.array([0.2, 0.3, 0.4])
    cam = _cam(W, H, f, cx=16.5, cy=16.5)
    sh = ((rgb - 0.5) / C0).reshape(1, 1, 3)
    sc = _scene([[0.0, 0.0, z]], [[math.log(r)] * 3], [[0.3, 0.0, 0.0, 0.0]], [o], sh, 0)
    g = S.random_upstream(3, (H, W, 3)).astype(np.float64)
    out = O.render(sc, cam, bg=bg, dL_dimg=g)
    sxx = f * f * r * r / (z * z) + 0.3
    X, Y = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
    dx, dy = 16.5 - X, 16.5 - Y
    sig = 0.5 * (dx ** 2 + dy ** 2) / sxx
    al = o * np.exp(-sig)
    on = al >= 1 / 255
    img = np.where(on[..., None], rgb * al[..., None] + (1 - al[..., None]) * bg, bg)
    np.testing.assert_allclose(out["img"], img, atol=1e-14)
    np.testing.assert_allclose(out["T"], np.where(on, 1 - al, 1.0), atol=1e-14)
    # gradients
    gd = (g * (rgb - bg)).sum(-1)  # dL/dalpha per pixel
    dsig = -gd * al * on          # dL/dsigma
    np.testing.assert_allclose(out["opacities"][0], (gd * np.exp(-sig) * on).sum(), rtol=1e-12)
    np.testing.assert_allclose(out["sh"][0, 0], (g * (al * on)[..., None]).sum((0, 1)) * C0, rtol=1e-12)
    # d(sigma)/d(Sigma'_xx) + d(sigma)/d(Sigma'_yy) with Sigma'_xx = Sigma'_yy
    dsig_dsxx = -sig / sxx
    np.testing.assert_allclose(out["log_scales"][0].sum(),
                               (dsig * dsig_dsxx * 2 * f * f * r * r / (z * z)).sum(), rtol=1e-10)
    dLdz = (dsig * dsig_dsxx * (-2 * f * f * r * r / z ** 3)).sum()
    dLdx = (dsig * (-dx) / sxx).sum() * f / z * -1
    dLdy = (dsig * (-dy) / sxx).sum() * f / z * -1
    np.testing.assert_allclose(out["means"][0], [dLdx, dLdy, dLdz], rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(out["w2c"][:3, 3], [dLdx, dLdy, dLdz], rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(out["quats"][0], 0.0, atol=1e-12)


def test_two_gaussian_ordering_closed_form():
    W = H = 17
    cam = _cam(W, H, 20.0, cx=8.5, cy=8.5)
    # index 0 is the BACK Gaussian: depth order, not index order, decides
    rgb = np.array([[0.9, 0.1, 0.2], [0.2, 0.8, 0.4]])
    sh = ((rgb - 0.5) / C0).reshape(2, 1, 3)
    sc = _scene([[0, 0, 5.0], [0, 0, 3.0]], [[-2.0] * 3, [-2.3] * 3], [[1, 0, 0, 0]] * 2, [0.6, 0.45], sh, 0)
    bg = np.array([0.05, 0.1, 0.15])
    out = O.render(sc, cam, bg=bg)
    a_front, a_back = 0.45, 0.6  # at the centre pixel sigma = 0
    want = rgb[1] * a_front + rgb[0] * a_back * (1 - a_front) + (1 - a_front) * (1 - a_back) * bg
    np.testing.assert_allclose(out["img"][8, 8], want, atol=1e-15)
    assert out["T"][8, 8] == pytest.approx((1 - a_front) * (1 - a_back), abs=1e-15)


def test_alpha_clamp_and_early_stop():
    # 12 stacked opaque Gaussians on the axis: alpha clamps at 0.99, and the
    # third would take T below 1e-4 (0.01^3 = 1e-6), so exactly two contribute.
    n = 12
    cam = _cam(9, 9, 10.0, cx=4.5, cy=4.5)
    sh = np.zeros((n, 1, 3))
    sc = _scene([[0, 0, 2.0 + 0.1 * i] for i in range(n)], [[-1.0] * 3] * n, [[1, 0, 0, 0]] * n,
                [0.999] * n, sh, 0)
    g = np.zeros((9, 9, 3))
    g[4, 4] = 1.0  # upstream only at the centre pixel, where sigma = 0
    out = O.render(sc, cam, bg=(1, 1, 1), dL_dimg=g)
    assert out["T"][4, 4] == pytest.approx(0.01 * 0.01, rel=1e-12)
    assert out["n_contrib"][4, 4] == 2
    # colour 0.5 everywhere: img = 0.5 (1 - T) + T
    assert out["img"][4, 4, 0] == pytest.approx(0.5 * (1 - 1e-4) + 1e-4, rel=1e-12)
    # clamped alpha passes no gradient to opacity; Gaussians after the stop get none at all
    assert np.all(out["opacities"] == 0.0)
    assert np.all(out["sh"][:2] != 0.0) and np.all(out["sh"][2:] == 0.0)


# ---------------------------------------------------------------------------
# Invariants
# ---------------------------------------------------------------------------

def _white(scene):
    sh = np.zeros_like(np.asarray(scene.sh, np.float64))
    sh[:, 0, :] = 0.5 / C0
    return S.Scene(scene.means, scene.log_scales, scene.quats, scene.opacities, sh, scene.sh_degree)


@pytest.mark.parametrize("seed", [21, 22])
def test_transmittance_invariants(seed):
    wl = S.small_view(seed=seed, n=1500, width=64, height=48, log_scale_mean=-2.2)
    sc = _white(wl.scene)
    sc.opacities = np.clip(np.asarray(sc.opacities, np.float64) * 1.3, 0, 0.995)
    cam = wl.cameras[0]
    o0 = O.render(sc, cam, bg=(0, 0, 0))
    np.testing.assert_allclose(o0["img"], np.repeat(1 - o0["T"][..., None], 3, -1), atol=1e-13)
    o1 = O.render(sc, cam, bg=(1, 1, 1))
    np.testing.assert_allclose(o1["img"], 1.0, atol=1e-13)
    assert o0["T"].min() >= 1e-4
    assert (o0["T"] < 2e-4).any(), "scene should reach the early stop somewhere"


def test_translation_invariance_identity():
    # translating scene and camera together leaves the image unchanged:
    # sum_i dL/dmu_i = R_cw^T dL/dt_cw
    rng = np.random.default_rng(5)
    n = 150
    cam = _cam(80, 64, 70.0, pose=_random_pose(rng, 5.0))
    sc = _scene(rng.uniform(-1, 1, (n, 3)), rng.normal(-2.3, 0.4, (n, 3)), rng.standard_normal((n, 4)),
                rng.uniform(0.1, 0.95, n), rng.normal(0, 0.4, (n, 16, 3)), 3)
    g = rng.standard_normal((64, 80, 3))
    out = O.render(sc, cam, bg=(0.1, 0.2, 0.3), dL_dimg=g)
    W = cam.world_to_cam[:3, :3]
    lhs = out["means"].sum(0)
    rhs = W.T @ out["w2c"][:3, 3]
    np.testing.assert_allclose(lhs, rhs, rtol=1e-10, atol=1e-10 * np.abs(lhs).max())


def _qmul(a, b):
    aw, av = a[0], a[1:]
    bw, bv = b[..., 0], b[..., 1:]
    w = aw * bw - bv @ av
    v = aw * bv + bw[..., None] * av + np.cross(av, bv)
    return np.concatenate([w[..., None], v], -1)


def test_rotation_invariance_identity_degree0():
    # rotating scene (means and Gaussian orientations) and camera together
    # about the origin leaves a degree-0 image unchanged; the derivative of
    # that along each axis k is zero:
    #   sum_i g_mu_i . (k x mu_i) + sum_i g_q_i . ((0, k/2) (x) q_i) - <g_W, W [k]x> = 0
    rng = np.random.default_rng(6)
    n = 120
    cam = _cam(72, 60, 70.0, pose=_random_pose(rng, 5.0))
    sc = _scene(rng.uniform(-1, 1, (n, 3)), rng.normal(-2.3, 0.4, (n, 3)), rng.standard_normal((n, 4)),
                rng.uniform(0.1, 0.95, n), rng.normal(0, 0.4, (n, 1, 3)), 0)
    g = rng.standard_normal((60, 72, 3))
    out = O.render(sc, cam, bg=(0.3, 0.2, 0.1), dL_dimg=g)
    W = cam.world_to_cam[:3, :3]
    scale = np.abs(out["means"]).sum() + np.abs(out["w2c"]).sum()
    for k in np.eye(3):
        K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
        term_mu = np.sum(out["means"] * (sc.means @ K.T))
        dq = _qmul(np.r_[0.0, k / 2], sc.quats)
        term_q = np.sum(out["quats"] * dq)
        term_w = -np.sum(out["w2c"][:3, :3] * (W @ K))
        assert abs(term_mu + term_q + term_w) < 1e-10 * scale


# ---------------------------------------------------------------------------
# Independent implementations and finite differences
# ---------------------------------------------------------------------------

CASES = [
    dict(seed=31, n=60, w=50, h=37, deg=0),
    dict(seed=32, n=80, w=40, h=40, deg=1),
    dict(seed=33, n=70, w=33, h=29, deg=2),
    dict(seed=34, n=90, w=48, h=36, deg=3),
]


def _wide_scene(c):
    """small_view recipe widened so that the Jacobian clamp, the near plane,
    colour clamping and the 0.99 alpha clamp all occur."""
    wl = S.small_view(seed=c["seed"], n=c["n"], width=c["w"], height=c["h"], sh_degree=c["deg"],
                      z_range=(-0.5, 4.0), xy_half=2.5, log_scale_mean=-1.8)
    sc = wl.scene
    rng = np.random.default_rng(c["seed"])
    op = np.asarray(sc.opacities, np.float64).copy()
    op[rng.choice(len(op), len(op) // 6, replace=False)] = 0.999
    sh = np.asarray(sc.sh, np.float64).copy()
    if sh.shape[1] > 1:
        sh[:, 1:] *= 6.0
    return _scene(sc.means, sc.log_scales, sc.quats, op, sh, sc.sh_degree), wl.cameras[0]


@pytest.mark.parametrize("c", CASES, ids=lambda c: f"deg{c['deg']}")
def test_dense_and_tiled_oracles_agree(c):
    sc, cam = _wide_scene(c)
    rng = np.random.default_rng(c["seed"] + 100)
    bg = rng.uniform(0, 1, 3)
    g = rng.standard_normal((c["h"], c["w"], 3))
    a = O.render(sc, cam, bg=bg, dL_dimg=g)
    b = D.render(sc, cam, bg=bg, dL_dimg=g)
    np.testing.assert_allclose(a["img"], b["img"], atol=1e-12)
    np.testing.assert_allclose(a["T"], b["T"], atol=1e-12)
    for k in ("means", "log_scales", "quats", "opacities", "sh", "w2c"):
        ref = b[k]
        assert np.linalg.norm(a[k] - ref) <= 1e-10 * max(np.linalg.norm(ref), 1e-30), k
    # the scenes really exercise the clamps
    pr = O.project(sc, cam)
    assert (~pr["visible"]).any()


def _loss(sc, cam, g, bg):
    return float((O.render(sc, cam, bg=bg)["img"] * g).sum())


def test_gradients_match_central_differences():
    # seed chosen so that no pixel has a decision (alpha vs 1/255 or 0.99,
    # T vs 1e-4, depth order) within a margin 100x wider than any h-step moves
    rng = np.random.default_rng(48)
    n = 6
    cam = _cam(28, 22, 30.0, pose=S.look_at([0.3, -0.2, -4.0], target=[0, 0, 0.5], up=[0, -1, 0]))
    sc = _scene(np.c_[rng.uniform(-0.4, 0.4, (n, 2)), rng.uniform(-0.3, 0.8, n)],
                rng.normal(-1.9, 0.2, (n, 3)), rng.standard_normal((n, 4)), rng.uniform(0.3, 0.9, n),
                rng.normal(0, 0.3, (n, 4, 3)), 1)
    bg = np.array([0.2, 0.1, 0.3])
    g = rng.standard_normal((22, 28, 3))
    out = O.render(sc, cam, bg=bg, dL_dimg=g)
    # FD is valid only away from the discrete decisions
    amb = O.render(sc, cam, bg=bg, eps_alpha=1e-4, eps_t=1e-6)["ambig"]
    assert not amb.any()
    h = 1e-6
    for name in ("means", "log_scales", "quats", "opacities", "sh"):
        arr = getattr(sc, name)
        fd = np.zeros_like(arr)
        for idx in np.ndindex(arr.shape):
            keep = arr[idx]
            arr[idx] = keep + h
            lp = _loss(sc, cam, g, bg)
            arr[idx] = keep - h
            lm = _loss(sc, cam, g, bg)
            arr[idx] = keep
            fd[idx] = (lp - lm) / (2 * h)
        np.testing.assert_allclose(out[name], fd, rtol=1e-5, atol=1e-6 * np.abs(fd).max(), err_msg=name)
    # 6-DoF pose gradient through the SE(3) exponential (scipy expm)
    T0 = cam.world_to_cam.copy()
    fd = np.zeros(6)
    for i in range(6):
        xi = np.zeros(6)
        vals = []
        for sgn in (1, -1):
            xi[i] = sgn * h
            Xi = np.zeros((4, 4))
            Xi[:3, :3] = [[0, -xi[5], xi[4]], [xi[5], 0, -xi[3]], [-xi[4], xi[3], 0]]
            Xi[:3, 3] = xi[:3]
            c2 = _cam(28, 22, 30.0, pose=expm(Xi) @ T0)
            vals.append(_loss(sc, c2, g, bg))
        fd[i] = (vals[0] - vals[1]) / (2 * h)
    np.testing.assert_allclose(out["twist"], fd, rtol=1e-5, atol=1e-6 * np.abs(fd).max())


def test_tile_mask_restricts_exactly():
    # the sampled-tile mode used for full-size parity equals the full render
    wl = S.small_view(seed=12, n=500, width=90, height=70, sh_degree=1)
    sc, cam = wl.scene, wl.cameras[0]
    tx, ty = O.tile_grid(cam)
    rng = np.random.default_rng(0)
    mask = np.zeros(tx * ty, np.uint8)
    mask[rng.choice(tx * ty, 7, replace=False)] = 1
    pix = np.zeros((70, 90), bool)
    for t in np.nonzero(mask)[0]:
        pix[(t // tx) * 16:(t // tx + 1) * 16, (t % tx) * 16:(t % tx + 1) * 16] = True
    g = rng.standard_normal((70, 90, 3)) * pix[..., None]
    full = O.render(sc, cam, dL_dimg=g)
    part = O.render(sc, cam, dL_dimg=g, tile_mask=mask)
    np.testing.assert_array_equal(part["img"][pix], full["img"][pix])
    for k in ("means", "log_scales", "quats", "opacities", "sh", "w2c"):
        np.testing.assert_allclose(part[k], full[k], rtol=1e-13, atol=1e-15)
