"""Pins of the FP64 update oracle (oracle/update.py) against things it does
not share code with: torch's Adam, first-step closed forms, the SE(3)
exponential's closed form, and a similarity matrix built from axis-angle."""
import numpy as np
import pytest

from oracle import update as U

LRS = dict(means=1.6e-4, log_scales=5e-3, quats=1e-3, opacities=5e-2, sh_dc=2.5e-3, sh_rest=1.25e-4)


def _state(rng, n=50, deg=2):
    K = (deg + 1) ** 2
    shapes = dict(means=(n, 3), log_scales=(n, 3), quats=(n, 4), opacities=(n,), sh=(n, K, 3))
    p = {k: rng.standard_normal(s) for k, s in shapes.items()}
    p["opacities"] = rng.uniform(0.05, 0.95, n)
    zero = {k: np.zeros(s) for k, s in shapes.items()}
    return p, zero, shapes


def test_adam_matches_torch_adam_over_three_steps():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    p, zero, shapes = _state(rng)
    P, M, V = p, dict(zero), dict(zero)
    # torch reference: one parameter group per learning rate, opacity as a logit
    tp = {k: torch.tensor(p[k], dtype=torch.float64, requires_grad=True) for k in ("means", "log_scales", "quats")}
    sh_dc = torch.tensor(p["sh"][:, :1], dtype=torch.float64, requires_grad=True)
    sh_rest = torch.tensor(p["sh"][:, 1:], dtype=torch.float64, requires_grad=True)
    o = p["opacities"]
    logit = torch.tensor(np.log(o) - np.log1p(-o), dtype=torch.float64, requires_grad=True)
    groups = [{"params": [tp[k]], "lr": LRS[k]} for k in tp]
    groups += [{"params": [sh_dc], "lr": LRS["sh_dc"]}, {"params": [sh_rest], "lr": LRS["sh_rest"]},
               {"params": [logit], "lr": LRS["opacities"]}]
    opt = torch.optim.Adam(groups, betas=(0.9, 0.999), eps=1e-8)
    for step in (1, 2, 3):
        g = {k: rng.standard_normal(s) for k, s in shapes.items()}
        P, M, V = U.adam(P, g, M, V, step, LRS, 0.9, 0.999, 1e-8)
        for k in tp:
            tp[k].grad = torch.tensor(g[k])
        sh_dc.grad = torch.tensor(g["sh"][:, :1])
        sh_rest.grad = torch.tensor(g["sh"][:, 1:])
        sig = torch.sigmoid(logit.detach())
        logit.grad = sig * (1 - sig) * torch.tensor(g["opacities"])
        opt.step()
    for k in tp:
        np.testing.assert_allclose(P[k], tp[k].detach().numpy(), rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(P["sh"][:, :1], sh_dc.detach().numpy(), rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(P["sh"][:, 1:], sh_rest.detach().numpy(), rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(P["opacities"], torch.sigmoid(logit).detach().numpy(), rtol=1e-10)


def test_adam_first_step_is_a_signed_step_of_lr():
    # from zero moments, m_hat = g and v_hat = g^2: the step is -lr g / (|g| + eps)
    rng = np.random.default_rng(1)
    p, zero, shapes = _state(rng, n=20, deg=0)
    g = {k: rng.standard_normal(s) for k, s in shapes.items()}
    P, M, V = U.adam(p, g, zero, zero, 1, LRS, 0.9, 0.999, 1e-15)
    np.testing.assert_allclose(P["means"] - p["means"], -LRS["means"] * np.sign(g["means"]), rtol=1e-9)
    np.testing.assert_allclose(P["sh"] - p["sh"], -LRS["sh_dc"] * np.sign(g["sh"]), rtol=1e-9)
    np.testing.assert_allclose(M["quats"], 0.1 * g["quats"], rtol=1e-12)
    np.testing.assert_allclose(V["quats"], 0.001 * g["quats"] ** 2, rtol=1e-12)


def test_sparse_adam_leaves_unseen_rows_alone():
    rng = np.random.default_rng(2)
    p, zero, shapes = _state(rng)
    g = {k: rng.standard_normal(s) for k, s in shapes.items()}
    vis = rng.random(50) < 0.4
    P, M, V = U.adam(p, g, zero, zero, 1, LRS, 0.9, 0.999, 1e-15, visible=vis)
    for k in U.KEYS:
        np.testing.assert_array_equal(P[k][~vis], p[k][~vis])
        np.testing.assert_array_equal(M[k][~vis], 0.0)
        assert np.all(P[k][vis] != p[k][vis])


def test_se3_exponential_closed_forms():
    th = 0.7
    E = U.se3_exp([0, 0, 0, 0, 0, th])  # rotation about z
    np.testing.assert_allclose(E[:3, :3], [[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1]],
                               atol=1e-14)
    np.testing.assert_allclose(E[:3, 3], 0.0, atol=1e-15)
    E = U.se3_exp([0.3, -0.2, 0.5, 0, 0, 0])  # pure translation
    np.testing.assert_allclose(E, np.block([[np.eye(3), np.array([[0.3], [-0.2], [0.5]])], [np.zeros((1, 3)), 1]]),
                               atol=1e-15)
    # screw motion about z: translation along the axis is unchanged, the rest
    # follows the left Jacobian (1 - cos th) / th [z]x + ...
    rho = np.array([1.0, 0.0, 2.0])
    E = U.se3_exp(np.r_[rho, 0, 0, th])
    np.testing.assert_allclose(E[:3, 3], [np.sin(th) / th, (1 - np.cos(th)) / th, 2.0], atol=1e-14)


def test_pose_step_moves_by_the_adam_twist():
    rng = np.random.default_rng(3)
    T = np.stack([np.eye(4), U.se3_exp(rng.standard_normal(6) * 0.3)])
    g = rng.standard_normal((2, 6))
    out, m, v = U.pose_step(T, g, np.zeros((2, 6)), np.zeros((2, 6)), 1, 1e-3, 0.9, 0.999, 1e-15)
    for k in range(2):
        xi = -1e-3 * np.sign(g[k])
        np.testing.assert_allclose(out[k], U.se3_exp(xi) @ T[k], atol=1e-13)
        np.testing.assert_allclose(out[k][:3, :3] @ out[k][:3, :3].T, np.eye(3), atol=1e-12)


def _axis_angle(axis, ang):
    a = np.asarray(axis, float) / np.linalg.norm(axis)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + np.sin(ang) * K + (1 - np.cos(ang)) * K @ K


def test_sim3_relocation_matches_a_similarity_matrix():
    rng = np.random.default_rng(4)
    n = 30
    means = rng.standard_normal((n, 3))
    quats = rng.standard_normal((n, 4))
    quats /= np.linalg.norm(quats, axis=1, keepdims=True)
    ls = rng.normal(-3, 0.5, (n, 3))
    kf = rng.integers(-1, 3, n)
    sims = []
    for k in range(3):
        axis, ang = rng.standard_normal(3), rng.uniform(0, np.pi)
        q = np.r_[np.cos(ang / 2), np.sin(ang / 2) * axis / np.linalg.norm(axis)]
        sims.append(np.r_[rng.uniform(0.5, 2.0), q, rng.standard_normal(3)])
    sims = np.array(sims)
    mu, q2, ls2 = U.sim3_relocate(means, quats, ls, kf, sims)
    for i in range(n):
        k = kf[i]
        if k < 0:
            np.testing.assert_array_equal(mu[i], means[i])
            continue
        s, q, t = sims[k, 0], sims[k, 1:5], sims[k, 5:]
        axis = q[1:] / np.linalg.norm(q[1:])
        ang = 2 * np.arctan2(np.linalg.norm(q[1:]), q[0])
        Rk = _axis_angle(axis, ang)
        S = np.eye(4)
        S[:3, :3], S[:3, 3] = s * Rk, t
        np.testing.assert_allclose(mu[i], (S @ np.r_[means[i], 1])[:3], atol=1e-12)
        # the new rotation is R_k times the old one
        np.testing.assert_allclose(U.quat_rotation(q2[i]), Rk @ U.quat_rotation(quats[i]), atol=1e-12)
        np.testing.assert_allclose(ls2[i], ls[i] + np.log(s), atol=1e-14)
