"""Pins of the FP64 bundle-adjustment oracle (oracle/ba.py) against things it
does not share code with: closed-form projections, the rotation about one axis,
central finite differences of the residual, the full (un-eliminated) normal
equations, the large-damping limit and noise-free recovery of the generator's
ground truth (observations the generator made through the intrinsic matrix)."""
import numpy as np
import pytest

from oracle import ba as B
from paper_2607_14481_amd.ba_scenes import make_problem


def _problem(P):
    lm, cam, uv = P.flat_observations()
    return {"free_slot": P.free_slot, "c": np.array(P.principal), "obs_lm": lm, "obs_cam": cam, "obs_uv": uv}


def _state(P, which="init"):
    return {"poses": getattr(P, f"{which}_poses"), "f": getattr(P, f"{which}_focal"),
            "landmarks": getattr(P, f"{which}_landmarks")}


def _small(seed=0, **kw):
    args = dict(n_cams=6, n_landmarks=25, n_fixed=2, max_obs=4, pixel_noise=0.3)
    args.update(kw)
    return make_problem(seed, **args)


def test_projection_closed_forms():
    I = np.concatenate([np.eye(3), np.zeros((3, 1))], 1)[None]
    c = np.array([320.0, 240.0])
    pts = np.array([[0.0, 0.0, 2.0], [1.0, 0.0, 1.0], [0.0, -0.5, 2.0]])
    lm, cam = np.arange(3), np.zeros(3, np.int64)
    r = B.residuals_jacobians(I, 500.0, c, pts, lm, cam, np.zeros((3, 2)))[0]
    np.testing.assert_allclose(r, [[320.0, 240.0], [820.0, 240.0], [320.0, 115.0]], rtol=0, atol=1e-12)
    # a translated camera: the point one unit in front of it, one unit back
    T = np.concatenate([np.eye(3), np.array([[0.0], [0.0], [1.0]])], 1)[None]
    r = B.residuals_jacobians(T, 400.0, c, np.array([[0.5, 0.0, 1.0]]), np.zeros(1, np.int64), np.zeros(1, np.int64),
                              np.zeros((1, 2)))[0]
    np.testing.assert_allclose(r, [[420.0, 240.0]], atol=1e-12)


def test_se3_exp_closed_forms():
    th = 0.7
    E = B.se3_exp(np.array([0.0, 0.0, 0.0, 0.0, 0.0, th]))
    Rz = np.array([[np.cos(th), -np.sin(th), 0.0], [np.sin(th), np.cos(th), 0.0], [0.0, 0.0, 1.0]])
    np.testing.assert_allclose(E[:3, :3], Rz, atol=1e-14)
    np.testing.assert_allclose(E[:3, 3], 0.0, atol=1e-14)
    E = B.se3_exp(np.array([0.1, -0.2, 0.3, 0.0, 0.0, 0.0]))
    np.testing.assert_allclose(E[:3, :3], np.eye(3), atol=1e-15)
    np.testing.assert_allclose(E[:3, 3], [0.1, -0.2, 0.3], atol=1e-15)
    # a screw along the rotation axis: translation along the axis is unchanged
    E = B.se3_exp(np.array([0.0, 0.0, 0.5, 0.0, 0.0, th]))
    np.testing.assert_allclose(E[:3, 3], [0.0, 0.0, 0.5], atol=1e-14)


def test_jacobians_match_central_differences():
    P = _small(1)
    pr, st = _problem(P), _state(P)
    r, Jx, Jf, Jp = B.residuals_jacobians(st["poses"], st["f"], pr["c"], st["landmarks"], pr["obs_lm"], pr["obs_cam"],
                                          pr["obs_uv"])

    def res(poses, f, pts):
        return B.residuals_jacobians(poses, f, pr["c"], pts, pr["obs_lm"], pr["obs_cam"], pr["obs_uv"])[0]

    h = 1e-6
    for k in range(6):
        e = np.zeros(6)
        e[k] = h
        plus, minus = st["poses"].copy(), st["poses"].copy()
        for i in range(P.n_cams):
            T = np.vstack([st["poses"][i], [0, 0, 0, 1]])
            plus[i] = (B.se3_exp(e) @ T)[:3]
            minus[i] = (B.se3_exp(-e) @ T)[:3]
        fd = (res(plus, st["f"], st["landmarks"]) - res(minus, st["f"], st["landmarks"])) / (2 * h)
        np.testing.assert_allclose(Jx[:, :, k], fd, rtol=1e-6, atol=1e-4)
    fd = (res(st["poses"], st["f"] + h, st["landmarks"]) - res(st["poses"], st["f"] - h, st["landmarks"])) / (2 * h)
    np.testing.assert_allclose(Jf, fd, rtol=1e-7, atol=1e-7)
    for a in range(3):
        plus, minus = st["landmarks"].copy(), st["landmarks"].copy()
        plus[:, a] += h
        minus[:, a] -= h
        fd = (res(st["poses"], st["f"], plus) - res(st["poses"], st["f"], minus)) / (2 * h)
        np.testing.assert_allclose(Jp[:, :, a], fd, rtol=1e-6, atol=1e-4)


def _finite_difference_system(pr, st, n_unknowns, h=1e-6):
    """J of the stacked residual over every unknown by central differences of
    apply_step (so the column order and the fixed keyframes come from the
    update, not from the Jacobian code), and r."""
    r0 = B.residuals_jacobians(st["poses"], st["f"], pr["c"], st["landmarks"], pr["obs_lm"], pr["obs_cam"],
                               pr["obs_uv"])[0].reshape(-1)
    J = np.zeros((len(r0), n_unknowns))
    for k in range(n_unknowns):
        e = np.zeros(n_unknowns)
        e[k] = h
        rp = B.residuals_jacobians(**_args(pr, B.apply_step(pr, st, e)))[0].reshape(-1)
        rm = B.residuals_jacobians(**_args(pr, B.apply_step(pr, st, -e)))[0].reshape(-1)
        J[:, k] = (rp - rm) / (2 * h)
    return J, r0


def _args(pr, st):
    return dict(poses=st["poses"], f=st["f"], c=pr["c"], landmarks=st["landmarks"], obs_lm=pr["obs_lm"],
                obs_cam=pr["obs_cam"], obs_uv=pr["obs_uv"])


def test_normal_equations_are_those_of_the_finite_difference_jacobian():
    P = _small(2)
    pr, st = _problem(P), _state(P)
    H, g = B.normal_equations(pr, st)
    J, r = _finite_difference_system(pr, st, len(g))
    scale = np.abs(H).max()
    np.testing.assert_allclose(H, J.T @ J, rtol=0, atol=1e-6 * scale)
    np.testing.assert_allclose(g, J.T @ r, rtol=0, atol=1e-6 * np.abs(g).max())


@pytest.mark.parametrize("n_fixed", [0, 2, 6])
def test_schur_step_equals_the_full_solve(n_fixed):
    P = _small(3, n_fixed=n_fixed)
    pr, st = _problem(P), _state(P)
    for lam in (1e-4, 0.5):
        d_dense = B.step_dense(pr, st, lam)
        d_schur = B.step_schur(pr, st, lam)
        np.testing.assert_allclose(d_schur, d_dense, rtol=1e-8, atol=1e-10 * np.abs(d_dense).max())


def test_large_damping_limit_is_a_scaled_gradient_step():
    # (H + lam diag H) d = -g  =>  lam d -> -g / diag H as lam -> infinity
    P = _small(4)
    pr, st = _problem(P), _state(P)
    H, g = B.normal_equations(pr, st)
    lam = 1e9
    d = B.step_schur(pr, st, lam)
    np.testing.assert_allclose(lam * d, -g / np.diag(H), rtol=1e-6, atol=1e-12)


def test_noise_free_problem_recovers_the_ground_truth():
    P = make_problem(5, n_cams=8, n_landmarks=200, n_fixed=3, max_obs=5)
    pr = _problem(P)
    assert B.cost(pr, _state(P, "gt")) < 1e-18 * len(pr["obs_lm"])
    st, costs = B.solve(pr, _state(P), iters=10, lam=1e-4)
    assert costs[0] > 1.0
    assert costs[-1] < 1e-16 * costs[0] + 1e-20
    np.testing.assert_allclose(st["poses"], P.gt_poses, atol=1e-8)
    np.testing.assert_allclose(st["landmarks"], P.gt_landmarks, atol=1e-8)
    assert abs(st["f"] - P.gt_focal) < 1e-6
    fixed = P.free_slot < 0
    assert np.array_equal(st["poses"][fixed], P.init_poses[fixed])


def test_every_step_lowers_the_cost_on_a_noisy_problem():
    P = make_problem(6, n_cams=8, n_landmarks=150, n_fixed=2, max_obs=6, pixel_noise=0.5)
    st, costs = B.solve(_problem(P), _state(P), iters=6, lam=1e-4)
    assert all(b < a for a, b in zip(costs, costs[1:]))
    # at the optimum the residual is at the noise level: 1/2 sum r^2 ~ 1/2 * 0.25 per coordinate
    n = 2 * int((P.obs_cam >= 0).sum())
    assert costs[-1] < 0.5 * 0.25 * n


def test_generator_builds_the_stated_structure():
    P = make_problem(0)
    assert P.n_cams == 20 and P.n_landmarks == 10_000 and P.max_obs == 8
    assert int((P.free_slot < 0).sum()) == 4
    assert sorted(P.free_slot[P.free_slot >= 0].tolist()) == list(range(16))
    counts = (P.obs_cam >= 0).sum(axis=1)
    assert counts.min() == 2 and counts.max() == 8
    for j in range(0, P.n_landmarks, 97):   # runs of consecutive keyframes, valid slots first
        row = P.obs_cam[j]
        m = int(counts[j])
        assert (row[m:] == -1).all() and (np.diff(row[:m]) == 1).all()
    # every landmark in front of every camera that sees it, at depth above 1.4
    lm, cam, _ = P.flat_observations()
    X = np.einsum("oab,ob->oa", P.gt_poses[cam, :, :3], P.gt_landmarks[lm]) + P.gt_poses[cam, :, 3]
    assert X[:, 2].min() > 1.4
