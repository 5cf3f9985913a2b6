"""FP64 reference of the local bundle adjustment.

TEST INFRASTRUCTURE ONLY: nothing in the product imports this module.  Plain
numpy (scipy's matrix exponential for the pose retraction), written from the
definitions with no blocking or fusion.

The problem is the paper's local BA (Sec. 5.1, "Local Bundle Adjustment", and
the appendix paragraph "Fast Bundle Adjustment"): N keyframes of which n_f are
held fixed, K landmarks each observed by a fixed subset of the keyframes, GPU
residual and Jacobian kernels and a dense Schur complement; its runtime is
reported for 10 iterations of a synthesized problem with 20 poses and 10,000
landmarks, with the intrinsics optimised too (the BA runtime table).  Our
readings, where the paper is silent:

* pinhole camera, one focal length f shared by all keyframes (the optimised
  intrinsic), principal point c fixed: pi(X) = f (X / Z, Y / Z) + c;
* poses T_i world -> camera (3 x 4), perturbed on the left, T <- exp(xi^) T,
  xi = (rho, phi), translation first;
* cost 1/2 sum over observations of |pi(f, T_i p_j) - z_ij|^2;
* Levenberg-Marquardt steps with a fixed damping lambda on the diagonal,
  (H + lambda diag(H)) delta = -g with H = J^T J and g = J^T r, every step
  taken (no acceptance test: the runtime is for a fixed iteration count);
* the camera-side unknowns are the free poses in slot order (6 each), then f.

Functions:

* ``residuals_jacobians`` -- r, and the Jacobians w.r.t. the pose twist, f and
  the landmark, per observation;
* ``normal_equations`` -- the full H and g over (camera side, landmarks), for
  small problems (a pin of the Schur form);
* ``step_dense`` / ``step_schur`` -- one damped step, by solving the full
  system, and by eliminating the landmarks first (the paper's formulation);
* ``apply_step``, ``solve``, ``cost``.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import expm


def skew(v):
    return np.array([[0.0, -v[2], v[1]], [v[2], 0.0, -v[0]], [-v[1], v[0], 0.0]])


def residuals_jacobians(poses, f, c, landmarks, obs_lm, obs_cam, obs_uv):
    """Per observation o of landmark obs_lm[o] in keyframe obs_cam[o]:
    r (O, 2), J_pose (O, 2, 6) w.r.t. the left twist of the keyframe's pose,
    J_f (O, 2) w.r.t. f and J_p (O, 2, 3) w.r.t. the landmark."""
    poses = np.asarray(poses, np.float64)
    P = np.asarray(landmarks, np.float64)[obs_lm]
    R = poses[obs_cam, :, :3]
    t = poses[obs_cam, :, 3]
    X = np.einsum("oab,ob->oa", R, P) + t                 # camera-frame point
    x, y, z = X[:, 0], X[:, 1], X[:, 2]
    r = np.stack([f * x / z + c[0], f * y / z + c[1]], 1) - np.asarray(obs_uv, np.float64)
    dpi = np.zeros((len(X), 2, 3))                        # d pi / d X
    dpi[:, 0, 0] = f / z
    dpi[:, 0, 2] = -f * x / (z * z)
    dpi[:, 1, 1] = f / z
    dpi[:, 1, 2] = -f * y / (z * z)
    # exp(xi^) X ~ X + rho + phi x X: dX/drho = I, dX/dphi = -[X]x
    J_pose = np.zeros((len(X), 2, 6))
    for o in range(len(X)):
        J_pose[o, :, :3] = dpi[o]
        J_pose[o, :, 3:] = -dpi[o] @ skew(X[o])
    J_f = np.stack([x / z, y / z], 1)
    J_p = np.einsum("oab,obc->oac", dpi, R)
    return r, J_pose, J_f, J_p


def n_free_of(free_slot):
    """Number of free keyframes (slots are 0 .. n_free - 1, -1 = fixed)."""
    return int(np.max(free_slot)) + 1 if len(free_slot) and np.max(free_slot) >= 0 else 0


def camera_columns(cam, free_slot, n_free):
    """Columns of the camera-side unknowns an observation in keyframe `cam`
    touches: its pose twist (if free) and f (the last column)."""
    s = int(free_slot[cam])
    pose_cols = list(range(6 * s, 6 * s + 6)) if s >= 0 else []
    return pose_cols, 6 * n_free


def normal_equations(problem, state):
    """Full H = J^T J and g = J^T r over (camera side, then the landmarks,
    3 per landmark), without damping."""
    free_slot = problem["free_slot"]
    n_free = n_free_of(free_slot)
    K = len(state["landmarks"])
    Dc = 6 * n_free + 1
    D = Dc + 3 * K
    obs_lm, obs_cam = problem["obs_lm"], problem["obs_cam"]
    r, Jx, Jf, Jp = residuals_jacobians(state["poses"], state["f"], problem["c"], state["landmarks"], obs_lm,
                                        obs_cam, problem["obs_uv"])
    H = np.zeros((D, D))
    g = np.zeros(D)
    for o in range(len(r)):
        J = np.zeros((2, D))
        pose_cols, fcol = camera_columns(obs_cam[o], free_slot, n_free)
        if pose_cols:
            J[:, pose_cols] = Jx[o]
        J[:, fcol] = Jf[o]
        j = int(obs_lm[o])
        J[:, Dc + 3 * j:Dc + 3 * j + 3] = Jp[o]
        H += J.T @ J
        g += J.T @ r[o]
    return H, g


def _damp(H, lam):
    H = H.copy()
    H[np.diag_indices_from(H)] *= 1.0 + lam
    return H


def step_dense(problem, state, lam):
    """delta = -(H + lam diag(H))^-1 g over all unknowns."""
    H, g = normal_equations(problem, state)
    return -np.linalg.solve(_damp(H, lam), g)


def step_schur(problem, state, lam):
    """The same step with the landmarks eliminated first:
    S = Hcc - sum_j Hcp_j Hpp_j^-1 Hcp_j^T, s = gc - sum_j Hcp_j Hpp_j^-1 gp_j,
    delta_c = -S^-1 s, delta_p_j = -Hpp_j^-1 (gp_j + Hcp_j^T delta_c)
    (damping applied to the diagonals of Hcc and of every Hpp_j first).
    Returns the full step vector (camera side, then 3 per landmark)."""
    free_slot = problem["free_slot"]
    n_free = n_free_of(free_slot)
    K = len(state["landmarks"])
    Dc = 6 * n_free + 1
    obs_lm, obs_cam = problem["obs_lm"], problem["obs_cam"]
    r, Jx, Jf, Jp = residuals_jacobians(state["poses"], state["f"], problem["c"], state["landmarks"], obs_lm,
                                        obs_cam, problem["obs_uv"])
    Hcc = np.zeros((Dc, Dc))
    gc = np.zeros(Dc)
    Hpp = np.zeros((K, 3, 3))
    gp = np.zeros((K, 3))
    Hcp = np.zeros((K, Dc, 3))
    for o in range(len(r)):
        Jc = np.zeros((2, Dc))
        pose_cols, fcol = camera_columns(obs_cam[o], free_slot, n_free)
        if pose_cols:
            Jc[:, pose_cols] = Jx[o]
        Jc[:, fcol] = Jf[o]
        j = int(obs_lm[o])
        Hcc += Jc.T @ Jc
        gc += Jc.T @ r[o]
        Hpp[j] += Jp[o].T @ Jp[o]
        gp[j] += Jp[o].T @ r[o]
        Hcp[j] += Jc.T @ Jp[o]
    Hcc = _damp(Hcc, lam)
    S = Hcc.copy()
    s = gc.copy()
    Hpp_inv = np.zeros_like(Hpp)
    for j in range(K):
        Hpp_inv[j] = np.linalg.inv(_damp(Hpp[j], lam))
        S -= Hcp[j] @ Hpp_inv[j] @ Hcp[j].T
        s -= Hcp[j] @ Hpp_inv[j] @ gp[j]
    dc = -np.linalg.solve(S, s)
    dp = np.zeros((K, 3))
    for j in range(K):
        dp[j] = -Hpp_inv[j] @ (gp[j] + Hcp[j].T @ dc)
    return np.concatenate([dc, dp.reshape(-1)])


def se3_exp(xi):
    """exp of the twist (rho, phi) as a 4 x 4 matrix (the matrix exponential)."""
    A = np.zeros((4, 4))
    A[:3, :3] = skew(xi[3:])
    A[:3, 3] = xi[:3]
    return expm(A)


def apply_step(problem, state, delta):
    """T_i <- exp(xi_i^) T_i for the free poses, f += df, p_j += dp_j."""
    free_slot = problem["free_slot"]
    n_free = n_free_of(free_slot)
    Dc = 6 * n_free + 1
    poses = np.array(state["poses"], np.float64, copy=True)
    for i, s in enumerate(free_slot):
        if s >= 0:
            T = np.eye(4)
            T[:3, :] = poses[i]
            poses[i] = (se3_exp(delta[6 * s:6 * s + 6]) @ T)[:3, :]
    return {"poses": poses, "f": float(state["f"]) + float(delta[Dc - 1]),
            "landmarks": np.asarray(state["landmarks"], np.float64) + delta[Dc:].reshape(-1, 3)}


def cost(problem, state):
    r = residuals_jacobians(state["poses"], state["f"], problem["c"], state["landmarks"], problem["obs_lm"],
                            problem["obs_cam"], problem["obs_uv"])[0]
    return 0.5 * float(np.sum(r * r))


def solve(problem, state, iters, lam):
    """`iters` Schur steps; returns the final state and the cost before each
    step and after the last."""
    costs = [cost(problem, state)]
    for _ in range(iters):
        state = apply_step(problem, state, step_schur(problem, state, lam))
        costs.append(cost(problem, state))
    return state, costs


def project(problem, state):
    """pi(f, T_i p_j) of every observation (the residual against zero)."""
    return residuals_jacobians(state["poses"], state["f"], problem["c"], state["landmarks"], problem["obs_lm"],
                               problem["obs_cam"], np.zeros((len(problem["obs_lm"]), 2)))[0]
