"""Seeded synthetic local bundle-adjustment problems.

This module builds inputs only: camera poses, landmarks, which keyframes see
which landmark, observations and a perturbed starting point.  It holds none of
the solver's arithmetic (no residual, Jacobian, normal equations, Schur
complement or pose retraction); the FP64 oracle and the GPU solver both consume
what it returns.

The paper times its local BA on a synthesized problem with 20 keyframes and
10,000 landmarks, 4 of the keyframes held fixed, each landmark seen by a fixed
covisibility-chosen subset of the keyframes, and the focal length optimised
(Sec. 5.1 and the BA runtime table).  The recipe here:

* keyframes on a 120-degree arc of radius 4 around the origin, with small
  height jitter, each looking at the origin (x right, y down, z forward);
* landmarks uniform in the cube [-1.5, 1.5]^3, so every depth is above 1.4;
* landmark j is seen by m_j keyframes, m_j uniform in [min_obs, max_obs], which
  form a run of consecutive keyframes along the arc (neighbouring keyframes are
  the covisible ones) starting at a uniform position;
* ``n_fixed`` keyframes drawn without replacement are held fixed;
* observations are the ground-truth landmarks imaged through the intrinsic
  matrix [[f, 0, cx], [0, f, cy], [0, 0, 1]] (homogeneous coordinates), plus
  Gaussian pixel noise of standard deviation ``pixel_noise``;
* the starting point perturbs every free pose by a rotation about a random
  axis (angle ~ N(0, rot_noise)) and a translation ~ N(0, trans_noise), every
  landmark by N(0, point_noise) per axis, and the focal length by a factor
  1 + N(0, focal_noise).

Layouts (shared with the library's C ABI): poses are world-to-camera 3x4
row-major float64; ``obs_cam`` is int32 [K, max_obs] with the valid entries
first and -1 after them; ``obs_uv`` is float64 [K, max_obs, 2] (zero where
unused); ``free_slot`` is int32 [N], the index of a free keyframe among the
free ones in keyframe order, -1 for a fixed one.

Draw order from ``Generator(PCG64(seed))``: heights, landmarks, counts, run
starts, fixed keyframes, pixel noise, pose rotations, pose translations,
landmark perturbations, focal perturbation.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class BAProblem:
    width: int
    height: int
    principal: tuple           # (cx, cy)
    free_slot: np.ndarray      # int32 [N]
    obs_cam: np.ndarray        # int32 [K, M]
    obs_uv: np.ndarray         # float64 [K, M, 2]
    gt_poses: np.ndarray       # float64 [N, 3, 4]
    gt_focal: float
    gt_landmarks: np.ndarray   # float64 [K, 3]
    init_poses: np.ndarray
    init_focal: float
    init_landmarks: np.ndarray

    @property
    def n_cams(self):
        return len(self.free_slot)

    @property
    def n_landmarks(self):
        return len(self.obs_cam)

    @property
    def max_obs(self):
        return self.obs_cam.shape[1]

    def flat_observations(self):
        """(obs_lm, obs_cam, obs_uv) of the valid observations, landmark-major."""
        lm, k = np.nonzero(self.obs_cam >= 0)
        return lm.astype(np.int64), self.obs_cam[lm, k].astype(np.int64), self.obs_uv[lm, k]


def _look_at(centre, target):
    """World-to-camera 3x4 whose camera sits at `centre` looking at `target`,
    x to the right and y down in the image."""
    z = target - centre
    z = z / np.linalg.norm(z)
    up = np.array([0.0, -1.0, 0.0])
    x = np.cross(up, z)
    x = x / np.linalg.norm(x)
    y = np.cross(z, x)
    R = np.stack([x, y, z])
    return np.concatenate([R, (-R @ centre)[:, None]], 1)


def _axis_angle_matrix(axis, angle):
    """Rotation about a unit axis (Rodrigues' formula)."""
    k = np.array([[0.0, -axis[2], axis[1]], [axis[2], 0.0, -axis[0]], [-axis[1], axis[0], 0.0]])
    return np.eye(3) + np.sin(angle) * k + (1.0 - np.cos(angle)) * (k @ k)


def make_problem(seed=0, n_cams=20, n_landmarks=10_000, n_fixed=4, max_obs=8, min_obs=2, width=640, height=480,
                 focal=500.0, pixel_noise=0.0, rot_noise=0.01, trans_noise=0.02, point_noise=0.02,
                 focal_noise=0.01) -> BAProblem:
    if not (2 <= min_obs <= max_obs <= n_cams):
        raise ValueError("need 2 <= min_obs <= max_obs <= n_cams")
    if not (0 <= n_fixed <= n_cams):
        raise ValueError("need 0 <= n_fixed <= n_cams")
    rng = np.random.Generator(np.random.PCG64(seed))
    N, K, M = n_cams, n_landmarks, max_obs
    heights = rng.normal(0.0, 0.3, N)
    angles = np.deg2rad(-60.0 + 120.0 * np.arange(N) / max(N - 1, 1))
    poses = np.stack([_look_at(np.array([4.0 * np.sin(a), h, -4.0 * np.cos(a)]), np.zeros(3))
                      for a, h in zip(angles, heights)])
    pts = rng.uniform(-1.5, 1.5, (K, 3))
    counts = rng.integers(min_obs, max_obs + 1, K)
    starts = rng.integers(0, N - counts + 1)
    obs_cam = np.full((K, M), -1, np.int32)
    for j in range(K):
        obs_cam[j, :counts[j]] = np.arange(starts[j], starts[j] + counts[j])
    fixed = rng.choice(N, n_fixed, replace=False)
    free_slot = np.full(N, -1, np.int32)
    free = np.setdiff1d(np.arange(N), fixed)
    free_slot[free] = np.arange(len(free))
    cx, cy = width / 2.0, height / 2.0
    Kmat = np.array([[focal, 0.0, cx], [0.0, focal, cy], [0.0, 0.0, 1.0]])
    obs_uv = np.zeros((K, M, 2))
    noise = rng.normal(0.0, 1.0, (K, M, 2)) * pixel_noise
    for j in range(K):
        for k in range(counts[j]):
            h = Kmat @ (poses[obs_cam[j, k]] @ np.append(pts[j], 1.0))
            obs_uv[j, k] = h[:2] / h[2] + noise[j, k]
    # starting point
    axes = rng.normal(0.0, 1.0, (N, 3))
    axes /= np.linalg.norm(axes, axis=1, keepdims=True)
    ang = rng.normal(0.0, rot_noise, N)
    dt = rng.normal(0.0, trans_noise, (N, 3))
    init_poses = poses.copy()
    for i in free:
        Rn = _axis_angle_matrix(axes[i], ang[i])
        init_poses[i, :, :3] = Rn @ poses[i, :, :3]
        init_poses[i, :, 3] = Rn @ poses[i, :, 3] + dt[i]
    init_pts = pts + rng.normal(0.0, point_noise, (K, 3))
    init_focal = focal * (1.0 + rng.normal(0.0, focal_noise))
    return BAProblem(width, height, (cx, cy), free_slot, obs_cam, obs_uv, poses, float(focal), pts, init_poses,
                     float(init_focal), init_pts)
