"""FP64 reference of the parameter updates around the rasterizer.

Test infrastructure only: nothing in the product imports this module.  Plain
numpy (and scipy's matrix exponential), written from the definitions, with no
blocking or fusion:

* ``adam`` -- one Adam step of the joint optimisation (the paper trains the
  model for 30 iterations per keyframe, Sec. 5.2; its renderer's lineage
  optimises with Adam).  Opacities are stepped on their logit.
* ``pose_step`` -- Adam on each view's 6-DoF twist gradient (translation
  first), then the left retraction T <- exp(xi^) T (joint pose optimisation,
  Sec. 1 and Sec. 3).
* ``sim3_relocate`` -- each Gaussian follows the Sim(3) correction of the
  keyframe that spawned it, with scale and rotation updated accordingly
  (Sec. 6.3).
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import expm

KEYS = ("means", "log_scales", "quats", "opacities", "sh")
OPACITY_LO, OPACITY_HI = 1e-7, 1.0 - 1e-7


def _adam_moments(g, m, v, b1, b2):
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    return m, v


def _adam_delta(m, v, step, lr, b1, b2, eps):
    m_hat = m / (1.0 - b1 ** step)
    v_hat = v / (1.0 - b2 ** step)
    return -lr * m_hat / (np.sqrt(v_hat) + eps)


def adam(params: dict, grads: dict, exp_avg: dict, exp_avg_sq: dict, step: int, lrs: dict, beta1: float,
         beta2: float, eps: float, visible=None):
    """Returns updated copies (params, exp_avg, exp_avg_sq) as float64.

    lrs: means, log_scales, quats, opacities, sh_dc, sh_rest.  visible: bool
    [n] or None; rows that are not visible keep parameters and moments."""
    P = {k: np.array(params[k], np.float64) for k in KEYS}
    M = {k: np.array(exp_avg[k], np.float64) for k in KEYS}
    V = {k: np.array(exp_avg_sq[k], np.float64) for k in KEYS}
    G = {k: np.asarray(grads[k], np.float64) for k in KEYS}
    n = P["means"].shape[0]
    rows = np.ones(n, bool) if visible is None else np.asarray(visible, bool)
    for k in ("means", "log_scales", "quats", "sh"):
        m, v = _adam_moments(G[k][rows], M[k][rows], V[k][rows], beta1, beta2)
        if k == "sh":
            lr = np.full(P["sh"].shape[1:], lrs["sh_rest"])
            lr[0, :] = lrs["sh_dc"]
        else:
            lr = lrs[k]
        P[k][rows] = P[k][rows] + _adam_delta(m, v, step, lr, beta1, beta2, eps)
        M[k][rows], V[k][rows] = m, v
    # opacity: step on the logit l = ln(o / (1 - o)); dL/dl = o (1 - o) dL/do
    o = np.clip(P["opacities"][rows], OPACITY_LO, OPACITY_HI)
    logit = np.log(o) - np.log1p(-o)
    m, v = _adam_moments(o * (1.0 - o) * G["opacities"][rows], M["opacities"][rows], V["opacities"][rows],
                         beta1, beta2)
    logit = logit + _adam_delta(m, v, step, lrs["opacities"], beta1, beta2, eps)
    P["opacities"][rows] = 1.0 / (1.0 + np.exp(-logit))
    M["opacities"][rows], V["opacities"][rows] = m, v
    return P, M, V


def hat(xi):
    """4x4 matrix of a twist (rho, phi): [[phi^, rho], [0, 0]]."""
    rho, phi = np.asarray(xi[:3], np.float64), np.asarray(xi[3:], np.float64)
    X = np.zeros((4, 4))
    X[:3, :3] = [[0.0, -phi[2], phi[1]], [phi[2], 0.0, -phi[0]], [-phi[1], phi[0], 0.0]]
    X[:3, 3] = rho
    return X


def se3_exp(xi):
    return expm(hat(xi))


def pose_step(world_to_cam, dL_dtwist, exp_avg, exp_avg_sq, step: int, lr: float, beta1: float, beta2: float,
              eps: float):
    """Returns (world_to_cam [V, 4, 4], exp_avg, exp_avg_sq) as float64."""
    T = np.array(world_to_cam, np.float64).reshape(-1, 4, 4)
    m, v = _adam_moments(np.asarray(dL_dtwist, np.float64), np.asarray(exp_avg, np.float64),
                         np.asarray(exp_avg_sq, np.float64), beta1, beta2)
    xi = _adam_delta(m, v, step, lr, beta1, beta2, eps)
    out = np.stack([se3_exp(xi[k]) @ T[k] for k in range(T.shape[0])])
    return out, m, v


def quat_rotation(q):
    """Rotation matrix of the unit quaternion (w, x, y, z)."""
    w, x, y, z = (float(c) for c in q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def quat_mul(a, b):
    """Hamilton product a * b of (w, x, y, z) quaternions (rows of b, one a)."""
    aw, ax, ay, az = (float(c) for c in a)
    b = np.asarray(b, np.float64)
    bw, bx, by, bz = b[..., 0], b[..., 1], b[..., 2], b[..., 3]
    return np.stack([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw], -1)


def sim3_relocate(means, quats, log_scales, keyframe_of, sim3):
    """sim3 [K, 8] = (s, qw, qx, qy, qz, tx, ty, tz).  Returns float64 copies."""
    mu = np.array(means, np.float64)
    q = np.array(quats, np.float64)
    ls = np.array(log_scales, np.float64)
    kf = np.asarray(keyframe_of)
    S = np.asarray(sim3, np.float64)
    for k in range(S.shape[0]):
        idx = kf == k
        if not idx.any():
            continue
        s, qk, t = S[k, 0], S[k, 1:5], S[k, 5:8]
        mu[idx] = s * mu[idx] @ quat_rotation(qk).T + t
        q[idx] = quat_mul(qk, q[idx])
        ls[idx] = ls[idx] + np.log(s)
    return mu, q, ls
