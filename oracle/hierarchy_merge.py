"""FP64 reference of the merge that builds a Gaussian hierarchy's inner nodes.

TEST INFRASTRUCTURE ONLY: nothing in the product imports this module; it
imports nothing from the product.  Plain numpy, one group at a time.

The paper keeps large scenes tractable with a hierarchy whose inner nodes
replace groups of Gaussians by one merged Gaussian, chosen by a KL-divergence
criterion (Sec. 7.1, "Adaptive Gaussian Merging and Retrieval"; a node holds
position, opacity, rotation, scale and SH coefficients, Sec. 7).  Reading
(the paper gives no formula): the merged Gaussian is the single Gaussian q
that minimises KL(p || q) for the mixture p = sum_i w_i N(mu_i, Sigma_i) of
the children, whose weights are their opacities normalised to sum to one.
That minimiser matches the mixture's first two moments:

    w_i   = o_i / sum_j o_j
    mu    = sum_i w_i mu_i
    Sigma = sum_i w_i (Sigma_i + (mu_i - mu)(mu_i - mu)^T)

with Sigma_i = R(q_i) diag(exp(2 s_i)) R(q_i)^T (q_i normalised first).  The
merged opacity composites the children's coverage, 1 - prod_i (1 - o_i), and
the merged SH coefficients are the w-weighted mean of the children's.  The
covariance is stored like any node's: log-scales and a rotation, from its
eigendecomposition (eigenvalues ascending, eigenvectors as the rotation's
columns with determinant +1; variances below 1e-12 are raised to 1e-12).
"""
from __future__ import annotations

import numpy as np

MIN_VAR = 1e-12


def rotation(q) -> np.ndarray:
    """Rotation matrix of the quaternion (w, x, y, z), normalised first."""
    w, x, y, z = np.asarray(q, np.float64) / np.linalg.norm(np.asarray(q, np.float64))
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def covariance(log_scales, quat) -> np.ndarray:
    """Sigma = R diag(exp(2 s)) R^T of one Gaussian."""
    R = rotation(quat)
    return R @ np.diag(np.exp(2.0 * np.asarray(log_scales, np.float64))) @ R.T


def merge_moments(means, covs, opacities, shs):
    """The merged Gaussian of one group, before factorisation.

    means [k, 3], covs [k, 3, 3], opacities [k], shs [k, K, 3] -> (mu [3],
    Sigma [3, 3], opacity, sh [K, 3])."""
    means = np.asarray(means, np.float64)
    covs = np.asarray(covs, np.float64)
    o = np.asarray(opacities, np.float64)
    shs = np.asarray(shs, np.float64)
    w = o / o.sum()
    mu = np.zeros(3)
    for i in range(len(o)):
        mu += w[i] * means[i]
    sigma = np.zeros((3, 3))
    for i in range(len(o)):
        d = means[i] - mu
        sigma += w[i] * (covs[i] + np.outer(d, d))
    opacity = 1.0 - np.prod(1.0 - o)
    sh = np.zeros(shs.shape[1:])
    for i in range(len(o)):
        sh += w[i] * shs[i]
    return mu, sigma, opacity, sh


def factor(sigma):
    """(log-scales ascending [3], rotation [3, 3] with det +1) of a covariance."""
    vals, vecs = np.linalg.eigh(np.asarray(sigma, np.float64))
    if np.linalg.det(vecs) < 0:
        vecs[:, 2] = -vecs[:, 2]
    return 0.5 * np.log(np.maximum(vals, MIN_VAR)), vecs


def merge_group(means, log_scales, quats, opacities, shs):
    """One parent from its children's stored parameters.  Returns a dict with
    mean, cov (the moment-matched covariance), log_scales, rot (its factors),
    opacity and sh."""
    covs = [covariance(s, q) for s, q in zip(log_scales, quats)]
    mu, sigma, o, sh = merge_moments(means, covs, opacities, shs)
    ls, rot = factor(sigma)
    return {"mean": mu, "cov": sigma, "log_scales": ls, "rot": rot, "opacity": o, "sh": sh}


def cross_entropy(means, covs, opacities, mu_q, sigma_q) -> float:
    """-E_p[log q] for the opacity-weighted mixture p of the children and the
    Gaussian q = N(mu_q, sigma_q), in closed form: KL(p || q) is this minus
    the entropy of p, which does not depend on q."""
    o = np.asarray(opacities, np.float64)
    w = o / o.sum()
    inv = np.linalg.inv(sigma_q)
    _, logdet = np.linalg.slogdet(2.0 * np.pi * np.asarray(sigma_q, np.float64))
    ce = 0.5 * logdet
    for i in range(len(w)):
        d = np.asarray(means[i], np.float64) - mu_q
        ce += w[i] * 0.5 * (np.trace(inv @ covs[i]) + d @ inv @ d)
    return float(ce)


def build_levels(means, log_scales, quats, opacities, shs, levels, branching=8):
    """A whole hierarchy from leaves already in their final order: level l+1
    merges runs of `branching` consecutive level-l nodes (the last run may be
    shorter), `levels` times or until one node is left.  Returns the nodes of
    every level as lists (level 0 first) of dicts with mean, log_scales, quat
    (w >= 0), opacity, sh and cov.  For small inputs only (one group at a
    time)."""
    cur = [{"mean": np.asarray(m, np.float64), "log_scales": np.asarray(s, np.float64),
            "quat": np.asarray(q, np.float64), "opacity": float(o), "sh": np.asarray(h, np.float64)}
           for m, s, q, o, h in zip(means, log_scales, quats, opacities, shs)]
    out = [cur]
    for _ in range(levels):
        if len(cur) <= 1:
            break
        nxt = []
        for g in range(0, len(cur), branching):
            kids = cur[g:g + branching]
            r = merge_group([k["mean"] for k in kids], [k["log_scales"] for k in kids],
                            [k["quat"] for k in kids], [k["opacity"] for k in kids], [k["sh"] for k in kids])
            nxt.append({"mean": r["mean"], "log_scales": r["log_scales"], "quat": quat_of(r["rot"]),
                        "opacity": r["opacity"], "sh": r["sh"], "cov": r["cov"]})
        out.append(nxt)
        cur = nxt
    return out


def quat_of(R) -> np.ndarray:
    """Unit quaternion (w, x, y, z), w >= 0, of a proper rotation matrix, from
    its axis and angle (scipy-free; checked against scipy in the pins)."""
    R = np.asarray(R, np.float64)
    c = np.clip((np.trace(R) - 1.0) / 2.0, -1.0, 1.0)
    angle = np.arccos(c)
    if angle < 1e-8:
        return np.array([1.0, 0.0, 0.0, 0.0])
    if np.pi - angle < 1e-6:  # near a half turn: the axis from R + I
        M = (R + np.eye(3)) / 2.0
        k = int(np.argmax(np.diag(M)))
        axis = M[:, k] / np.sqrt(M[k, k])
    else:
        axis = np.array([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]]) / (2.0 * np.sin(angle))
    axis /= np.linalg.norm(axis)
    q = np.concatenate([[np.cos(angle / 2)], np.sin(angle / 2) * axis])
    return q if q[0] >= 0 else -q
