"""Level-of-detail hierarchy over a leaf Gaussian set, and its per-view cut.

Host-side preparation of the hierarchical workload; the rasterizer then runs
over the selected cut like over any other Gaussian set.

The paper keeps large scenes tractable with a hierarchy whose inner nodes are
merges of their children, chosen per view by screen size (Sec. 7, "A
Progressive Gaussian Hierarchy": nodes hold full Gaussian parameters; children
are merged by a KL-divergence criterion; rendering descends from the roots
until nodes are finer than a pixel threshold or are leaves).  This module builds
an octree-style version of it, as the hierarchical workload is defined:

  * leaves are ordered along a Morton (Z-order) curve of their quantised
    centres, and every run of 8 consecutive nodes becomes one parent, level by
    level (the last run of a level may be shorter);
  * a parent is the moment-matched merge of its children: with weights
    w_i = o_i / sum_j o_j, mean = sum w_i mu_i, covariance =
    sum w_i (Sigma_i + (mu_i - mean)(mu_i - mean)^T).  Among all single
    Gaussians this is the one that minimises KL(mixture || single), which is
    how the KL criterion is read here.  Opacity = 1 - prod(1 - o_i) (the
    children's coverage composited), SH = the w-weighted mean.  The covariance
    is factored back into log-scales and a quaternion by an eigendecomposition;
  * the cut starts at the roots and replaces a node by its children while the
    node's screen size S = f * max_axis_scale / distance is at least the
    threshold (1.5 px), stopping at leaves.  The distance is to the camera
    centre, so S is defined for nodes beside or behind the camera too.

Everything is numpy, FP64 internally, FP32 in the stored parameters.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Tuple

import numpy as np

from .scenes import Camera, Scene

BRANCHING = 8


@dataclass
class Hierarchy:
    nodes: Scene              # every node: leaves first (level 0), then level 1, ...
    level_start: np.ndarray   # int64 [levels + 2]: nodes of level l are [level_start[l], level_start[l+1])
    parent: np.ndarray        # int64 [n_nodes], -1 for roots
    child_start: np.ndarray   # int64 [n_nodes], -1 for leaves; children are consecutive
    child_count: np.ndarray   # int32 [n_nodes], 0 for leaves

    @property
    def levels(self) -> int:
        return len(self.level_start) - 1

    @property
    def roots(self) -> np.ndarray:
        return np.arange(self.level_start[-2], self.level_start[-1])

    def level_of(self, idx) -> np.ndarray:
        return np.searchsorted(self.level_start, np.asarray(idx), side="right") - 1


def _spread_bits(v: np.ndarray) -> np.ndarray:
    """Puts the low 21 bits of v at every third bit position (0, 3, 6, ...)."""
    v = v.astype(np.uint64) & np.uint64(0x1FFFFF)
    for shift, mask in ((32, 0x1F00000000FFFF), (16, 0x1F0000FF0000FF), (8, 0x100F00F00F00F00F),
                        (4, 0x10C30C30C30C30C3), (2, 0x1249249249249249)):
        v = (v | (v << np.uint64(shift))) & np.uint64(mask)
    return v


def morton_codes(points: np.ndarray) -> np.ndarray:
    """63-bit Morton codes of points quantised to 2^21 cubic cells along the
    longest side of their bounding box (cubic, so that a run of 8 codes is a
    compact cell whatever the box's aspect ratio)."""
    p = np.asarray(points, np.float64)
    lo, hi = p.min(0), p.max(0)
    ext = max(float((hi - lo).max()), 1e-30)
    q = np.floor((p - lo) / ext * (2 ** 21 - 1) + 0.5).astype(np.int64)
    return _spread_bits(q[:, 0]) | (_spread_bits(q[:, 1]) << np.uint64(1)) | (_spread_bits(q[:, 2]) << np.uint64(2))


def quat_to_rotation(q: np.ndarray) -> np.ndarray:
    """[N, 4] (w, x, y, z), any length -> [N, 3, 3] rotation of the unit quaternion."""
    q = np.asarray(q, np.float64)
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], -2)


def rotation_to_quat(r: np.ndarray) -> np.ndarray:
    """[N, 3, 3] proper rotations -> [N, 4] unit quaternions (w, x, y, z), w >= 0.
    Each row uses the largest of the four squared components, so no division
    is by a small number."""
    r = np.asarray(r, np.float64)
    tr = np.trace(r, axis1=1, axis2=2)
    # 4 * (w^2, x^2, y^2, z^2)
    sq = np.stack([1 + tr, 1 + 2 * r[:, 0, 0] - tr, 1 + 2 * r[:, 1, 1] - tr, 1 + 2 * r[:, 2, 2] - tr], 1)
    k = np.argmax(sq, axis=1)
    s = np.sqrt(np.maximum(sq[np.arange(len(r)), k], 1e-300))  # = 2 |component k|
    d = 2.0 * s  # the other components are (sums or differences of entries) / (4 |component k|)
    q = np.empty((len(r), 4))
    m = k == 0
    q[m] = np.stack([s[m] / 2, (r[m, 2, 1] - r[m, 1, 2]) / d[m], (r[m, 0, 2] - r[m, 2, 0]) / d[m],
                     (r[m, 1, 0] - r[m, 0, 1]) / d[m]], 1)
    m = k == 1
    q[m] = np.stack([(r[m, 2, 1] - r[m, 1, 2]) / d[m], s[m] / 2, (r[m, 0, 1] + r[m, 1, 0]) / d[m],
                     (r[m, 0, 2] + r[m, 2, 0]) / d[m]], 1)
    m = k == 2
    q[m] = np.stack([(r[m, 0, 2] - r[m, 2, 0]) / d[m], (r[m, 0, 1] + r[m, 1, 0]) / d[m], s[m] / 2,
                     (r[m, 1, 2] + r[m, 2, 1]) / d[m]], 1)
    m = k == 3
    q[m] = np.stack([(r[m, 1, 0] - r[m, 0, 1]) / d[m], (r[m, 0, 2] + r[m, 2, 0]) / d[m],
                     (r[m, 1, 2] + r[m, 2, 1]) / d[m], s[m] / 2], 1)
    q *= np.where(q[:, :1] < 0, -1.0, 1.0)
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def covariance(log_scales: np.ndarray, quats: np.ndarray) -> np.ndarray:
    """Sigma = R diag(exp(2 s)) R^T, [N, 3, 3] in FP64."""
    r = quat_to_rotation(quats)
    return np.einsum("nij,nj,nkj->nik", r, np.exp(2.0 * np.asarray(log_scales, np.float64)), r)


def factor_covariance(cov: np.ndarray, min_var: float = 1e-12) -> Tuple[np.ndarray, np.ndarray]:
    """Symmetric positive semi-definite [N, 3, 3] -> (log-scales [N, 3], quaternions [N, 4])."""
    vals, vecs = np.linalg.eigh(cov)
    vals = np.maximum(vals, min_var)
    det = np.linalg.det(vecs)
    vecs[:, :, 2] *= np.where(det < 0, -1.0, 1.0)[:, None]  # make it a proper rotation
    return 0.5 * np.log(vals), rotation_to_quat(vecs)


def merge_groups(mu, cov, opac, sh, starts):
    """Moment-matched merge of consecutive groups of nodes.

    mu [n, 3], cov [n, 3, 3], opac [n], sh [n, K, 3] (FP64), starts: first index
    of each group (ascending, starts[0] = 0).  Returns the parents' (mu, cov,
    opac, sh)."""
    n = len(mu)
    counts = np.diff(np.append(starts, n))
    group = np.repeat(np.arange(len(starts)), counts)
    wsum = np.add.reduceat(opac, starts)
    w = opac / wsum[group]
    mu_p = np.add.reduceat(w[:, None] * mu, starts)
    d = mu - mu_p[group]
    cov_p = np.add.reduceat(w[:, None, None] * (cov + d[:, :, None] * d[:, None, :]), starts)
    opac_p = -np.expm1(np.add.reduceat(np.log1p(-opac), starts))
    sh_p = np.add.reduceat(w[:, None, None] * sh, starts)
    return mu_p, cov_p, opac_p, sh_p


def build(leaves: Scene, levels: int = 7, branching: int = BRANCHING) -> Hierarchy:
    """Builds `levels` merge levels above the leaves (reordered in Morton order)."""
    order = np.argsort(morton_codes(leaves.means), kind="stable")
    leaves = leaves.subset(order)
    mu = leaves.means.astype(np.float64)
    cov = covariance(leaves.log_scales, leaves.quats)
    opac = np.minimum(leaves.opacities.astype(np.float64), 1.0 - 1e-12)
    sh = leaves.sh.astype(np.float64)
    parts = [(leaves.means, leaves.log_scales, leaves.quats, leaves.opacities, leaves.sh)]
    level_start = [0, len(mu)]
    child_start = [np.full(len(mu), -1, np.int64)]
    child_count = [np.zeros(len(mu), np.int32)]
    parents = []
    for _ in range(levels):
        n = len(mu)
        if n <= 1:
            break
        starts = np.arange(0, n, branching)
        mu, cov, opac, sh = merge_groups(mu, cov, opac, sh, starts)
        opac = np.minimum(opac, 1.0 - 1e-12)
        ls, q = factor_covariance(cov)
        parts.append((mu.astype(np.float32), ls.astype(np.float32), q.astype(np.float32),
                      opac.astype(np.float32), sh.astype(np.float32)))
        base_prev = level_start[-2]
        base = level_start[-1]
        child_start.append(base_prev + starts)
        child_count.append(np.diff(np.append(starts, n)).astype(np.int32))
        parents.append(base + np.repeat(np.arange(len(starts)), np.diff(np.append(starts, n))))
        level_start.append(base + len(starts))
    total = level_start[-1]
    parent = np.full(total, -1, np.int64)
    for l, p in enumerate(parents):
        parent[level_start[l]:level_start[l + 1]] = p
    nodes = Scene(*[np.concatenate([p[i] for p in parts]) for i in range(5)], leaves.sh_degree)
    return Hierarchy(nodes, np.asarray(level_start, np.int64), parent,
                     np.concatenate(child_start), np.concatenate(child_count))


def screen_size(h: Hierarchy, idx: np.ndarray, cam: Camera) -> np.ndarray:
    """S = f * largest axis scale / distance to the camera centre, in pixels."""
    w2c = np.asarray(cam.world_to_cam, np.float64)
    centre = -w2c[:3, :3].T @ w2c[:3, 3]
    dist = np.linalg.norm(h.nodes.means[idx].astype(np.float64) - centre, axis=1)
    smax = np.exp(h.nodes.log_scales[idx].astype(np.float64).max(axis=1))
    return max(cam.fx, cam.fy) * smax / np.maximum(dist, 1e-9)


def select_cut(h: Hierarchy, cam: Camera, tau: float = 1.5) -> np.ndarray:
    """Node indices of the cut for `cam`: descend from the roots while S >= tau."""
    frontier = h.roots
    out = []
    while frontier.size:
        leaf = h.child_count[frontier] == 0
        take = leaf | (screen_size(h, frontier, cam) < tau)
        out.append(frontier[take])
        exp = frontier[~take]
        cnt = h.child_count[exp].astype(np.int64)
        first = np.repeat(h.child_start[exp], cnt)
        within = np.arange(int(cnt.sum())) - np.repeat(np.cumsum(cnt) - cnt, cnt)
        frontier = first + within
    return np.sort(np.concatenate(out))


def lod_workload(seed=4, n_leaves=4_000_000, levels=7, tau=1.5):
    """The hierarchical level-of-detail workload: a 7-level, branching-8
    hierarchy over 4M leaves along a 2 km street and its 1.5 px cut for one
    1920x1080 view down the street.  The Workload's scene is the cut; meta
    holds its size and per-level counts, extra["hierarchy"] the hierarchy."""
    from .scenes import Workload, street_leaves
    leaves, cam, target = street_leaves(seed, n_leaves)
    h = build(leaves, levels)
    cut = select_cut(h, cam, tau)
    per_level = np.bincount(h.level_of(cut), minlength=h.levels)
    meta = {"seed": seed, "leaves": n_leaves, "nodes": int(h.level_start[-1]), "levels": h.levels - 1,
            "tau_px": tau, "cut": int(cut.size), "cut_per_level": per_level.tolist()}
    return Workload("lod_cut_1080p", h.nodes.subset(cut), [cam], target_cameras=[target], meta=meta,
                    extra={"hierarchy": h, "cut": cut})
