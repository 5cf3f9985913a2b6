"""FP64 reference of the per-view level-of-detail cut of a Gaussian hierarchy.

Test infrastructure only: nothing in the product imports this module.  It
follows the traversal the paper describes for rendering a stored hierarchy
(Sec. 7.2): start with the roots (nodes without a parent) and descend until a
node is finer than the threshold or is a leaf.  The screen size of a node is
read as S = max(fx, fy) * (largest axis scale) / (distance of its mean to the
camera centre) -- the projected extent of its largest axis in pixels; the
distance (not the depth) keeps S defined beside and behind the camera.
"""
from __future__ import annotations

import numpy as np


def camera_centre(world_to_cam) -> np.ndarray:
    T = np.asarray(world_to_cam, np.float64).reshape(4, 4)
    return -T[:3, :3].T @ T[:3, 3]


def screen_size(means, log_scales, world_to_cam, focal) -> np.ndarray:
    d = np.linalg.norm(np.asarray(means, np.float64) - camera_centre(world_to_cam), axis=1)
    return float(focal) * np.exp(np.asarray(log_scales, np.float64).max(axis=1)) / np.maximum(d, 1e-9)


def cut(means, log_scales, parent, world_to_cam, focal, tau) -> np.ndarray:
    """Ascending node indices of the cut.  parent [n] (negative for roots)."""
    parent = np.asarray(parent, np.int64)
    n = parent.shape[0]
    # children lists from the parent links
    has_parent = parent >= 0
    order = np.argsort(parent[has_parent], kind="stable")
    kids = np.nonzero(has_parent)[0][order]
    counts = np.bincount(parent[has_parent], minlength=n)
    first = np.concatenate([[0], np.cumsum(counts)])
    S = screen_size(means, log_scales, world_to_cam, focal)
    out = []
    frontier = np.nonzero(~has_parent)[0]
    while frontier.size:
        stop = (counts[frontier] == 0) | (S[frontier] < tau)
        out.append(frontier[stop])
        go = frontier[~stop]
        frontier = np.concatenate([kids[first[g]:first[g + 1]] for g in go]) if go.size else go
    return np.sort(np.concatenate(out)) if out else np.zeros(0, np.int64)


def ambiguous(means, log_scales, world_to_cam, focal, tau, rel=1e-9) -> np.ndarray:
    """Nodes whose screen size ties the threshold within `rel`."""
    S = screen_size(means, log_scales, world_to_cam, focal)
    return np.abs(S / tau - 1.0) < rel
