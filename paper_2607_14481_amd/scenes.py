"""Seeded synthetic scenes and cameras for the rasterizer workloads.

This module builds inputs only.  It holds none of the rasterizer's arithmetic
(projection, colour evaluation, binning, compositing or their derivatives); both
the FP64 oracle and the GPU path consume what it returns.

The paper measures on captured datasets that are not available here, so these
draws stand in for them: Gaussian counts follow the paper's captures (1.3-3.7 M
trained Gaussians in the memory-scaling table of the appendix, 6.7 M at the
out-of-memory point of the hierarchy study), and the per-Gaussian distributions
are the ones fixed by the workload definitions below.  No dataset item is used.

Conventions (shared with the library's C ABI):
  * quaternions are stored (w, x, y, z) and need not be unit length;
  * opacities are activated values in [0, 1];
  * scales are stored as natural logarithms;
  * SH coefficients are laid out [N, K, 3] with K = (degree + 1)^2;
  * world_to_cam is a row-major 4x4 rigid transform with OpenCV axes
    (x right, y down, z forward); pixel centres sit at integer + 1/2.

Every generator draws from numpy ``Generator(PCG64(seed))`` in a fixed order:
means, log-scales, quaternions, opacities, SH DC, remaining SH, cameras, target
perturbation.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

# A degree-0 colour is (basis value) * DC + 1/2 with basis value 1 / (2 sqrt(pi)).
# Drawing the *colour* uniformly in [0, 1] therefore means drawing DC uniformly in
# [-sqrt(pi), sqrt(pi)]; this factor maps a drawn colour to its DC coefficient.
_DC_PER_UNIT_COLOUR = 2.0 * np.sqrt(np.pi)


@dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    world_to_cam: np.ndarray  # [4, 4] float32, row-major
    near: float = 0.2

    def copy_with_pose(self, world_to_cam: np.ndarray) -> "Camera":
        return Camera(self.width, self.height, self.fx, self.fy, self.cx, self.cy,
                      np.asarray(world_to_cam, np.float32).copy(), self.near)


@dataclass
class Scene:
    means: np.ndarray       # [N, 3] float32
    log_scales: np.ndarray  # [N, 3] float32
    quats: np.ndarray       # [N, 4] float32, (w, x, y, z)
    opacities: np.ndarray   # [N] float32 in [0, 1]
    sh: np.ndarray          # [N, K, 3] float32
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def with_means(self, means: np.ndarray) -> "Scene":
        return Scene(np.asarray(means, np.float32), self.log_scales, self.quats,
                     self.opacities, self.sh, self.sh_degree)

    def subset(self, idx) -> "Scene":
        return Scene(self.means[idx], self.log_scales[idx], self.quats[idx],
                     self.opacities[idx], self.sh[idx], self.sh_degree)


@dataclass
class Workload:
    name: str
    scene: Scene
    cameras: List[Camera]
    # the optimisation target: either a second scene (jittered means) or a
    # second set of camera poses, rendered by whichever path is under test
    target_scene: Optional[Scene] = None
    target_cameras: Optional[List[Camera]] = None
    meta: dict = field(default_factory=dict)
    extra: dict = field(default_factory=dict)  # objects that do not serialise (e.g. a hierarchy)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def _unit_quats(rng, n):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def _gaussian_body(rng, means, sh_degree, log_scale_mean=-3.0, log_scale_std=0.5,
                   sh_rest_std=0.1):
    """Draws everything after the means, in the fixed order."""
    n = means.shape[0]
    k = (sh_degree + 1) ** 2
    log_scales = rng.normal(log_scale_mean, log_scale_std, (n, 3))
    quats = _unit_quats(rng, n)
    opac = _sigmoid(rng.standard_normal(n))
    sh = np.zeros((n, k, 3))
    sh[:, 0, :] = (rng.uniform(0.0, 1.0, (n, 3)) - 0.5) * _DC_PER_UNIT_COLOUR
    if k > 1:
        sh[:, 1:, :] = rng.normal(0.0, sh_rest_std, (n, k - 1, 3))
    return Scene(means.astype(np.float32), log_scales.astype(np.float32),
                 quats.astype(np.float32), opac.astype(np.float32),
                 sh.astype(np.float32), sh_degree)


def look_at(eye, target=(0.0, 0.0, 0.0), up=(0.0, 0.0, 1.0)) -> np.ndarray:
    """World->camera 4x4 (OpenCV axes) for a camera at `eye` looking at `target`.

    Rows of the rotation are the camera's right, down and forward axes in world
    coordinates.  `up` is replaced by +y when it is nearly parallel to the view
    direction.
    """
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    up = np.asarray(up, np.float64)
    if abs(np.dot(f, up)) > 0.99:
        up = np.array([0.0, 1.0, 0.0])
    r = np.cross(f, up)
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    m = np.eye(4)
    m[0, :3], m[1, :3], m[2, :3] = r, d, f
    m[:3, 3] = -m[:3, :3] @ eye
    return m


def axis_angle_matrix(axis, angle) -> np.ndarray:
    """Rotation matrix about a unit axis (Rodrigues' formula)."""
    a = np.asarray(axis, np.float64)
    a = a / np.linalg.norm(a)
    k = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + np.sin(angle) * k + (1 - np.cos(angle)) * (k @ k)


def pinhole(width, height, world_to_cam, f=None, near=0.2) -> Camera:
    f = float(width) if f is None else float(f)
    return Camera(int(width), int(height), f, f, width / 2.0, height / 2.0,
                  np.asarray(world_to_cam, np.float32), near)


# ----------------------------------------------------------------------------
# Workloads
# ----------------------------------------------------------------------------

def small_view(seed=1, n=1000, width=128, height=128, sh_degree=0, jitter=0.01,
               z_range=(2.0, 6.0), xy_half=1.0, log_scale_mean=-3.0) -> Workload:
    """Single 128x128 pinhole view (fx = fy = 128, cx = cy = 64), identity pose,
    1,000 Gaussians with x, y ~ U(-1, 1), z ~ U(2, 6), log-scales ~ N(-3, 0.5),
    unit quaternions from normalised N(0, 1)^4, opacity = sigmoid(N(0, 1)),
    SH degree 0 with colour ~ U(0, 1); the target renders the same scene with
    means jittered by N(0, 0.01^2).  Width/height/n/degree are parameters so
    that small variants of the same recipe serve the tests.
    """
    rng = _rng(seed)
    means = np.empty((n, 3))
    means[:, :2] = rng.uniform(-xy_half, xy_half, (n, 2))
    means[:, 2] = rng.uniform(z_range[0], z_range[1], n)
    scene = _gaussian_body(rng, means, sh_degree, log_scale_mean=log_scale_mean)
    f = 128.0 * width / 128.0
    cam = Camera(width, height, f, f, width / 2.0, height / 2.0, np.eye(4, dtype=np.float32))
    jittered = scene.means + rng.normal(0.0, jitter, (n, 3)).astype(np.float32)
    return Workload("small_view", scene, [cam], target_scene=scene.with_means(jittered),
                    meta={"seed": seed})


def _box_scene(rng, n, half=10.0, sh_degree=3):
    means = rng.uniform(-half, half, (n, 3))
    return _gaussian_body(rng, means, sh_degree)


def single_view_1080p(seed=2, n=200_000, distance=40.0) -> Workload:
    """Single 1920x1080 view of 200k Gaussians in a 20 m box (SH degree 3, rest
    coefficients ~ N(0, 0.1)); camera 40 m from the box centre in a uniformly
    random direction, looking at it; target = the pose left-multiplied by a
    0.5 degree rotation about a random axis and a 2 cm translation."""
    rng = _rng(seed)
    scene = _box_scene(rng, n)
    d = rng.standard_normal(3)
    d /= np.linalg.norm(d)
    w2c = look_at(d * distance)
    cam = pinhole(1920, 1080, w2c)
    axis = rng.standard_normal(3)
    tdir = rng.standard_normal(3)
    tdir /= np.linalg.norm(tdir)
    delta = np.eye(4)
    delta[:3, :3] = axis_angle_matrix(axis, np.deg2rad(0.5))
    delta[:3, 3] = 0.02 * tdir
    target = cam.copy_with_pose((delta @ w2c.astype(np.float64)).astype(np.float32))
    return Workload("single_view_1080p", scene, [cam], target_cameras=[target],
                    meta={"seed": seed, "distance": distance})


RESOLUTIONS = ((640, 480), (1280, 720), (1920, 1080))


def multi_view_ring(seed=3, n=1_000_000, n_views=8, radius=15.0) -> Workload:
    """1M Gaussians (20 m box, SH degree 3) seen by 8 cameras at angles
    2*pi*k/8 on a 15 m circle in the z = 0 plane, each looking at the centre,
    each with a resolution drawn uniformly from 640x480 / 1280x720 / 1920x1080."""
    rng = _rng(seed)
    scene = _box_scene(rng, n)
    res = rng.integers(0, len(RESOLUTIONS), n_views)
    cams = []
    for k in range(n_views):
        ang = 2 * np.pi * k / n_views
        eye = radius * np.array([np.cos(ang), np.sin(ang), 0.0])
        w, h = RESOLUTIONS[res[k]]
        cams.append(pinhole(w, h, look_at(eye)))
    return Workload("multi_view_ring", scene, cams, meta={"seed": seed, "res_idx": res.tolist()})


def perturbed_pose(world_to_cam, seed, degrees=0.5, metres=0.02) -> np.ndarray:
    """Left-multiplies a pose by a rotation of `degrees` about a random axis and
    a translation of `metres` in a random direction (seeded)."""
    rng = _rng(seed)
    axis = rng.standard_normal(3)
    tdir = rng.standard_normal(3)
    tdir /= np.linalg.norm(tdir)
    delta = np.eye(4)
    delta[:3, :3] = axis_angle_matrix(axis, np.deg2rad(degrees))
    delta[:3, 3] = metres * tdir
    return (delta @ np.asarray(world_to_cam, np.float64)).astype(np.float32)


def headline_view(seed=3, n=1_000_000) -> Workload:
    """The first 1920x1080 camera of the 8-view ring over the 1M-Gaussian scene;
    the optimisation target is rendered from that pose perturbed by 0.5 degrees
    and 2 cm (as for the single-view 1080p workload)."""
    wl = multi_view_ring(seed=seed, n=n)
    idx = next(i for i, c in enumerate(wl.cameras) if c.width == 1920)
    cam = wl.cameras[idx]
    target = cam.copy_with_pose(perturbed_pose(cam.world_to_cam, seed + 1000))
    return Workload("headline_1080p_1M", wl.scene, [cam], target_cameras=[target],
                    meta={"seed": seed, "ring_index": idx})


def random_upstream(seed, shape) -> np.ndarray:
    """Fixed N(0, 1) upstream gradient used by parity tests in place of a loss."""
    return _rng(seed).standard_normal(shape).astype(np.float32)


def street_leaves(seed=4, n=4_000_000, length=2000.0, width=20.0, height=10.0, eye_height=2.0,
                  max_heading_deg=10.0):
    """Leaf Gaussians of the hierarchical level-of-detail workload: a 2 km street
    (x in [0, 2000], y in [-10, 10], z in [0, 10] metres) with centres uniform
    in it and the box scene's other distributions (log-scales ~ N(-3, 0.5),
    SH degree 3); one 1920x1080 camera at the start of the street, (-1, 0, 2),
    looking down it at a seeded heading within +-10 degrees (up = +z); the
    target pose is perturbed by 0.5 degrees and 2 cm.
    Returns (leaves, camera, target camera)."""
    rng = _rng(seed)
    means = np.empty((n, 3))
    means[:, 0] = rng.uniform(0.0, length, n)
    means[:, 1] = rng.uniform(-width / 2, width / 2, n)
    means[:, 2] = rng.uniform(0.0, height, n)
    leaves = _gaussian_body(rng, means, 3)
    az = np.deg2rad(rng.uniform(-max_heading_deg, max_heading_deg))
    eye = np.array([-1.0, 0.0, eye_height])
    cam = pinhole(1920, 1080, look_at(eye, eye + np.array([np.cos(az), np.sin(az), 0.0])))
    target = cam.copy_with_pose(perturbed_pose(cam.world_to_cam, seed + 1000))
    return leaves, cam, target
