"""ctypes front-end of the FP64 C oracle (the tiled, hand-differentiated one).

TEST INFRASTRUCTURE ONLY.  Only tests, the package smoke check and the
benchmark's CPU-baseline leg may import this module.  It does not import the
GPU package, and the GPU package never imports it.

Scenes and cameras are duck-typed: any object with the attributes
``means, log_scales, quats, opacities, sh, sh_degree`` (numpy arrays) and
``width, height, fx, fy, cx, cy, near, world_to_cam`` respectively.  All
arithmetic happens in float64 on copies of the inputs.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

G_FIELDS = ("u", "v", "A", "B", "C", "o", "r", "g", "b")


class OrCamera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_double), ("fy", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double), ("near_plane", C.c_double),
                ("w2c", C.c_double * 16)]


class OrOpts(C.Structure):
    _fields_ = [("tile_w", C.c_int32), ("tile_h", C.c_int32), ("alpha_max", C.c_double),
                ("alpha_min", C.c_double), ("t_min", C.c_double), ("eps_alpha", C.c_double),
                ("eps_t", C.c_double), ("eps_z_rel", C.c_double)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIB_PATH)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        up = C.POINTER(C.c_uint32)
        bp = C.POINTER(C.c_uint8)
        L.or_render.restype = C.c_int64
        L.or_render.argtypes = [C.c_int64, C.c_int, dp, dp, dp, dp, dp, C.POINTER(OrCamera), dp,
                                C.POINTER(OrOpts), bp, dp, dp, ip, bp, dp, dp, dp, dp, dp, dp, dp, dp]
        L.or_project.restype = None
        L.or_project.argtypes = [C.c_int64, C.c_int, dp, dp, dp, dp, dp, C.POINTER(OrCamera),
                                 C.c_int, C.c_int, dp, ip, ip, up]
        L.or_bin.restype = C.c_int64
        L.or_bin.argtypes = [C.c_int64, ip, ip, up, C.c_int32, C.c_int32, C.c_int64, up, up, up]
        L.or_sh_basis.restype = None
        L.or_sh_basis.argtypes = [C.c_int, dp, dp]
        L.or_quat_to_rot.restype = None
        L.or_quat_to_rot.argtypes = [dp, dp]
        L.or_pose_twist.restype = None
        L.or_pose_twist.argtypes = [dp, dp, dp]
        L.or_default_opts.restype = None
        L.or_default_opts.argtypes = [C.POINTER(OrOpts)]
        _lib = L
    return _lib


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, t):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(t))


def _cam(cam) -> OrCamera:
    c = OrCamera()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.near_plane = float(getattr(cam, "near", 0.2))
    w = np.asarray(cam.world_to_cam, np.float64).reshape(16)
    for i in range(16):
        c.w2c[i] = float(w[i])
    return c


def default_opts(tile=(16, 16), **kw) -> OrOpts:
    o = OrOpts()
    lib().or_default_opts(C.byref(o))
    o.tile_w, o.tile_h = int(tile[0]), int(tile[1])
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def tile_grid(cam, tile=(16, 16)):
    return (-(-int(cam.width) // tile[0]), -(-int(cam.height) // tile[1]))


def render(scene, cam, bg=(0.0, 0.0, 0.0), tile=(16, 16), tile_mask=None, dL_dimg=None,
           want_screen=False, **opt_kw) -> dict:
    """Forward (and, with dL_dimg, backward) of one view in float64.

    Returns img [H, W, 3], T [H, W], n_contrib [H, W], ambig [H, W] (bool;
    ambig_why holds the reasons as bits: 1 alpha near 1/255, 2 near the 0.99
    clamp, 4 transmittance near the stop, 8 a float32 depth tie),
    M (pair count) and, with dL_dimg, gradients of every parameter, the 4x4
    pose gradient ``w2c`` and its 6-DoF twist (translation first).
    """
    L = lib()
    n = int(scene.means.shape[0])
    deg = int(scene.sh_degree)
    means, ls, qs, op, sh = (_d(scene.means), _d(scene.log_scales), _d(scene.quats),
                             _d(scene.opacities), _d(scene.sh))
    H, W = int(cam.height), int(cam.width)
    img = np.full((H, W, 3), np.nan)
    T = np.full((H, W), np.nan)
    nc = np.full((H, W), -1, np.int32)
    amb = np.zeros((H, W), np.uint8)
    ccam = _cam(cam)
    opts = default_opts(tile, **opt_kw)
    bgd = _d(bg)
    mask = None if tile_mask is None else np.ascontiguousarray(tile_mask, np.uint8)
    out = {}
    if dL_dimg is not None:
        g = _d(dL_dimg).reshape(H, W, 3)
        gm, gl, gq = np.zeros_like(means), np.zeros_like(ls), np.zeros_like(qs)
        go, gs = np.zeros_like(op), np.zeros_like(sh)
        gw = np.zeros(16)
        gscr = np.zeros((n, 9)) if want_screen else None
    else:
        g = gm = gl = gq = go = gs = gw = gscr = None
    dp = C.c_double
    m = L.or_render(n, deg, _ptr(means, dp), _ptr(ls, dp), _ptr(qs, dp), _ptr(op, dp), _ptr(sh, dp),
                    C.byref(ccam), _ptr(bgd, dp), C.byref(opts), _ptr(mask, C.c_uint8),
                    _ptr(img, dp), _ptr(T, dp), _ptr(nc, C.c_int32), _ptr(amb, C.c_uint8),
                    _ptr(g, dp), _ptr(gm, dp), _ptr(gl, dp), _ptr(gq, dp), _ptr(go, dp), _ptr(gs, dp),
                    _ptr(gw, dp), _ptr(gscr, dp))
    out.update(img=img, T=T, n_contrib=nc, ambig=amb.astype(bool), ambig_why=amb, M=int(m))
    if dL_dimg is not None:
        out.update(means=gm, log_scales=gl, quats=gq, opacities=go, sh=gs, w2c=gw.reshape(4, 4),
                   twist=pose_twist(gw.reshape(4, 4), cam.world_to_cam))
        if want_screen:
            out["screen"] = gscr
    return out


def project(scene, cam, tile=(16, 16)) -> dict:
    """Per-Gaussian projection records in float64 (stage A1 of the path)."""
    L = lib()
    n = int(scene.means.shape[0])
    means, ls, qs, op, sh = (_d(scene.means), _d(scene.log_scales), _d(scene.quats),
                             _d(scene.opacities), _d(scene.sh))
    rec = np.zeros((n, 16))
    rect = np.zeros((n, 4), np.int32)
    trect = np.zeros((n, 4), np.int32)
    zb = np.zeros(n, np.uint32)
    ccam = _cam(cam)
    dp = C.c_double
    L.or_project(n, int(scene.sh_degree), _ptr(means, dp), _ptr(ls, dp), _ptr(qs, dp), _ptr(op, dp),
                 _ptr(sh, dp), C.byref(ccam), int(tile[0]), int(tile[1]), _ptr(rec, dp),
                 _ptr(rect, C.c_int32), _ptr(trect, C.c_int32), _ptr(zb, C.c_uint32))
    return dict(u=rec[:, 0], v=rec[:, 1], z=rec[:, 2], cov=rec[:, 3:6], conic=rec[:, 6:9],
                opacity=rec[:, 9], rgb=rec[:, 10:13], visible=rec[:, 13] > 0.5, rect=rect,
                trect=trect, zbits=zb)


def bin_pairs(visible, trect, zbits, tiles_x, tiles_y):
    """Sorted (tile, gid) pairs and per-tile [start, end) from tile boxes and
    depth bits (integer work only)."""
    L = lib()
    vis = np.ascontiguousarray(visible, np.int32)
    tr = np.ascontiguousarray(trect, np.int32)
    zb = np.ascontiguousarray(zbits, np.uint32)
    n = int(vis.shape[0])
    n_tiles = int(tiles_x) * int(tiles_y)
    ranges = np.zeros((n_tiles, 2), np.uint32)
    m = L.or_bin(n, _ptr(vis, C.c_int32), _ptr(tr, C.c_int32), _ptr(zb, C.c_uint32), int(tiles_x),
                 int(tiles_y), 0, None, None, _ptr(ranges, C.c_uint32))
    tiles = np.zeros(max(m, 1), np.uint32)
    gids = np.zeros(max(m, 1), np.uint32)
    L.or_bin(n, _ptr(vis, C.c_int32), _ptr(tr, C.c_int32), _ptr(zb, C.c_uint32), int(tiles_x),
             int(tiles_y), m, _ptr(tiles, C.c_uint32), _ptr(gids, C.c_uint32), _ptr(ranges, C.c_uint32))
    return tiles[:m], gids[:m], ranges


def sh_basis(degree, dirs) -> np.ndarray:
    L = lib()
    dirs = _d(np.atleast_2d(dirs))
    out = np.zeros((dirs.shape[0], 16))
    for i in range(dirs.shape[0]):
        row = np.ascontiguousarray(dirs[i])
        o = np.zeros(16)
        L.or_sh_basis(int(degree), _ptr(row, C.c_double), _ptr(o, C.c_double))
        out[i] = o
    return out[:, : (degree + 1) ** 2]


def quat_to_rot(q) -> np.ndarray:
    q = _d(q)
    R = np.zeros(9)
    lib().or_quat_to_rot(_ptr(q, C.c_double), _ptr(R, C.c_double))
    return R.reshape(3, 3)


def pose_twist(G, T) -> np.ndarray:
    g = _d(G).reshape(16)
    t = _d(T).reshape(16)
    out = np.zeros(6)
    lib().or_pose_twist(_ptr(g, C.c_double), _ptr(t, C.c_double), _ptr(out, C.c_double))
    return out


def render_views(scene, cams, bgs=None, dL_dimgs=None, tile=(16, 16), **kw):
    """Several views: images per view; parameter gradients summed over views;
    pose gradients per view."""
    outs = []
    tot = None
    for v, cam in enumerate(cams):
        bg = (0.0, 0.0, 0.0) if bgs is None else bgs[v]
        g = None if dL_dimgs is None else dL_dimgs[v]
        o = render(scene, cam, bg=bg, tile=tile, dL_dimg=g, **kw)
        outs.append(o)
        if g is not None:
            if tot is None:
                tot = {k: o[k].copy() for k in ("means", "log_scales", "quats", "opacities", "sh")}
            else:
                for k in tot:
                    tot[k] += o[k]
    return outs, tot
