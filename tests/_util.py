"""Shared test helpers: run the HIP path through the C ABI and reshape its
outputs to the oracle's conventions (images [H, W, 3])."""
from __future__ import annotations

import sys

import numpy as np


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def params_to_device(scene, device="cuda"):
    import torch
    return [torch.tensor(np.ascontiguousarray(getattr(scene, k), np.float32), device=device)
            for k in ("means", "log_scales", "quats", "opacities", "sh")]


def poses_to_device(cams, device="cuda"):
    import torch
    return torch.tensor(np.stack([np.asarray(c.world_to_cam, np.float32) for c in cams]), device=device)


def planar_to_hwc(rgb_flat, cams):
    out, o = [], 0
    x = rgb_flat.detach().cpu().numpy() if hasattr(rgb_flat, "detach") else np.asarray(rgb_flat)
    for c in cams:
        h, w = int(c.height), int(c.width)
        out.append(x[o:o + 3 * h * w].reshape(3, h, w).transpose(1, 2, 0))
        o += 3 * h * w
    return out


def hwc_to_planar(imgs):
    return np.concatenate([np.ascontiguousarray(np.asarray(i, np.float32).transpose(2, 0, 1)).reshape(-1)
                           for i in imgs])


def gpu_render(scene, cams, bg=(0.0, 0.0, 0.0), upstream=None, tile_h=16, persistent=False, sync=True,
               export=False):
    """Forward (+ backward with an [H, W, 3] upstream per view) on the GPU."""
    import torch
    from paper_2607_14481_amd import gsr
    from paper_2607_14481_amd.rasterizer import GaussianRasterizer

    rast = GaussianRasterizer(cams, scene.sh_degree, tile_h=tile_h, persistent=persistent, sync=sync)
    rast.stats = True
    params = params_to_device(scene)
    w2c = poses_to_device(cams)
    rgb, ws = rast.forward(params, w2c, bg)
    torch.cuda.synchronize()
    res = dict(imgs=planar_to_hwc(rgb, cams), rgb=rgb, ws=ws, rast=rast, stats=gsr.query_stats(ws))
    if export:
        res["state"] = gsr.export_state(ws, params, scene.sh_degree, cams, rast.cfg)
    if upstream is not None:
        g = torch.tensor(hwc_to_planar(upstream), device="cuda")
        grads, g_w2c, g_tw = rast.backward(ws, params, w2c, bg, rgb, g)
        torch.cuda.synchronize()
        for k, t in zip(("means", "log_scales", "quats", "opacities", "sh"), grads):
            res[k] = t.cpu().numpy().astype(np.float64)
        res["w2c"] = g_w2c.cpu().numpy().astype(np.float64)
        res["twist"] = g_tw.cpu().numpy().astype(np.float64)
    return res


def rel_err(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


GRAD_KEYS = ("means", "log_scales", "quats", "opacities", "sh")


def oracle_bin_from_gpu_state(st, cams, n, tile_h=16):
    """Tier (i): the oracle's integer binning fed with the GPU's boxes and depth bits."""
    from oracle import oracle as O
    rec = st["records"]
    bx = rec[:, 9].view(np.uint32)
    by = rec[:, 10].view(np.uint32)
    vis = st["tile_counts"] > 0
    tiles_all, items_all = [], []
    tile_off = 0
    ranges = []
    for v, c in enumerate(cams):
        sl = slice(v * n, (v + 1) * n)
        trect = np.stack([(bx[sl] & 0xffff) // 16, (by[sl] & 0xffff) // tile_h,
                          (bx[sl] >> 16) // 16, (by[sl] >> 16) // tile_h], 1).astype(np.int32)
        tx, ty = O.tile_grid(c, (16, tile_h))
        t, g, r = O.bin_pairs(vis[sl], trect, st["depth_keys"][sl], tx, ty)
        base = sum(len(x) for x in tiles_all)
        tiles_all.append(t.astype(np.uint64) + tile_off)
        items_all.append(g.astype(np.uint64) + v * n)
        rr = r.astype(np.int64)
        nonempty = rr[:, 1] > rr[:, 0]
        rr[nonempty] += base
        ranges.append(rr)
        tile_off += tx * ty
    return (np.concatenate(tiles_all), np.concatenate(items_all), np.concatenate(ranges))
