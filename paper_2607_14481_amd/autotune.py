"""Autotuner for the batched multi-view form.

Picks, by measurement on the workload itself, how many views go into one
launch sequence, the tile height (16 x {8, 16, 32} pixels; results are
independent of it because tile membership is the exact alpha >= 1/255 box),
whether compositing runs as persistent work-queue launches and, when all
views go into one call, whether that call is the fused one-call step
(gsr_rasterize_step_l1; bitwise the same results as forward + backward_l1).  Results are
cached in a JSON file keyed by the workload's signature and the device.
"""
from __future__ import annotations

import json
import os
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from .rasterizer import GaussianRasterizer

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "gsr_autotune.json")


def signature(n: int, sh_degree: int, cams: Sequence) -> str:
    sizes = ",".join(f"{c.width}x{c.height}" for c in cams)
    return f"{torch.cuda.get_device_name()}|n={n}|deg={sh_degree}|views={sizes}"


class MultiViewStep:
    """One optimisation step over all views: forward, L1 loss against the
    targets, backward; gradients summed over views.  Views are split into
    launch groups of `views_per_launch`; with one group and `fused`, the step
    is one gsr_rasterize_step_l1 call."""

    def __init__(self, cams, sh_degree, params, w2c, targets, views_per_launch=8, tile_h=16, persistent=False,
                 sync=True, capacity_hint: Optional[List[int]] = None, fused: bool = False):
        self.params = params
        self.groups = []
        V = len(cams)
        for g0 in range(0, V, views_per_launch):
            idx = list(range(g0, min(V, g0 + views_per_launch)))
            rast = GaussianRasterizer([cams[i] for i in idx], sh_degree, tile_h=tile_h, persistent=persistent,
                                      sync=sync)
            if capacity_hint is not None:
                rast.capacity = int(sum(capacity_hint[i] for i in idx) * 1.3) + 4096
            tgt = torch.cat([targets[i] for i in idx])
            self.groups.append((rast, w2c[idx].contiguous(), tgt))
        self.numel = sum(t.numel() for t in targets)
        self.fused = bool(fused) and len(self.groups) == 1
        self.ws = [None] * len(self.groups)
        self.out = [None] * len(self.groups)

    def __call__(self, keep_workspaces=False):
        total = None
        pose = []
        for k, (rast, w2c, tgt) in enumerate(self.groups):
            if self.fused:  # the call's own mean absolute error is the step's loss
                rgb, ws, grads, g_w2c, _ = rast.step_l1(self.params, w2c, (0.0, 0.0, 0.0), tgt,
                                                        ws=self.ws[k] if keep_workspaces else None, out=self.out[k])
                if keep_workspaces:
                    self.ws[k], self.out[k] = ws, rgb
                return grads, g_w2c
            rgb, ws = rast.forward(self.params, w2c, ws=self.ws[k] if keep_workspaces else None, out=self.out[k])
            if keep_workspaces:
                self.ws[k], self.out[k] = ws, rgb
            if len(self.groups) == 1:  # the call's own mean absolute error is the step's loss
                grads, g_w2c, _ = rast.backward_l1(ws, self.params, w2c, (0.0, 0.0, 0.0), rgb, tgt)
            else:
                grad = torch.sign(rgb - tgt) / self.numel
                grads, g_w2c, _ = rast.backward(ws, self.params, w2c, (0.0, 0.0, 0.0), rgb, grad)
            total = grads if total is None else [a + b for a, b in zip(total, grads)]
            pose.append(g_w2c)
        return total, torch.cat(pose)


def _time(step, steps, warmup):
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        step()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def autotune(cams, sh_degree, params, w2c, targets, candidates: Optional[List[Dict]] = None, steps: int = 5,
             warmup: int = 2, cache_path: Optional[str] = DEFAULT_CACHE, log=None) -> Dict:
    """Returns {"best": config, "ms": {config_key: ms}}; config = dict(views_per_launch, tile_h, persistent,
    fused)."""
    V = len(cams)
    n = int(params[0].shape[0])
    sig = signature(n, sh_degree, cams)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            with open(cache_path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if sig in cache:
        return cache[sig]
    if candidates is None:
        vpl = sorted({v for v in (1, 2, 4, 8, V) if v <= V})
        candidates = [dict(views_per_launch=v, tile_h=th, persistent=p, fused=f)
                      for v in vpl for th in (8, 16, 32) for p in (False, True)
                      for f in ((False, True) if v >= V else (False,))]
    results = {}
    best, best_ms = None, float("inf")
    for cand in candidates:
        step = MultiViewStep(cams, sh_degree, params, w2c, targets, **cand)
        ms = _time(step, steps, warmup)
        key = f"v{cand['views_per_launch']}_th{cand['tile_h']}_p{int(cand['persistent'])}" + \
            ("_fused" if cand.get("fused") else "")
        results[key] = round(ms, 4)
        if log:
            log(f"[autotune] {key}: {ms:.3f} ms")
        if ms < best_ms:
            best, best_ms = cand, ms
        del step
    out = {"best": best, "best_ms": best_ms, "ms": results}
    if cache_path:
        try:
            os.makedirs(os.path.dirname(cache_path), exist_ok=True)
            cache[sig] = out
            with open(cache_path, "w") as f:
                json.dump(cache, f, indent=1)
        except OSError:
            pass
    return out
