"""PyTorch front-end: workspace management and the autograd Function.

PyTorch provides device memory and streams only.  Every stage of the
forward and backward passes runs in the HIP library through the C ABI.

The joint optimisation of the paper (Gaussians and camera poses, Sec. 1 and
Sec. 5.2) needs gradients with respect to every Gaussian parameter and to each
view's world->camera matrix; `rasterize` returns an image whose backward
delivers both.  Per-pixel compositing state is recomputed in the backward, not
stored: the workspace keeps only the sorted pairs, per-item records and two
values per pixel (final transmittance, last contributor).
"""
from __future__ import annotations

from typing import List, Optional, Sequence

import torch

from . import gsr

PARAM_NAMES = ("means", "log_scales", "quats", "opacities", "sh")


class GaussianRasterizer:
    """Rasterizes a fixed set of cameras (intrinsics) for a Gaussian scene.

    Capacity: the number of (tile, Gaussian) pairs is data dependent.  In the
    default synchronous mode every forward checks it once on the host and
    grows the workspace when needed.  With ``sync=False`` the forward never
    waits: the capacity is the last measured pair count times `headroom`, and
    an overflow is reported by `check_overflow` after the fact, which also
    sizes the sort of tile lists longer than 4096 entries for later forwards.
    """

    def __init__(self, cams: Sequence, sh_degree: int, tile_h: int = 16, persistent: bool = False,
                 sync: bool = True, headroom: float = 1.3, min_capacity: int = 1 << 16,
                 persistent_ctas: int = 0, device=None, active_count: Optional[torch.Tensor] = None):
        """active_count: None, or a one-element int64 device tensor holding how
        many leading Gaussians take part (the rest of the parameter arrays is
        capacity and is never read), e.g. the size of a level-of-detail cut
        computed on the device."""
        if len(cams) < 1 or len(cams) > gsr.GSR_MAX_VIEWS:
            raise ValueError(f"1..{gsr.GSR_MAX_VIEWS} views per call")
        self.cams = list(cams)
        self.sh_degree = int(sh_degree)
        self.active_count = active_count  # kept alive: the launch config holds its address
        self.cfg = gsr.launch_config(tile_h, persistent_ctas, active_count=active_count)
        self.persistent = bool(persistent)
        self.sync = bool(sync)
        self.headroom = float(headroom)
        self.capacity = int(min_capacity)
        self.device = torch.device("cuda") if device is None else torch.device(device)
        self.sizes = [(int(c.height), int(c.width)) for c in self.cams]
        self.total_pixels = sum(h * w for h, w in self.sizes)
        self.stats = False  # count work in the forward (slower; for measurement)
        self.last_pairs = None
        self.last_twist_grad = None

    @property
    def flags(self) -> int:
        return ((gsr.GSR_FLAG_SYNC if self.sync else 0) | (gsr.GSR_FLAG_PERSISTENT if self.persistent else 0)
                | (gsr.GSR_FLAG_STATS if self.stats else 0))

    def workspace(self, n: int, capacity: Optional[int] = None) -> torch.Tensor:
        cap = self.capacity if capacity is None else int(capacity)
        nb = gsr.workspace_bytes(n, self.cams, cap, self.cfg)
        return torch.empty(nb, dtype=torch.uint8, device=self.device)

    def forward(self, params: Sequence[torch.Tensor], world_to_cam: torch.Tensor, bg=(0.0, 0.0, 0.0),
                ws: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None):
        """Returns (planar images of all views, workspace)."""
        params = [gsr._as_param(t, nm) for t, nm in zip(params, PARAM_NAMES)]
        w2c = gsr._as_param(world_to_cam, "world_to_cam").reshape(len(self.cams), 16)
        n = int(params[0].shape[0])
        rgb = out if out is not None else torch.empty(3 * self.total_pixels, dtype=torch.float32, device=self.device)
        for _ in range(8):
            if ws is None:
                ws = self.workspace(n)
            try:
                gsr.rasterize_forward(ws, params, self.sh_degree, self.cams, w2c, bg, rgb, None, self.flags, self.cfg)
            except gsr.CapacityError:
                needed, _, _ = gsr.query_pairs(ws)
                self.capacity = max(self.capacity, int(needed * self.headroom) + 1024)
                ws = None
                continue
            return rgb, ws
        raise RuntimeError("pair capacity did not converge")

    def check_overflow(self, ws: torch.Tensor) -> bool:
        """Blocking: True if the last forward on ws skipped binning; records
        the pair count and raises the capacity for the next workspace."""
        needed, cap, ovf = gsr.query_pairs(ws)
        self.last_pairs = needed
        if ovf or needed * self.headroom > self.capacity:
            self.capacity = max(self.capacity, int(needed * self.headroom) + 1024)
        # lists longer than one workgroup sorts: enqueue enough merge passes for
        # the longest one seen (the synchronous forward sizes them itself)
        longest = gsr.query_stats(ws)["longest_list"]
        self.cfg.long_list_passes = max(int(self.cfg.long_list_passes), gsr.long_list_passes(longest))
        return ovf

    def backward(self, ws: torch.Tensor, params: Sequence[torch.Tensor], world_to_cam: torch.Tensor, bg,
                 rgb: torch.Tensor, grad_rgb: torch.Tensor, want_pose: bool = True):
        params = [gsr._as_param(t, nm) for t, nm in zip(params, PARAM_NAMES)]
        w2c = gsr._as_param(world_to_cam, "world_to_cam").reshape(len(self.cams), 16)
        grads = [torch.empty_like(t) for t in params]
        V = len(self.cams)
        g_w2c = torch.empty((V, 16), dtype=torch.float32, device=self.device) if want_pose else None
        g_tw = torch.empty((V, 6), dtype=torch.float32, device=self.device) if want_pose else None
        gsr.rasterize_backward(ws, params, self.sh_degree, self.cams, w2c, bg, rgb, grad_rgb.contiguous(), grads,
                               g_w2c, g_tw, self.flags & gsr.GSR_FLAG_PERSISTENT, self.cfg)
        return grads, (g_w2c.reshape(V, 4, 4) if want_pose else None), g_tw

    def backward_l1(self, ws: torch.Tensor, params: Sequence[torch.Tensor], world_to_cam: torch.Tensor, bg,
                    rgb: torch.Tensor, target: torch.Tensor, want_pose: bool = True):
        """Backward of the mean absolute error between rgb and target (same
        planar layout), with dL/drgb formed inside the library."""
        params = [gsr._as_param(t, nm) for t, nm in zip(params, PARAM_NAMES)]
        w2c = gsr._as_param(world_to_cam, "world_to_cam").reshape(len(self.cams), 16)
        grads = [torch.empty_like(t) for t in params]
        V = len(self.cams)
        g_w2c = torch.empty((V, 16), dtype=torch.float32, device=self.device) if want_pose else None
        g_tw = torch.empty((V, 6), dtype=torch.float32, device=self.device) if want_pose else None
        gsr.rasterize_backward_l1(ws, params, self.sh_degree, self.cams, w2c, bg, rgb,
                                  gsr._as_param(target, "target"), grads, g_w2c, g_tw,
                                  self.flags & gsr.GSR_FLAG_PERSISTENT, self.cfg)
        return grads, (g_w2c.reshape(V, 4, 4) if want_pose else None), g_tw

    def step_l1(self, params: Sequence[torch.Tensor], world_to_cam: torch.Tensor, bg, target: torch.Tensor,
                ws: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None, want_pose: bool = True):
        """Forward and the backward of the mean absolute error against target
        in one library call: the same image, gradients and workspace state as
        forward() then backward_l1().  Returns (rgb, ws, grads, 4x4 pose
        gradients, twist gradients)."""
        params = [gsr._as_param(t, nm) for t, nm in zip(params, PARAM_NAMES)]
        w2c = gsr._as_param(world_to_cam, "world_to_cam").reshape(len(self.cams), 16)
        tgt = gsr._as_param(target, "target")
        n = int(params[0].shape[0])
        rgb = out if out is not None else torch.empty(3 * self.total_pixels, dtype=torch.float32, device=self.device)
        grads = [torch.empty_like(t) for t in params]
        V = len(self.cams)
        g_w2c = torch.empty((V, 16), dtype=torch.float32, device=self.device) if want_pose else None
        g_tw = torch.empty((V, 6), dtype=torch.float32, device=self.device) if want_pose else None
        for _ in range(8):
            if ws is None:
                ws = self.workspace(n)
            try:
                gsr.rasterize_step_l1(ws, params, self.sh_degree, self.cams, w2c, bg, tgt, rgb, grads, g_w2c, g_tw,
                                      None, self.flags, self.cfg)
            except gsr.CapacityError:
                needed, _, _ = gsr.query_pairs(ws)
                self.capacity = max(self.capacity, int(needed * self.headroom) + 1024)
                ws = None
                continue
            return rgb, ws, grads, (g_w2c.reshape(V, 4, 4) if want_pose else None), g_tw
        raise RuntimeError("pair capacity did not converge")

    def split(self, rgb: torch.Tensor) -> List[torch.Tensor]:
        """Planar concatenated images -> list of [3, H, W] views."""
        out, o = [], 0
        for h, w in self.sizes:
            out.append(rgb[o:o + 3 * h * w].view(3, h, w))
            o += 3 * h * w
        return out


class _Rasterize(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rast: GaussianRasterizer, bg, means, log_scales, quats, opacities, sh, world_to_cam):
        params = [t.detach().contiguous() for t in (means, log_scales, quats, opacities, sh)]
        w2c = world_to_cam.detach().contiguous()
        rgb, ws = rast.forward(params, w2c, bg)
        ctx.rast, ctx.bg, ctx.ws = rast, bg, ws
        ctx.want_pose = world_to_cam.requires_grad
        ctx.save_for_backward(*params, w2c, rgb)
        return rgb

    @staticmethod
    def backward(ctx, grad_rgb):
        *params, w2c, rgb = ctx.saved_tensors
        grads, g_w2c, g_tw = ctx.rast.backward(ctx.ws, params, w2c, ctx.bg, rgb, grad_rgb, want_pose=True)
        ctx.rast.last_twist_grad = g_tw
        ctx.ws = None
        return (None, None, *grads, g_w2c.reshape(w2c.shape) if ctx.want_pose else None)


def rasterize(means, log_scales, quats, opacities, sh, world_to_cam, rasterizer: GaussianRasterizer,
              bg=(0.0, 0.0, 0.0)) -> torch.Tensor:
    """Differentiable render of all of the rasterizer's views.

    Returns planar images concatenated over views (see GaussianRasterizer.split).
    Gradients flow to every Gaussian parameter and to world_to_cam [V, 4, 4];
    the 6-DoF twist gradient of each view is left in rasterizer.last_twist_grad.
    """
    return _Rasterize.apply(rasterizer, tuple(float(x) for x in bg), means, log_scales, quats, opacities, sh,
                            world_to_cam)
