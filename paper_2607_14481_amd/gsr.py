"""ctypes binding of the C ABI in include/gsr.h (argument marshalling only).

Every step of the rasterizer runs in the HIP library; this module only turns
torch tensors into pointers and status codes into exceptions.  Loading fails
loudly when the library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgsr.so")

GSR_OK = 0
GSR_ERR_INVALID_ARGUMENT = 1
GSR_ERR_WORKSPACE_TOO_SMALL = 2
GSR_ERR_CAPACITY = 3
GSR_ERR_HIP = 4
GSR_ERR_UNSUPPORTED = 5
GSR_MAX_VIEWS = 32
GSR_FLAG_SYNC = 1
GSR_FLAG_PERSISTENT = 2
GSR_FLAG_STATS = 4

EXPORTED = ("gsr_version", "gsr_status_string", "gsr_last_error", "gsr_workspace_bytes",
            "gsr_rasterize_forward", "gsr_rasterize_backward", "gsr_rasterize_backward_l1",
            "gsr_rasterize_step_l1", "gsr_query_pairs",
            "gsr_query_stats",
            "gsr_export_state", "gsr_adam_step", "gsr_pose_step", "gsr_sim3_relocate",
            "gsr_hierarchy_cut_scratch_bytes", "gsr_hierarchy_cut", "gsr_hierarchy_cut_static",
            "gsr_hierarchy_layout", "gsr_hierarchy_build", "gsr_gather_gaussians",
            "gsr_ba_workspace_bytes", "gsr_ba_plan_create", "gsr_ba_plan_destroy", "gsr_ba_solve")


class GsrError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{status_string(status)}: {message}")
        self.status = status


class CapacityError(GsrError):
    pass


class gsr_camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("near_plane", C.c_float)]


class gsr_gaussians(C.Structure):
    _fields_ = [("n", C.c_int64), ("sh_degree", C.c_int32), ("means", C.c_void_p), ("log_scales", C.c_void_p),
                ("quats", C.c_void_p), ("opacities", C.c_void_p), ("sh", C.c_void_p)]


class gsr_gaussian_grads(C.Structure):
    _fields_ = [("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacities", C.c_void_p), ("sh", C.c_void_p)]


class gsr_launch_config(C.Structure):
    _fields_ = [("tile_h", C.c_int32), ("persistent_ctas", C.c_int32), ("stage_events", C.c_void_p),
                ("long_list_passes", C.c_int32), ("reserved0", C.c_int32), ("active_count", C.c_void_p)]


class gsr_param_set(C.Structure):
    _fields_ = [("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacities", C.c_void_p), ("sh", C.c_void_p)]


class gsr_adam_config(C.Structure):
    _fields_ = [("lr_means", C.c_float), ("lr_log_scales", C.c_float), ("lr_quats", C.c_float),
                ("lr_opacities", C.c_float), ("lr_sh_dc", C.c_float), ("lr_sh_rest", C.c_float),
                ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float), ("sparse", C.c_int32),
                ("reserved", C.c_int32 * 4)]


class gsr_stats(C.Structure):
    _fields_ = [("visible", C.c_int64), ("pairs", C.c_int64), ("evaluations", C.c_int64),
                ("contributors", C.c_int64), ("replays", C.c_int64), ("long_lists", C.c_int64),
                ("longest_list", C.c_int64)]


STAGES = ("project", "compact", "emit", "tile_sort", "composite_fwd", "composite_bwd", "project_bwd")


_lib = None


def lib():
    """The loaded library; raises if it was not built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP rasterizer library not built: {LIB_PATH} is missing "
                               "(run `python -m paper_2607_14481_amd.build`)")
        L = C.CDLL(LIB_PATH)
        vp, sz = C.c_void_p, C.c_size_t
        L.gsr_version.restype = C.c_int
        L.gsr_status_string.restype = C.c_char_p
        L.gsr_status_string.argtypes = [C.c_int]
        L.gsr_last_error.restype = C.c_char_p
        L.gsr_workspace_bytes.restype = sz
        L.gsr_workspace_bytes.argtypes = [C.c_int64, C.c_int32, C.POINTER(gsr_camera), C.c_int64,
                                          C.POINTER(gsr_launch_config)]
        L.gsr_rasterize_forward.restype = C.c_int
        L.gsr_rasterize_forward.argtypes = [vp, sz, C.POINTER(gsr_gaussians), C.c_int32, C.POINTER(gsr_camera),
                                            vp, C.POINTER(C.c_float), C.POINTER(gsr_launch_config), vp, vp,
                                            C.c_uint32, vp]
        L.gsr_rasterize_backward.restype = C.c_int
        L.gsr_rasterize_backward.argtypes = [vp, sz, C.POINTER(gsr_gaussians), C.c_int32, C.POINTER(gsr_camera),
                                             vp, C.POINTER(C.c_float), C.POINTER(gsr_launch_config), vp, vp,
                                             C.POINTER(gsr_gaussian_grads), vp, vp, C.c_uint32, vp]
        L.gsr_rasterize_backward_l1.restype = C.c_int
        L.gsr_rasterize_backward_l1.argtypes = L.gsr_rasterize_backward.argtypes
        L.gsr_rasterize_step_l1.restype = C.c_int
        L.gsr_rasterize_step_l1.argtypes = [vp, sz, C.POINTER(gsr_gaussians), C.c_int32, C.POINTER(gsr_camera),
                                            vp, C.POINTER(C.c_float), C.POINTER(gsr_launch_config), vp, vp, vp,
                                            C.POINTER(gsr_gaussian_grads), vp, vp, C.c_uint32, vp]
        L.gsr_query_pairs.restype = C.c_int
        L.gsr_query_pairs.argtypes = [vp, sz, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int32), vp]
        L.gsr_query_stats.restype = C.c_int
        L.gsr_query_stats.argtypes = [vp, sz, C.POINTER(gsr_stats), vp]
        L.gsr_export_state.restype = C.c_int
        L.gsr_export_state.argtypes = [vp, sz, C.POINTER(gsr_gaussians), C.c_int32, C.POINTER(gsr_camera),
                                       C.POINTER(gsr_launch_config), vp, vp, vp, vp, vp, vp, vp, vp]
        L.gsr_adam_step.restype = C.c_int
        L.gsr_adam_step.argtypes = [vp, sz, C.c_int64, C.c_int32, C.c_int32, C.POINTER(gsr_camera),
                                    C.POINTER(gsr_launch_config), C.POINTER(gsr_param_set),
                                    C.POINTER(gsr_gaussian_grads), C.POINTER(gsr_param_set),
                                    C.POINTER(gsr_param_set), C.c_int64, C.POINTER(gsr_adam_config), vp]
        L.gsr_pose_step.restype = C.c_int
        L.gsr_pose_step.argtypes = [vp, vp, vp, vp, C.c_int32, C.c_int64, C.c_float, C.c_float, C.c_float,
                                    C.c_float, vp]
        L.gsr_sim3_relocate.restype = C.c_int
        L.gsr_sim3_relocate.argtypes = [C.POINTER(gsr_param_set), C.c_int64, vp, vp, C.c_int32, vp]
        L.gsr_hierarchy_cut_scratch_bytes.restype = sz
        L.gsr_hierarchy_cut_scratch_bytes.argtypes = [C.c_int64]
        L.gsr_hierarchy_cut.restype = C.c_int
        L.gsr_hierarchy_cut.argtypes = [C.POINTER(gsr_gaussians), vp, vp, C.POINTER(gsr_camera), vp, C.c_float, vp,
                                        sz, vp, vp, C.POINTER(C.c_int64), vp]
        L.gsr_hierarchy_cut_static.restype = C.c_int
        L.gsr_hierarchy_cut_static.argtypes = [C.POINTER(gsr_gaussians), vp, vp, C.POINTER(gsr_camera), vp,
                                               C.c_float, vp, vp, C.POINTER(C.c_int64), vp]
        L.gsr_hierarchy_layout.restype = C.c_int
        L.gsr_hierarchy_layout.argtypes = [C.c_int64, C.c_int32, C.c_int32, vp, C.POINTER(C.c_int32)]
        L.gsr_hierarchy_build.restype = C.c_int
        L.gsr_hierarchy_build.argtypes = [C.POINTER(gsr_param_set), C.c_int32, C.c_int64, C.c_int32, C.c_int32, vp,
                                          vp, vp]
        L.gsr_gather_gaussians.restype = C.c_int
        L.gsr_gather_gaussians.argtypes = [C.POINTER(gsr_gaussians), vp, C.c_int64, vp, C.POINTER(gsr_param_set),
                                           vp]
        L.gsr_ba_workspace_bytes.restype = sz
        L.gsr_ba_workspace_bytes.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32]
        L.gsr_ba_plan_create.restype = C.c_int
        L.gsr_ba_plan_create.argtypes = [C.c_int32, vp, C.c_int32, C.c_int32, vp, vp, sz, vp, C.POINTER(vp)]
        L.gsr_ba_plan_destroy.restype = C.c_int
        L.gsr_ba_plan_destroy.argtypes = [vp]
        L.gsr_ba_solve.restype = C.c_int
        L.gsr_ba_solve.argtypes = [vp, vp, vp, C.c_double, C.c_double, vp, vp, C.c_int32, C.c_double, vp, vp]
        _lib = L
    return _lib


def version() -> int:
    return lib().gsr_version()


def status_string(status: int) -> str:
    return lib().gsr_status_string(status).decode()


def last_error() -> str:
    return lib().gsr_last_error().decode()


def _check(status: int):
    if status != GSR_OK:
        cls = CapacityError if status == GSR_ERR_CAPACITY else GsrError
        raise cls(status, last_error())


# ----------------------------------------------------------------------------
# marshalling helpers
# ----------------------------------------------------------------------------

def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _stream_ptr(stream) -> C.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def cameras(cams: Sequence) -> "C.Array[gsr_camera]":
    """Host array of gsr_camera from objects with width/height/fx/fy/cx/cy/near."""
    arr = (gsr_camera * len(cams))()
    for i, c in enumerate(cams):
        arr[i].width, arr[i].height = int(c.width), int(c.height)
        arr[i].fx, arr[i].fy, arr[i].cx, arr[i].cy = float(c.fx), float(c.fy), float(c.cx), float(c.cy)
        arr[i].near_plane = float(getattr(c, "near", 0.2))
    return arr


def launch_config(tile_h: int = 16, persistent_ctas: int = 0, long_list_passes: int = 0,
                  active_count: Optional[torch.Tensor] = None) -> gsr_launch_config:
    """active_count: None, or a one-element int64 device tensor (see
    gsr_launch_config.active_count); the caller keeps it alive."""
    cfg = gsr_launch_config()
    cfg.tile_h = int(tile_h)
    cfg.persistent_ctas = int(persistent_ctas)
    cfg.long_list_passes = int(long_list_passes)
    if active_count is not None:
        if active_count.dtype != torch.int64 or not active_count.is_cuda:
            raise TypeError("active_count must be an int64 GPU tensor")
        cfg.active_count = active_count.data_ptr()
    return cfg


LONG_LIST_RUN = 4096  # entries one workgroup sorts; longer tile lists are merged from runs of this length


def long_list_passes(longest: int) -> int:
    """Merge passes that cover a tile list of `longest` entries (0 if one workgroup sorts it)."""
    runs = -(-int(longest) // LONG_LIST_RUN)
    return 0 if runs <= 1 else (runs - 1).bit_length()


def _as_param(t: torch.Tensor, name: str) -> torch.Tensor:
    if t.dtype != torch.float32 or not t.is_cuda:
        raise TypeError(f"{name} must be a float32 GPU tensor")
    return t.contiguous()


def gaussians_struct(means, log_scales, quats, opacities, sh, sh_degree: int) -> gsr_gaussians:
    g = gsr_gaussians()
    g.n = int(means.shape[0])
    g.sh_degree = int(sh_degree)
    g.means, g.log_scales, g.quats = _ptr(means), _ptr(log_scales), _ptr(quats)
    g.opacities, g.sh = _ptr(opacities), _ptr(sh)
    return g


# ----------------------------------------------------------------------------
# entry points (same names as the C ABI, minus the prefix)
# ----------------------------------------------------------------------------

def workspace_bytes(n: int, cams: Sequence, pair_capacity: int, cfg: Optional[gsr_launch_config] = None) -> int:
    arr = cameras(cams)
    nb = lib().gsr_workspace_bytes(int(n), len(cams), arr, int(pair_capacity),
                                   C.byref(cfg) if cfg is not None else None)
    if nb == 0:
        raise GsrError(GSR_ERR_INVALID_ARGUMENT, last_error())
    return int(nb)


def rasterize_forward(ws: torch.Tensor, params: Sequence[torch.Tensor], sh_degree: int, cams: Sequence,
                      world_to_cam: torch.Tensor, bg: Sequence[float], out_rgb: torch.Tensor,
                      out_T: Optional[torch.Tensor] = None, flags: int = 0,
                      cfg: Optional[gsr_launch_config] = None, stream=None):
    g = gaussians_struct(*params, sh_degree)
    arr = cameras(cams)
    bgc = (C.c_float * 3)(*[float(x) for x in bg])
    _check(lib().gsr_rasterize_forward(_ptr(ws), ws.numel(), C.byref(g), len(cams), arr, _ptr(world_to_cam), bgc,
                                       C.byref(cfg) if cfg is not None else None, _ptr(out_rgb), _ptr(out_T),
                                       int(flags), _stream_ptr(stream)))


def rasterize_backward(ws: torch.Tensor, params: Sequence[torch.Tensor], sh_degree: int, cams: Sequence,
                       world_to_cam: torch.Tensor, bg: Sequence[float], out_rgb: torch.Tensor,
                       dL_drgb: torch.Tensor, grads: Sequence[torch.Tensor],
                       dL_dworld_to_cam: Optional[torch.Tensor] = None, dL_dtwist: Optional[torch.Tensor] = None,
                       flags: int = 0, cfg: Optional[gsr_launch_config] = None, stream=None):
    g = gaussians_struct(*params, sh_degree)
    gr = gsr_gaussian_grads()
    gr.means, gr.log_scales, gr.quats, gr.opacities, gr.sh = [_ptr(t) for t in grads]
    arr = cameras(cams)
    bgc = (C.c_float * 3)(*[float(x) for x in bg])
    _check(lib().gsr_rasterize_backward(_ptr(ws), ws.numel(), C.byref(g), len(cams), arr, _ptr(world_to_cam), bgc,
                                        C.byref(cfg) if cfg is not None else None, _ptr(out_rgb), _ptr(dL_drgb),
                                        C.byref(gr), _ptr(dL_dworld_to_cam), _ptr(dL_dtwist), int(flags),
                                        _stream_ptr(stream)))


def rasterize_backward_l1(ws: torch.Tensor, params: Sequence[torch.Tensor], sh_degree: int, cams: Sequence,
                          world_to_cam: torch.Tensor, bg: Sequence[float], out_rgb: torch.Tensor,
                          target_rgb: torch.Tensor, grads: Sequence[torch.Tensor],
                          dL_dworld_to_cam: Optional[torch.Tensor] = None, dL_dtwist: Optional[torch.Tensor] = None,
                          flags: int = 0, cfg: Optional[gsr_launch_config] = None, stream=None):
    """Backward of the mean absolute error against target_rgb (same layout as out_rgb)."""
    g = gaussians_struct(*params, sh_degree)
    gr = gsr_gaussian_grads()
    gr.means, gr.log_scales, gr.quats, gr.opacities, gr.sh = [_ptr(t) for t in grads]
    arr = cameras(cams)
    bgc = (C.c_float * 3)(*[float(x) for x in bg])
    _check(lib().gsr_rasterize_backward_l1(_ptr(ws), ws.numel(), C.byref(g), len(cams), arr, _ptr(world_to_cam),
                                           bgc, C.byref(cfg) if cfg is not None else None, _ptr(out_rgb),
                                           _ptr(target_rgb), C.byref(gr), _ptr(dL_dworld_to_cam), _ptr(dL_dtwist),
                                           int(flags), _stream_ptr(stream)))


def rasterize_step_l1(ws: torch.Tensor, params: Sequence[torch.Tensor], sh_degree: int, cams: Sequence,
                      world_to_cam: torch.Tensor, bg: Sequence[float], target_rgb: torch.Tensor,
                      out_rgb: torch.Tensor, grads: Sequence[torch.Tensor],
                      dL_dworld_to_cam: Optional[torch.Tensor] = None, dL_dtwist: Optional[torch.Tensor] = None,
                      out_T: Optional[torch.Tensor] = None, flags: int = 0,
                      cfg: Optional[gsr_launch_config] = None, stream=None):
    """Forward and the backward of the mean absolute error against target_rgb
    in one call (the compositing passes fused per tile)."""
    g = gaussians_struct(*params, sh_degree)
    gr = gsr_gaussian_grads()
    gr.means, gr.log_scales, gr.quats, gr.opacities, gr.sh = [_ptr(t) for t in grads]
    arr = cameras(cams)
    bgc = (C.c_float * 3)(*[float(x) for x in bg])
    _check(lib().gsr_rasterize_step_l1(_ptr(ws), ws.numel(), C.byref(g), len(cams), arr, _ptr(world_to_cam), bgc,
                                       C.byref(cfg) if cfg is not None else None, _ptr(target_rgb), _ptr(out_rgb),
                                       _ptr(out_T), C.byref(gr), _ptr(dL_dworld_to_cam), _ptr(dL_dtwist),
                                       int(flags), _stream_ptr(stream)))


def query_pairs(ws: torch.Tensor, stream=None):
    needed, cap, ovf = C.c_int64(), C.c_int64(), C.c_int32()
    _check(lib().gsr_query_pairs(_ptr(ws), ws.numel(), C.byref(needed), C.byref(cap), C.byref(ovf),
                                 _stream_ptr(stream)))
    return int(needed.value), int(cap.value), bool(ovf.value)


def query_stats(ws: torch.Tensor, stream=None) -> dict:
    st = gsr_stats()
    _check(lib().gsr_query_stats(_ptr(ws), ws.numel(), C.byref(st), _stream_ptr(stream)))
    return {k: int(getattr(st, k)) for k, _ in gsr_stats._fields_}


def export_state(ws: torch.Tensor, params: Sequence[torch.Tensor], sh_degree: int, cams: Sequence,
                 cfg: Optional[gsr_launch_config] = None, stream=None) -> dict:
    """Copies of the last forward's sorted pairs, ranges and per-item records."""
    needed, cap, ovf = query_pairs(ws, stream)
    m = 0 if ovf else min(needed, cap)
    n = int(params[0].shape[0])
    items = n * len(cams)
    dev = ws.device
    cfg_ = cfg if cfg is not None else launch_config()
    th = cfg_.tile_h or 16
    tiles = sum(((int(c.width) + 15) // 16) * ((int(c.height) + th - 1) // th) for c in cams)
    out = dict(
        pair_tiles=torch.zeros(max(m, 1), dtype=torch.int32, device=dev),
        pair_items=torch.zeros(max(m, 1), dtype=torch.int32, device=dev),
        ranges=torch.zeros((tiles, 2), dtype=torch.int32, device=dev),
        records=torch.zeros((max(items, 1), 12), dtype=torch.float32, device=dev),
        centre_lo=torch.zeros((max(items, 1), 2), dtype=torch.float32, device=dev),
        depth_keys=torch.zeros(max(items, 1), dtype=torch.int32, device=dev),
        tile_counts=torch.zeros(max(items, 1), dtype=torch.int32, device=dev),
    )
    g = gaussians_struct(*params, sh_degree)
    arr = cameras(cams)
    _check(lib().gsr_export_state(_ptr(ws), ws.numel(), C.byref(g), len(cams), arr, C.byref(cfg_),
                                  _ptr(out["pair_tiles"]), _ptr(out["pair_items"]), _ptr(out["ranges"]),
                                  _ptr(out["records"]), _ptr(out["centre_lo"]), _ptr(out["depth_keys"]),
                                  _ptr(out["tile_counts"]), _stream_ptr(stream)))
    torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    res["pair_tiles"] = res["pair_tiles"][:m].view("uint32")
    res["pair_items"] = res["pair_items"][:m].view("uint32")
    res["ranges"] = res["ranges"].view("uint32")
    res["depth_keys"] = res["depth_keys"][:items].view("uint32")
    res["tile_counts"] = res["tile_counts"][:items].view("uint32")
    res["records"] = res["records"][:items]
    res["centre_lo"] = res["centre_lo"][:items]
    res["M"] = m
    return res


def param_set(tensors: Sequence[torch.Tensor]) -> gsr_param_set:
    ps = gsr_param_set()
    ps.means, ps.log_scales, ps.quats, ps.opacities, ps.sh = [_ptr(t) for t in tensors]
    return ps


def adam_config(lr_means=1.6e-4, lr_log_scales=5e-3, lr_quats=1e-3, lr_opacities=5e-2, lr_sh_dc=2.5e-3,
                lr_sh_rest=2.5e-3 / 20, beta1=0.9, beta2=0.999, eps=1e-15, sparse=False) -> gsr_adam_config:
    """Defaults are the 3DGS lineage's learning rates (position rate without its decay schedule)."""
    a = gsr_adam_config()
    a.lr_means, a.lr_log_scales, a.lr_quats, a.lr_opacities = lr_means, lr_log_scales, lr_quats, lr_opacities
    a.lr_sh_dc, a.lr_sh_rest = lr_sh_dc, lr_sh_rest
    a.beta1, a.beta2, a.eps, a.sparse = beta1, beta2, eps, int(bool(sparse))
    return a


def adam_step(params: Sequence[torch.Tensor], grads: Sequence[torch.Tensor], exp_avg: Sequence[torch.Tensor],
              exp_avg_sq: Sequence[torch.Tensor], sh_degree: int, step: int, acfg: gsr_adam_config,
              ws: Optional[torch.Tensor] = None, cams: Optional[Sequence] = None,
              cfg: Optional[gsr_launch_config] = None, stream=None):
    """In-place Adam step on the five Gaussian arrays (see gsr_adam_step)."""
    gr = gsr_gaussian_grads()
    gr.means, gr.log_scales, gr.quats, gr.opacities, gr.sh = [_ptr(t) for t in grads]
    p, m, v = param_set(params), param_set(exp_avg), param_set(exp_avg_sq)
    arr = cameras(cams) if cams is not None else None
    _check(lib().gsr_adam_step(_ptr(ws), ws.numel() if ws is not None else 0, int(params[0].shape[0]),
                               int(sh_degree), len(cams) if cams is not None else 0, arr,
                               C.byref(cfg) if cfg is not None else None, C.byref(p), C.byref(gr), C.byref(m),
                               C.byref(v), int(step), C.byref(acfg), _stream_ptr(stream)))


def pose_step(world_to_cam: torch.Tensor, dL_dtwist: torch.Tensor, exp_avg: torch.Tensor,
              exp_avg_sq: torch.Tensor, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-15, stream=None):
    """In-place Adam step on the twists and SE(3) retraction of world_to_cam [V, 4, 4]."""
    _check(lib().gsr_pose_step(_ptr(world_to_cam), _ptr(dL_dtwist), _ptr(exp_avg), _ptr(exp_avg_sq),
                               int(world_to_cam.shape[0]), int(step), float(lr), float(beta1), float(beta2),
                               float(eps), _stream_ptr(stream)))


def sim3_relocate(params: Sequence[torch.Tensor], keyframe_of: torch.Tensor, sim3: torch.Tensor, stream=None):
    """In-place Sim(3) relocation: sim3 [K, 8] = (s, qw, qx, qy, qz, tx, ty, tz); keyframe_of [n] int32."""
    if keyframe_of.dtype != torch.int32 or sim3.dtype != torch.float32:
        raise TypeError("keyframe_of must be int32 and sim3 float32")
    _check(lib().gsr_sim3_relocate(C.byref(param_set(params)), int(params[0].shape[0]), _ptr(keyframe_of),
                                   _ptr(sim3), int(sim3.shape[0]), _stream_ptr(stream)))


def _cut_args(nodes, parent, child_count, scratch, out):
    n = int(nodes[0].shape[0])
    if parent.dtype != torch.int32 or child_count.dtype != torch.int32:
        raise TypeError("parent and child_count must be int32")
    need = int(lib().gsr_hierarchy_cut_scratch_bytes(n))
    if scratch is None or scratch.numel() < need:
        scratch = torch.empty(max(need, 1), dtype=torch.uint8, device=nodes[0].device)
    if out is None or out.numel() < n:
        out = torch.empty(max(n, 1), dtype=torch.int32, device=nodes[0].device)
    return scratch, out


def hierarchy_cut(nodes: Sequence[torch.Tensor], sh_degree: int, parent: torch.Tensor, child_count: torch.Tensor,
                  cam, world_to_cam: torch.Tensor, tau: float = 1.5, scratch: Optional[torch.Tensor] = None,
                  out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Node indices (int32, ascending) of the per-view cut; see
    gsr_hierarchy_cut.  Blocking: the size is read back to the host."""
    scratch, out = _cut_args(nodes, parent, child_count, scratch, out)
    g = gaussians_struct(*nodes, sh_degree)
    arr = cameras([cam])
    n_cut = C.c_int64()
    _check(lib().gsr_hierarchy_cut(C.byref(g), _ptr(parent), _ptr(child_count), arr, _ptr(world_to_cam), float(tau),
                                   _ptr(scratch), scratch.numel(), _ptr(out), None, C.byref(n_cut),
                                   _stream_ptr(stream)))
    return out[:n_cut.value]


def hierarchy_cut_async(nodes: Sequence[torch.Tensor], sh_degree: int, parent: torch.Tensor,
                        child_count: torch.Tensor, cam, world_to_cam: torch.Tensor, tau: float,
                        scratch: torch.Tensor, out: torch.Tensor, count: torch.Tensor, stream=None) -> None:
    """The cut without a host round trip: node indices into out[:count] and
    their number into the int64 device tensor `count`, enqueued on the stream
    (capturable in a graph)."""
    if count.dtype != torch.int64 or not count.is_cuda:
        raise TypeError("count must be an int64 GPU tensor")
    scratch, out2 = _cut_args(nodes, parent, child_count, scratch, out)
    if out2 is not out:
        raise ValueError("out must hold one index per node")
    g = gaussians_struct(*nodes, sh_degree)
    arr = cameras([cam])
    _check(lib().gsr_hierarchy_cut(C.byref(g), _ptr(parent), _ptr(child_count), arr, _ptr(world_to_cam), float(tau),
                                   _ptr(scratch), scratch.numel(), _ptr(out), _ptr(count), None,
                                   _stream_ptr(stream)))


GSR_MAX_HIERARCHY_LEVELS = 30


def hierarchy_layout(n_leaves: int, levels: int, branching: int = 8):
    """First node of every level (leaves = level 0) and, last, the node count;
    see gsr_hierarchy_layout (host only)."""
    import numpy as np
    ls = np.zeros(GSR_MAX_HIERARCHY_LEVELS + 2, np.int64)
    nl = C.c_int32()
    _check(lib().gsr_hierarchy_layout(int(n_leaves), int(levels), int(branching),
                                      C.c_void_p(ls.ctypes.data), C.byref(nl)))
    return ls[:nl.value + 1].copy()


def hierarchy_build(nodes: Sequence[torch.Tensor], sh_degree: int, n_leaves: int, levels: int, branching: int = 8,
                    parent: Optional[torch.Tensor] = None, child_count: Optional[torch.Tensor] = None, stream=None):
    """Builds the inner nodes of a hierarchy in place (see gsr_hierarchy_build):
    `nodes` hold every node (leaves first, in their grouping order).  Returns
    (parent, child_count) int32 device tensors."""
    n = int(nodes[0].shape[0])
    ls = hierarchy_layout(n_leaves, levels, branching)
    if n < int(ls[-1]):
        raise ValueError(f"node arrays hold {n} rows, the hierarchy has {int(ls[-1])} nodes")
    dev = nodes[0].device
    if parent is None:
        parent = torch.empty(n, dtype=torch.int32, device=dev)
    if child_count is None:
        child_count = torch.empty(n, dtype=torch.int32, device=dev)
    _check(lib().gsr_hierarchy_build(C.byref(param_set(nodes)), int(sh_degree), int(n_leaves), int(levels),
                                     int(branching), _ptr(parent), _ptr(child_count), _stream_ptr(stream)))
    return parent, child_count


HIERARCHY_CUT_STATIC_MAX_NODES = 1 << 23  # the scratch-free cut's limit (gsr_hierarchy_cut_static)


def hierarchy_cut_static(nodes: Sequence[torch.Tensor], sh_degree: int, parent: torch.Tensor,
                         child_count: torch.Tensor, cam, world_to_cam: torch.Tensor, tau: float,
                         out: torch.Tensor, count: Optional[torch.Tensor] = None, stream=None) -> Optional[int]:
    """The cut through gsr_hierarchy_cut_static (no scratch argument, nothing
    allocated by the library): node indices into `out` (one int32 per node,
    caller-allocated).  With `count` (int64 device tensor) the size goes there
    and nothing is read back (returns None); without it the call blocks and
    returns the size."""
    n = int(nodes[0].shape[0])
    if parent.dtype != torch.int32 or child_count.dtype != torch.int32:
        raise TypeError("parent and child_count must be int32")
    if out.dtype != torch.int32 or out.numel() < n:
        raise ValueError("out must be an int32 tensor with one entry per node")
    if count is not None and (count.dtype != torch.int64 or not count.is_cuda):
        raise TypeError("count must be an int64 GPU tensor")
    g = gaussians_struct(*nodes, sh_degree)
    arr = cameras([cam])
    n_cut = C.c_int64()
    _check(lib().gsr_hierarchy_cut_static(C.byref(g), _ptr(parent), _ptr(child_count), arr, _ptr(world_to_cam),
                                          float(tau), _ptr(out), _ptr(count),
                                          None if count is not None else C.byref(n_cut), _stream_ptr(stream)))
    return None if count is not None else int(n_cut.value)


def gather_gaussians(src: Sequence[torch.Tensor], sh_degree: int, index: torch.Tensor, stream=None,
                     count: Optional[torch.Tensor] = None, dst: Optional[Sequence[torch.Tensor]] = None):
    """Rows `index` of the five arrays in contiguous tensors (new ones unless
    `dst` is given).  count: None, or an int64 device tensor: only the first
    min(count, len(index)) rows are copied (see gsr_gather_gaussians)."""
    m = int(index.numel())
    if dst is None:
        dst = [torch.empty((m,) + tuple(t.shape[1:]), dtype=t.dtype, device=t.device) for t in src]
    elif any(int(t.shape[0]) < m for t in dst):
        raise ValueError("dst arrays must hold len(index) rows")
    if count is not None and (count.dtype != torch.int64 or not count.is_cuda):
        raise TypeError("count must be an int64 GPU tensor")
    g = gaussians_struct(*src, sh_degree)
    _check(lib().gsr_gather_gaussians(C.byref(g), _ptr(index), m, _ptr(count), C.byref(param_set(dst)),
                                      _stream_ptr(stream)))
    return dst


# ----------------------------------------------------------------------------
# local bundle adjustment
# ----------------------------------------------------------------------------

def ba_workspace_bytes(n_cams: int, n_free: int, n_landmarks: int, max_obs: int) -> int:
    n = lib().gsr_ba_workspace_bytes(n_cams, n_free, n_landmarks, max_obs)
    if n == 0:
        raise GsrError(GSR_ERR_INVALID_ARGUMENT, last_error())
    return n


class BAPlan:
    """The structure of one bundle-adjustment problem (which keyframes are
    free, which keyframes see which landmark) uploaded into a device
    workspace this object owns.  free_slot: int32 [n_cams]; obs_cam: int32
    [n_landmarks, max_obs] (host arrays or CPU tensors)."""

    def __init__(self, free_slot, obs_cam, device="cuda", stream=None):
        fs = torch.as_tensor(free_slot, dtype=torch.int32).contiguous().cpu()
        oc = torch.as_tensor(obs_cam, dtype=torch.int32).contiguous().cpu()
        if oc.dim() != 2:
            raise ValueError("obs_cam must be [n_landmarks, max_obs]")
        self.n_cams, (self.n_landmarks, self.max_obs) = int(fs.numel()), oc.shape
        self.n_free = int((fs >= 0).sum())
        nbytes = ba_workspace_bytes(self.n_cams, self.n_free, self.n_landmarks, self.max_obs)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        handle = C.c_void_p()
        _check(lib().gsr_ba_plan_create(self.n_cams, _ptr(fs), self.n_landmarks, self.max_obs, _ptr(oc),
                                        _ptr(self.ws), nbytes, _stream_ptr(stream), C.byref(handle)))
        self._handle = handle

    def __del__(self):
        h = getattr(self, "_handle", None)
        if h is not None and _lib is not None:
            _lib.gsr_ba_plan_destroy(h)
            self._handle = None


def ba_solve(plan: BAPlan, poses: torch.Tensor, focal: torch.Tensor, principal, landmarks: torch.Tensor,
             obs_uv: torch.Tensor, iterations: int, lam: float, costs: Optional[torch.Tensor] = None, stream=None):
    """`iterations` damped Gauss-Newton steps on the device tensors (float64,
    contiguous, updated in place): poses [n_cams, 3, 4], focal [1],
    landmarks [n_landmarks, 3]; obs_uv [n_landmarks, max_obs, 2]; costs
    (optional) [iterations + 1] receives the cost before each step and after
    the last."""
    for name, t, shape in (("poses", poses, (plan.n_cams, 3, 4)), ("focal", focal, (1,)),
                           ("landmarks", landmarks, (plan.n_landmarks, 3)),
                           ("obs_uv", obs_uv, (plan.n_landmarks, plan.max_obs, 2))):
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != shape:
            raise ValueError(f"{name} must be a contiguous float64 device tensor of shape {shape}")
    if costs is not None and (costs.dtype != torch.float64 or not costs.is_cuda or costs.numel() < iterations + 1):
        raise ValueError("costs must be a float64 device tensor of at least iterations + 1 entries")
    _check(lib().gsr_ba_solve(plan._handle, _ptr(poses), _ptr(focal), float(principal[0]), float(principal[1]),
                              _ptr(landmarks), _ptr(obs_uv), int(iterations), float(lam), _ptr(costs),
                              _stream_ptr(stream)))
