"""Request loop: render and optimise requests against a growing Gaussian scene.

Live capture in the paper optimises the Gaussians asynchronously until the next
keyframe arrives, while new Gaussians are spawned per keyframe (Sec. 5.2) and
the scene must stay viewable (Sec. 7.2).  This module serves that mixture:

* the scene lives in capacity-sized device buffers; a keyframe appends
  Gaussians at the end, so every scene version is a prefix and a request bound
  to version N reads the first N Gaussians whatever is appended later;
* requests arrive by a Poisson process: "render" (forward of one view) and
  "optimise" (forward + L1 loss + backward over 1-4 views, returning the
  parameter and pose gradients);
* continuous batching: up to `slots` calls are in flight on their own streams,
  so their kernels overlap on the device; pending render requests are grouped
  into one multi-view call; a request is admitted only when a slot is free and
  the device memory it needs fits the HBM budget, otherwise it waits;
* every slot keeps its workspace resident and only grows it;
* the forward runs without host synchronisation; an overflowing pair capacity
  is detected on completion and the request is run again with room to spare.

Every request's result depends only on its own inputs (the rasterizer is
deterministic and calls do not share state), so a request's output is the same
alone and in the mix; `tests/test_gpu_serve.py` checks exactly that.
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np
import torch

from . import gsr
from . import scenes as S
from .rasterizer import GaussianRasterizer, PARAM_NAMES


# ----------------------------------------------------------------------------
# workload generation
# ----------------------------------------------------------------------------

@dataclass
class Request:
    rid: int
    t_arrival: float           # seconds from the start of the run
    kind: str                  # "render" or "optimise"
    cams: List[S.Camera]
    target_seed: int = 0
    version: int = 0           # scene prefix length the request is bound to
    # filled by the server
    t_admit: float = float("nan")
    t_done: float = float("nan")
    retries: int = 0
    call_views: int = 0        # views of the call that served it (renders may be grouped)
    result: Optional[dict] = None

    @property
    def pixels(self) -> int:
        return sum(c.width * c.height for c in self.cams)


def sphere_camera(rng, radius=30.0, wmin=256, wmax=1920, hmin=256, hmax=1080) -> S.Camera:
    d = rng.standard_normal(3)
    d /= np.linalg.norm(d)
    w = int(rng.integers(wmin, wmax + 1))
    h = int(rng.integers(hmin, hmax + 1))
    return S.pinhole(w, h, S.look_at(d * radius))


def make_requests(seed: int, rate: float, duration: float, render_frac: float = 0.5,
                  max_opt_views: int = 4, radius: float = 30.0) -> List[Request]:
    """Poisson arrivals (seeded exponential gaps) of render / optimise requests;
    resolutions uniform over 256x256..1920x1080, cameras on a sphere looking
    at the scene centre, optimise requests over 1..4 such views."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out, t, rid = [], 0.0, 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        kind = "render" if rng.uniform() < render_frac else "optimise"
        nv = 1 if kind == "render" else int(rng.integers(1, max_opt_views + 1))
        cams = [sphere_camera(rng, radius) for _ in range(nv)]
        out.append(Request(rid, t, kind, cams, target_seed=int(rng.integers(0, 2**31 - 1))))
        rid += 1
    return out


# ----------------------------------------------------------------------------
# resident growing scene
# ----------------------------------------------------------------------------

class GrowingScene:
    """Gaussian parameters in capacity-sized device buffers; keyframes append.

    Keyframe k appends `per_keyframe` Gaussians drawn from the 20 m box recipe
    with seed base_seed + k, so the scene at any version is reproducible."""

    def __init__(self, capacity: int, start: int, per_keyframe: int, sh_degree: int = 3, base_seed: int = 50,
                 half: float = 10.0, device="cuda"):
        self.capacity = int(capacity)
        self.per_keyframe = int(per_keyframe)
        self.sh_degree = int(sh_degree)
        self.base_seed = int(base_seed)
        self.half = half
        self.device = torch.device(device)
        K = (sh_degree + 1) ** 2
        shapes = dict(means=(3,), log_scales=(3,), quats=(4,), opacities=(), sh=(K, 3))
        self.bufs = {k: torch.zeros((self.capacity,) + shp, dtype=torch.float32, device=self.device)
                     for k, shp in shapes.items()}
        self.n = 0
        self.keyframes = 0
        self.start = int(start)
        self._append(self._draw(base_seed - 1, start))

    def _draw(self, seed: int, count: int) -> S.Scene:
        rng = np.random.Generator(np.random.PCG64(seed))
        means = rng.uniform(-self.half, self.half, (count, 3))
        return S._gaussian_body(rng, means, self.sh_degree)

    def _append(self, sc: S.Scene):
        m = sc.n
        if self.n + m > self.capacity:
            raise RuntimeError("scene capacity exhausted")
        for k in PARAM_NAMES:
            self.bufs[k][self.n:self.n + m].copy_(torch.from_numpy(np.asarray(getattr(sc, k), np.float32)),
                                                  non_blocking=False)
        self.n += m

    def add_keyframe(self):
        self._append(self._draw(self.base_seed + self.keyframes, self.per_keyframe))
        self.keyframes += 1

    def version_at(self, t: float, start: int, period: float) -> int:
        return min(self.capacity, start + self.per_keyframe * int(math.floor(t / period)))

    def params(self, version: int):
        return [self.bufs[k][:version] for k in PARAM_NAMES]

    def host_scene(self, version: int) -> S.Scene:
        """The first `version` Gaussians, drawn again on the host from the
        same seeds (for checks against a reference renderer)."""
        parts = [self._draw(self.base_seed - 1, self.start)]
        k = 0
        while sum(p.n for p in parts) < version:
            parts.append(self._draw(self.base_seed + k, self.per_keyframe))
            k += 1
        cat = {f: np.concatenate([np.asarray(getattr(p, f)) for p in parts])[:version] for f in PARAM_NAMES}
        return S.Scene(sh_degree=self.sh_degree, **cat)


# ----------------------------------------------------------------------------
# the server
# ----------------------------------------------------------------------------

PX_REF = 1920 * 1080

@dataclass
class Job:
    reqs: List[Request]
    stream: torch.cuda.Stream
    slot: int
    done: torch.cuda.Event
    rast: GaussianRasterizer
    ws: torch.Tensor
    rgb: torch.Tensor
    grads: Optional[list] = None
    pose_grad: Optional[torch.Tensor] = None
    upstream: Optional[torch.Tensor] = None
    bytes: int = 0


class Server:
    def __init__(self, scene: GrowingScene, slots: int = 4, group_renders: bool = True, max_group_views: int = 8,
                 hbm_budget: Optional[int] = None, keep_results: bool = False, pair_rate: float = 1.0,
                 safety: float = 1.5, tile_h: int = 16, loss: str = "l1"):
        """loss: "l1" (mean absolute error against the request's seeded
        U(0, 1) target, its image gradient formed inside the backward) or
        "upstream" (the backward takes a seeded N(0, 1) image gradient
        directly: every output is then a fixed function of the request's
        inputs, which is what a reference comparison needs)."""
        if loss not in ("l1", "upstream"):
            raise ValueError(f"loss {loss!r}")
        self.loss = loss
        self.scene = scene
        self.slots = max(1, int(slots))
        self.group = bool(group_renders)
        self.max_group_views = int(max_group_views)
        self.keep = bool(keep_results)
        self.safety = float(safety)
        self.tile_h = int(tile_h)
        # pairs per Gaussian and per unit of view weight (largest seen so far):
        # sizes the pair capacity
        self.pair_rate = float(pair_rate)
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info()
            hbm_budget = int(free * 0.8)
        self.hbm_budget = int(hbm_budget)
        self.streams = [torch.cuda.Stream() for _ in range(self.slots)]
        self.slot_ws: List[Optional[torch.Tensor]] = [None] * self.slots
        # admission accounting: every slot's resident workspace counts, busy
        # or idle, plus the outputs of the calls in flight
        self.resident_ws_bytes = 0
        self.in_flight_bytes = 0   # outputs (images, gradients) of the calls in flight
        self.peak_bytes = 0
        self.peak_bytes_shared = 0  # peak while two or more calls were in flight
        self.peak_allocated = 0     # measured: allocator peak above the start of the last run

    # -- sizing --------------------------------------------------------------
    @staticmethod
    def _view_weight(cams) -> float:
        """Pair count model: a Gaussian covers at least one tile of a view it
        sees, and its tile span grows with the view's resolution (focal length
        = width), so M ~ n * sum_v (1 + pixels_v / 1080p).  A model
        proportional to pixels alone, learned on small views, overestimates
        large ones many times over."""
        return sum(1.0 + c.width * c.height / PX_REF for c in cams)

    def _capacity(self, n: int, cams) -> int:
        return int(self.pair_rate * n * self._view_weight(cams) * self.safety) + 4096

    def _estimate(self, reqs: List[Request]):
        """(pair capacity, workspace bytes, bytes of the call's outputs):
        images, plus for an optimise call its target or upstream image, the
        parameter gradients and the pose gradients."""
        cams = [c for r in reqs for c in r.cams]
        n = max(r.version for r in reqs)
        cap = self._capacity(n, cams)
        ws_bytes = gsr.workspace_bytes(n, cams, cap, gsr.launch_config(self.tile_h))
        px = sum(c.width * c.height for c in cams)
        out = 3 * px * 4 * (2 if reqs[0].kind == "optimise" else 1)
        grads = (n * 4 * (11 + 3 * (self.scene.sh_degree + 1) ** 2) + 88 * len(cams)
                 if reqs[0].kind == "optimise" else 0)
        return cap, ws_bytes, out + grads

    def _slot_growth(self, slot: int, ws_bytes: int) -> int:
        """Bytes the slot's resident workspace would grow by for ws_bytes."""
        ws = self.slot_ws[slot]
        have = 0 if ws is None else ws.numel()
        return 0 if have >= ws_bytes else int(ws_bytes * 1.25) - have

    def _device_bytes(self) -> int:
        return self.resident_ws_bytes + self.in_flight_bytes

    # -- launching -----------------------------------------------------------
    def _launch(self, reqs: List[Request], slot: int, cap: int, ws_bytes: int, est: int) -> Job:
        cams = [c for r in reqs for c in r.cams]
        n = reqs[0].version
        for r in reqs:
            r.call_views = len(cams)
        st = self.streams[slot]
        with torch.cuda.stream(st):
            ws = self.slot_ws[slot]
            if ws is None or ws.numel() < ws_bytes:
                if ws is not None:
                    self.resident_ws_bytes -= ws.numel()
                self.slot_ws[slot] = None
                del ws
                ws = torch.empty(int(ws_bytes * 1.25), dtype=torch.uint8, device=self.scene.device)
                self.slot_ws[slot] = ws
                self.resident_ws_bytes += ws.numel()
            rast = GaussianRasterizer(cams, self.scene.sh_degree, tile_h=self.tile_h, sync=False,
                                      device=self.scene.device)
            params = self.scene.params(n)
            w2c = torch.tensor(np.stack([np.asarray(c.world_to_cam, np.float32) for c in cams]),
                               device=self.scene.device)
            if reqs[0].kind == "optimise" and self.loss == "l1":
                # forward, L1 against the request's target and backward in one call
                target = self._target(reqs[0], 3 * rast.total_pixels)
                rgb, _, grads, pose_grad, _ = rast.step_l1(params, w2c, (0.0, 0.0, 0.0), target, ws=ws)
                job = Job(reqs, st, slot, torch.cuda.Event(), rast, ws, rgb, bytes=est)
                job.grads, job.pose_grad = grads, pose_grad
            else:
                rgb, _ = rast.forward(params, w2c, (0.0, 0.0, 0.0), ws=ws)
                job = Job(reqs, st, slot, torch.cuda.Event(), rast, ws, rgb, bytes=est)
                if reqs[0].kind == "optimise":
                    job.upstream = self._upstream(reqs[0], rgb.numel())
                    job.grads, job.pose_grad, _ = rast.backward(ws, params, w2c, (0.0, 0.0, 0.0), rgb,
                                                                job.upstream)
            job.done.record(st)
        return job

    def _target(self, req: Request, numel: int) -> torch.Tensor:
        g = torch.Generator(device=self.scene.device)
        g.manual_seed(req.target_seed)
        return torch.rand(numel, generator=g, device=self.scene.device)

    def _upstream(self, req: Request, numel: int) -> torch.Tensor:
        g = torch.Generator(device=self.scene.device)
        g.manual_seed(req.target_seed)
        return torch.randn(numel, generator=g, device=self.scene.device)

    # -- the loop ------------------------------------------------------------
    def run(self, requests: List[Request], keyframe_period: float = 0.5, start_n: Optional[int] = None,
            bind_versions: bool = True, time_scale: float = 1.0) -> dict:
        """Serves `requests` in (scaled) wall-clock time; returns latency stats.

        bind_versions: each request reads the scene version of its arrival
        time (keyframes every `keyframe_period` seconds), independent of when
        it is admitted; False keeps the versions the requests already carry."""
        start_n = self.scene.n if start_n is None else start_n
        reqs = sorted(requests, key=lambda r: r.t_arrival)
        if bind_versions:
            for r in reqs:
                r.version = self.scene.version_at(r.t_arrival, start_n, keyframe_period)
        pending = collections.deque()
        retry = collections.deque()
        in_flight: Dict[int, Job] = {}
        torch.cuda.synchronize(self.scene.device)
        base_alloc = torch.cuda.memory_allocated(self.scene.device)
        torch.cuda.reset_peak_memory_stats(self.scene.device)
        free_slots = list(range(self.slots))
        nxt = 0
        done = 0
        t0 = time.perf_counter()
        clock = lambda: (time.perf_counter() - t0) * time_scale
        kf_due = keyframe_period
        while done < len(reqs):
            now = clock()
            # keyframes: the scene grows on schedule (appends never touch what requests read)
            while now >= kf_due:
                if self.scene.n + self.scene.per_keyframe <= self.scene.capacity:
                    self.scene.add_keyframe()
                kf_due += keyframe_period
            while nxt < len(reqs) and reqs[nxt].t_arrival <= now:
                pending.append(reqs[nxt])
                nxt += 1
            # completions
            for slot in list(in_flight):
                job = in_flight[slot]
                if not job.done.query():
                    continue
                tdone = clock()
                del in_flight[slot]
                free_slots.append(slot)
                needed, cap, ovf = gsr.query_pairs(job.ws, job.stream)
                w = self._view_weight([c for r in job.reqs for c in r.cams])
                self.pair_rate = max(self.pair_rate, needed / max(1.0, job.reqs[0].version * w))
                if ovf:
                    self.in_flight_bytes -= job.bytes
                    for r in job.reqs:
                        r.retries += 1
                        retry.append(r)
                    del job
                    continue
                self._finish(job, tdone)
                self.in_flight_bytes -= job.bytes
                done += len(job.reqs)
                del job  # its outputs go back to the allocator now, not at the next completion
            # admissions
            while free_slots and (retry or pending):
                src = retry if retry else pending
                head = src[0]
                group = [head]
                if self.group and head.kind == "render":
                    # gather more pending renders of the same scene version into one call
                    views = len(head.cams)
                    for r in list(src)[1:]:
                        if views >= self.max_group_views:
                            break
                        if r.kind == "render" and r.version == head.version:
                            group.append(r)
                            views += len(r.cams)
                cap, ws_bytes, est = self._estimate(group)
                # the slot whose resident workspace needs the least growth
                slot = min(free_slots, key=lambda k: (self._slot_growth(k, ws_bytes), k))
                need = self._slot_growth(slot, ws_bytes) + est
                if self._device_bytes() + need > self.hbm_budget:
                    # idle slots give back their workspaces first
                    for k in free_slots:
                        if k != slot and self.slot_ws[k] is not None:
                            self.resident_ws_bytes -= self.slot_ws[k].numel()
                            self.slot_ws[k] = None
                    if self._device_bytes() + need > self.hbm_budget and in_flight:
                        break  # wait for memory to free up (a call larger than the budget runs alone)
                for r in group:
                    src.remove(r)
                    r.t_admit = clock()
                free_slots.remove(slot)
                self.in_flight_bytes += est
                in_flight[slot] = self._launch(group, slot, cap, ws_bytes, est)
                self.peak_bytes = max(self.peak_bytes, self._device_bytes())
                if len(in_flight) > 1:
                    self.peak_bytes_shared = max(self.peak_bytes_shared, self._device_bytes())
            if not in_flight and not pending and not retry and nxt < len(reqs):
                wait = (reqs[nxt].t_arrival - clock()) / time_scale
                if wait > 0:
                    time.sleep(min(wait, 0.002))
            elif in_flight:
                time.sleep(0.00005)
        wall = clock()
        torch.cuda.synchronize(self.scene.device)
        self.peak_allocated = torch.cuda.max_memory_allocated(self.scene.device) - base_alloc
        return self._summary(reqs, wall)

    def _finish(self, job: Job, tdone: float):
        """Results of a completed call.  The copies run on the call's own
        stream, where its outputs were allocated: once the job is dropped the
        allocator may hand those blocks to the slot's next call, which that
        stream orders after the copies."""
        off = 0
        with torch.cuda.stream(job.stream):
            for r in job.reqs:
                r.t_done = tdone
                if self.keep:
                    res = {}
                    views = []
                    for c in r.cams:
                        k = 3 * c.width * c.height
                        views.append(job.rgb[off:off + k].detach().clone())
                        off += k
                    res["rgb"] = views
                    if job.grads is not None:
                        res["grads"] = [g.detach().clone() for g in job.grads]
                        res["pose_grad"] = job.pose_grad.detach().clone()
                    if job.upstream is not None:
                        res["upstream"] = job.upstream.detach().clone()
                    r.result = res
                else:
                    off += sum(3 * c.width * c.height for c in r.cams)
            if self.keep:
                job.stream.synchronize()

    def _summary(self, reqs: List[Request], wall: float) -> dict:
        lat = np.array([r.t_done - r.t_arrival for r in reqs]) * 1e3
        px_g = sum(r.pixels * r.version for r in reqs)
        by_kind = {}
        for kind in ("render", "optimise"):
            l = np.array([r.t_done - r.t_arrival for r in reqs if r.kind == kind]) * 1e3
            if len(l):
                by_kind[kind] = {"n": int(len(l)), "p50_ms": float(np.percentile(l, 50)),
                                 "p99_ms": float(np.percentile(l, 99))}
        return {
            "requests": len(reqs),
            "wall_s": wall,
            "throughput_req_s": len(reqs) / wall,
            "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)),
            "p999_ms": float(np.percentile(lat, 99.9)),
            "mean_ms": float(lat.mean()),
            "pixel_gaussians_per_s": px_g / wall,
            "retries": int(sum(r.retries for r in reqs)),
            "peak_inflight_bytes": int(self.peak_bytes),
            "peak_allocated_bytes": int(self.peak_allocated),
            "peak_shared_inflight_bytes": int(self.peak_bytes_shared),
            "hbm_budget": int(self.hbm_budget),
            "by_kind": by_kind,
            "slots": self.slots,
            "grouped_renders": self.group,
            "final_gaussians": self.scene.n,
        }
