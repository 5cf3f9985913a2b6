#!/usr/bin/env python
"""Benchmark of the differentiable Gaussian-splat rasterizer on one MI355X.

One step = one optimisation iteration of the joint Gaussian/pose optimisation
(the paper runs 30 of them per keyframe): forward rasterization of the view,
L1 loss against a target image, backward to every Gaussian parameter and to the
6-DoF camera pose.  No optimiser update.  Inputs are resident in HBM before the
timed region starts.

Default workload: the first 1920x1080 camera of the 8-camera ring (radius 15 m)
around 1,000,000 Gaussians in a 20 m box, SH degree 3; the target is rendered
from that pose perturbed by 0.5 degrees and 2 cm.

Prints ONE JSON line.  `value` is iterations/s of the plain form (one view per
launch sequence, no host synchronisation in the timed steps: synchronous
warm-up steps size the pair capacity).  Also reported: the same step captured
in a HIP graph, per-stage times from
HIP events recorded inside the timed region, the roofline of the dominant
kernel, and the FP64 CPU oracle timed on this host.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Published MI355X peaks (per GPU).
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3

# Algorithmic FP32 operations of the compositing definition, per unit (see the
# design notes): every list entry a pixel evaluates costs the offset, the
# quadratic form, the exponential and the opacity product (13); every Gaussian
# actually composited adds transmittance and colour updates (9).  The backward
# replays each position up to the pixel's last contributor (13) and, per
# contributor, forms the colour, alpha, sigma, conic and centre gradients (34).
FLOPS_FWD_EVAL, FLOPS_FWD_CONTRIB = 13, 9
FLOPS_BWD_EVAL, FLOPS_BWD_CONTRIB = 13, 34

# Plain copy used to calibrate the HBM byte counters: every dispatch reads and
# writes exactly this many bytes.
COPY_CAL_MIB, COPY_CAL_REPS = 384, 4


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(workload, kernel):
    """HBM bytes per dispatch of `kernel` from the committed byte-counter
    profile, if it covers this workload and the kernel sources it was taken on
    are the current ones (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{TRAFFIC_PROFILES.get(workload, '-')}_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    info = None
    for line in open(path):
        if line.startswith("traffic-json: "):
            info = json.loads(line[len("traffic-json: "):])
    if info is None or kernel not in info["kernel"]:
        return None
    h = hashlib.sha256()
    for f in info["sources"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest() != info["sources_sha256"]:
        return None
    return {"bytes": int(info["read_bytes"] + info["write_bytes"]),
            "note": f"FETCH_SIZE/{info['fetch_factor']} + WRITE_SIZE/{info['write_factor']} per dispatch "
                    f"({info['read_bytes'] / 1e6:.1f} MB read, {info['write_bytes'] / 1e6:.1f} MB written), "
                    f"from profiles/{os.path.basename(path)}"}


TRAFFIC_PROFILES = {"headline": "headline_1080p_1M"}
OTHER_WORKLOADS = ("small_view", "single_view_1080p", "lod_cut")


def host_cpu():
    """Logical CPUs this process may use and the host CPU's model name."""
    import subprocess
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        nproc = os.cpu_count()
    model = None
    try:
        for line in subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except Exception:  # pragma: no cover - reported as unknown
        pass
    return {"nproc": nproc, "model": model}


def _oracle_tile_share(rank, procs, ready, start, results):
    """One process of the all-core oracle timing: the unmodified oracle's
    fwd + bwd of the headline view restricted to one band of tile rows (its
    tile mask: those tiles' lists and pixels are the full render's, and the
    oracle drops the Gaussians that touch none of them).  Rendering starts
    when every process is ready."""
    import numpy as np
    from oracle import oracle as O
    wl, _ = make_workload("headline")
    sc, cam = wl.scene, wl.cameras[0]
    tx, ty = O.tile_grid(cam)
    row = np.arange(tx * ty) // tx
    mask = ((row * procs) // ty == rank).astype(np.uint8)
    rng = np.random.default_rng(0)
    shape = (cam.height, cam.width, 3)
    g = np.sign(rng.standard_normal(shape)) / float(np.prod(shape))  # L1-shaped upstream
    ready.put(rank)
    start.wait()
    t = time.time()
    O.render(sc, cam, bg=(0.0, 0.0, 0.0), tile_mask=mask, dL_dimg=g)
    results.put((rank, time.time() - t, time.time()))


def oracle_all_cores(procs, timeout=300.0):
    """Wall time of one headline fwd + bwd of the oracle split by tiles over
    `procs` fresh processes (spawned: no GPU state), from the moment all are
    ready to the last one's end.  Each process also projects and bins every
    Gaussian, the part a tile split does not divide.  Raises if a process
    ends early or the run exceeds `timeout` seconds."""
    import multiprocessing as mp
    import queue as q
    ctx = mp.get_context("spawn")
    ready, results, start = ctx.Queue(), ctx.Queue(), ctx.Event()
    ps = [ctx.Process(target=_oracle_tile_share, args=(r, procs, ready, start, results)) for r in range(procs)]
    for p in ps:
        p.start()

    def collect(src, n, deadline):
        out = []
        while len(out) < n:
            try:
                out.append(src.get(timeout=1.0))
            except q.Empty:
                if any(p.exitcode not in (None, 0) for p in ps):
                    raise RuntimeError("an oracle process ended early")
                if time.time() > deadline:
                    raise RuntimeError("oracle processes timed out")
        return out

    try:
        deadline = time.time() + timeout
        collect(ready, procs, deadline)
        t0 = time.time()
        start.set()
        res = collect(results, procs, deadline)
    finally:
        for p in ps:
            p.join(timeout=30)
            if p.is_alive():
                p.terminate()
    return max(r[2] for r in res) - t0, sorted(r[1] for r in res)


def make_workload(name):
    from paper_2607_14481_amd import scenes as S
    if name == "headline":
        wl = S.headline_view()
        desc = ("first 1920x1080 view of an 8-camera ring (r = 15 m) around 1,000,000 Gaussians "
                "in a 20 m box, SH degree 3; L1 loss vs a render from the pose perturbed by 0.5 deg / 2 cm; "
                "fwd + bwd incl. 6-DoF pose gradient")
    elif name == "single_view_1080p":
        wl = S.single_view_1080p()
        desc = ("single 1920x1080 view, 200,000 Gaussians in a 20 m box, SH degree 3, camera 40 m away; "
                "L1 loss vs a render from the pose perturbed by 0.5 deg / 2 cm; fwd + bwd incl. pose gradient")
    elif name == "small_view":
        wl = S.small_view()
        desc = "128x128 view, 1,000 Gaussians, SH degree 0; L1 loss vs a render of jittered means"
    elif name == "lod_cut":
        from paper_2607_14481_amd import hierarchy
        wl = hierarchy.lod_workload()
        desc = ("level-of-detail cut: 4,000,000 leaves along a 2 km street in a 7-level branching-8 hierarchy "
                "(moment-matched merges), 1.5 px screen-size cut for one 1920x1080 view down the street "
                f"({wl.scene.n} nodes, per level {wl.meta['cut_per_level']}); L1 loss vs a render from the pose "
                "perturbed by 0.5 deg / 2 cm; fwd + bwd incl. pose gradient")
    else:
        raise SystemExit(f"unknown workload {name}")
    return wl, desc


def measure_view(wl, steps, warmup, tile_h=16, persistent=False, graph=True, fused=True):
    """Times one workload's step (fwd + L1 + bwd incl. pose) in the plain form,
    again with per-stage HIP events, and replayed from a HIP graph.  fused: the
    step is one gsr_rasterize_step_l1 call (compositing forward and backward
    fused per tile); the two-pass form (forward, then backward_l1) is timed
    as well for comparison."""
    import numpy as np
    import torch
    from paper_2607_14481_amd import gsr
    from paper_2607_14481_amd.rasterizer import GaussianRasterizer
    dev = torch.device("cuda:0")
    sc, cams = wl.scene, wl.cameras
    params = [torch.tensor(np.asarray(getattr(sc, k), np.float32), device=dev)
              for k in ("means", "log_scales", "quats", "opacities", "sh")]
    w2c = torch.tensor(np.asarray(cams[0].world_to_cam, np.float32)[None], device=dev)
    bg = (0.0, 0.0, 0.0)
    rast = GaussianRasterizer(cams, sc.sh_degree, tile_h=tile_h, persistent=persistent, device=dev)

    # target image (untimed)
    if wl.target_cameras is not None:
        tw2c = torch.tensor(np.asarray(wl.target_cameras[0].world_to_cam, np.float32)[None], device=dev)
        target, _ = rast.forward(params, tw2c, bg)
    else:
        tparams = list(params)
        tparams[0] = torch.tensor(np.asarray(wl.target_scene.means, np.float32), device=dev)
        target, _ = rast.forward(tparams, w2c, bg)
    target = target.clone()
    numel = target.numel()

    def two_pass(ws=None, out=None, r=rast):
        rgb, ws = r.forward(params, w2c, bg, ws=ws, out=out)
        # mean |img - target|: its image gradient is formed inside the backward
        grads, g_w2c, g_tw = r.backward_l1(ws, params, w2c, bg, rgb, target)
        return rgb, ws, grads, g_tw

    def one_call(ws=None, out=None, r=rast):
        rgb, ws, grads, g_w2c, g_tw = r.step_l1(params, w2c, bg, target, ws=ws, out=out)
        return rgb, ws, grads, g_tw

    step = one_call if fused else two_pass

    # ---- plain form: one view per launch sequence, as a training loop runs it:
    # the warm-up steps (synchronous) size the pair capacity and the long-list
    # passes, the timed steps never wait for the host, and an overflow is
    # checked after them (it would void the run)
    for _ in range(warmup):
        _, ws, _, _ = step()
    rast.stats = True  # one instrumented step for the work counters, outside the timed region
    _, ws, _, _ = step()
    rast.stats = False
    torch.cuda.synchronize()
    stats = gsr.query_stats(ws)
    log(f"[bench] stats {stats}")
    assert not rast.check_overflow(ws)
    rast.sync = False
    ws = rast.workspace(sc.n)
    out = torch.empty_like(target)
    for _ in range(2):
        step(ws, out)
    # timed region: plain steps, nothing else on the stream
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(steps):
        step(ws, out)
    end.record()
    torch.cuda.synchronize()
    ms_plain = start.elapsed_time(end) / steps
    assert not rast.check_overflow(ws), "pair capacity overflowed during the timed steps"
    log(f"[bench] plain: {ms_plain:.3f} ms/step")
    ms_two_pass = None
    if fused:  # the same steps as two library calls, for comparison
        for _ in range(2):
            two_pass(ws, out)
        torch.cuda.synchronize()
        start.record()
        for _ in range(steps):
            two_pass(ws, out)
        end.record()
        torch.cuda.synchronize()
        ms_two_pass = start.elapsed_time(end) / steps
        assert not rast.check_overflow(ws)
        log(f"[bench] two-pass form: {ms_two_pass:.3f} ms/step")

    # the same steps again with HIP events recorded by the library between its
    # stages, on the stream the kernels run on (per-stage and per-kernel times)
    stage_ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2 * len(gsr.STAGES))]
                for _ in range(steps)]
    for evs in stage_ev:
        for e in evs:
            e.record()  # creates the underlying HIP events
    torch.cuda.synchronize()
    handles = [(gsr.C.c_void_p * (2 * len(gsr.STAGES)))(*[e.cuda_event for e in evs]) for evs in stage_ev]
    torch.cuda.synchronize()
    start.record()
    for k in range(steps):
        rast.cfg.stage_events = gsr.C.cast(handles[k], gsr.C.c_void_p)
        step(ws, out)
    end.record()
    torch.cuda.synchronize()
    rast.cfg.stage_events = None
    ms_instrumented = start.elapsed_time(end) / steps
    stage_ms = {}
    for s, name in enumerate(gsr.STAGES):
        vals = [evs[2 * s].elapsed_time(evs[2 * s + 1]) for evs in stage_ev]
        stage_ms[name] = float(np.mean(vals))
    log(f"[bench] with stage events: {ms_instrumented:.3f} ms/step; stages "
        + ", ".join(f"{k} {v:.3f}" for k, v in stage_ms.items()))

    # ---- graph form: the same step, no host synchronisation, replayed
    graph_ms = None
    graph_err = None
    if graph:
        try:
            grast = GaussianRasterizer(cams, sc.sh_degree, tile_h=tile_h, persistent=persistent, sync=False,
                                       device=dev)
            grast.capacity = int(stats["pairs"] * 1.3) + 4096
            gws = grast.workspace(sc.n)
            gout = torch.empty_like(target)
            s = torch.cuda.Stream()
            s.wait_stream(torch.cuda.current_stream())
            gstep = one_call if fused else two_pass
            with torch.cuda.stream(s):
                for _ in range(3):
                    gstep(gws, gout, grast)
            torch.cuda.current_stream().wait_stream(s)
            torch.cuda.synchronize()
            assert not grast.check_overflow(gws)
            cg = torch.cuda.CUDAGraph()
            with torch.cuda.graph(cg):
                gstep(gws, gout, grast)
            for _ in range(warmup):
                cg.replay()
            torch.cuda.synchronize()
            start.record()
            for _ in range(steps):
                cg.replay()
            end.record()
            torch.cuda.synchronize()
            graph_ms = start.elapsed_time(end) / steps
            assert not grast.check_overflow(gws)
            log(f"[bench] graph: {graph_ms:.3f} ms/step")
        except Exception as e:  # reported, never hidden
            graph_err = repr(e)
            log(f"[bench] graph form failed: {graph_err}")

    return {"ms_plain": ms_plain, "ms_instrumented": ms_instrumented, "stage_ms": stage_ms, "stats": stats,
            "graph_ms": graph_ms, "graph_err": graph_err, "ms_two_pass": ms_two_pass, "fused": fused}


TILE_HEIGHTS = (4, 8, 16, 32)


def pick_tile_h(wl, persistent=False, steps=5, fused=True, heights=TILE_HEIGHTS):
    """The tile height (16 x h pixels) at which this workload's step runs
    fastest, by a short timing of each (results do not depend on it: tile
    membership is the exact alpha >= 1/255 box).  Returns (h, {h: ms})."""
    import numpy as np
    import torch
    from paper_2607_14481_amd.rasterizer import GaussianRasterizer
    dev = torch.device("cuda:0")
    sc, cams = wl.scene, wl.cameras
    params = [torch.tensor(np.asarray(getattr(sc, k), np.float32), device=dev)
              for k in ("means", "log_scales", "quats", "opacities", "sh")]
    w2c = torch.tensor(np.asarray(cams[0].world_to_cam, np.float32)[None], device=dev)
    bg = (0.0, 0.0, 0.0)
    times = {}
    for h in heights:
        rast = GaussianRasterizer(cams, sc.sh_degree, tile_h=h, persistent=persistent, device=dev)
        target, ws = rast.forward(params, w2c, bg)  # (any target: only the time is used)
        target = target.clone()
        assert not rast.check_overflow(ws)
        rast.sync = False
        ws = rast.workspace(sc.n)

        def step():
            if fused:
                rast.step_l1(params, w2c, bg, target, ws=ws)
            else:
                rgb, w = rast.forward(params, w2c, bg, ws=ws)
                rast.backward_l1(w, params, w2c, bg, rgb, target)
        for _ in range(2):
            step()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            step()
        b.record()
        torch.cuda.synchronize()
        assert not rast.check_overflow(ws)
        times[h] = round(a.elapsed_time(b) / steps, 4)
        del rast, ws
    best = min(times, key=times.get)
    log(f"[bench] tile height by measurement: {best} ({times})")
    return best, times


def copy_rates(sizes_mb=(8, 16, 32, 64, 128, 256, 512), reps=40):
    """Rate of a plain device copy (torch's copy kernel, half the bytes read,
    half written) by the bytes one launch moves, launches back to back on one
    stream as in a step: the HBM rate a memory-bound kernel of that size can
    reach on this GPU, ramp-up and tail included.  Successive copies use
    successive regions of 1 GiB pools, so the data is not cache-resident."""
    import torch
    pool_floats = 1 << 28
    src = torch.ones(pool_floats, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    out = {}
    for mb in sizes_mb:
        n = (mb << 20) // 8
        slots = pool_floats // n

        def run(k):
            for i in range(k):
                o = (i % slots) * n
                dst[o:o + n].copy_(src[o:o + n])

        run(3)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        run(reps)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        out[f"{mb}MB"] = {"us": round(us, 2), "TB_s": round((mb << 20) / (us * 1e-6) / 1e12, 3)}
    del src, dst
    return out


def run_keyframe(wl, iterations=30, repeats=3):
    """The paper's per-keyframe optimisation (Sec. 5.2): `iterations` steps of
    forward, L1 loss, backward, fused Adam on the Gaussians the forward saw,
    and the pose step with SE(3) retraction, on the given single-view
    workload.  Also times the Sim(3) relocation of every Gaussian (loop
    closure, Sec. 6.3) with 100 keyframes."""
    import numpy as np
    import torch
    from paper_2607_14481_amd import gsr
    from paper_2607_14481_amd.rasterizer import GaussianRasterizer
    sc, cams = wl.scene, wl.cameras
    dev = torch.device("cuda")
    base = [torch.tensor(np.asarray(getattr(sc, k), np.float32), device=dev)
            for k in ("means", "log_scales", "quats", "opacities", "sh")]
    rast = GaussianRasterizer(cams, sc.sh_degree)
    tw2c = torch.tensor(np.asarray(wl.target_cameras[0].world_to_cam, np.float32)[None], device=dev)
    target, tws = rast.forward(base, tw2c)
    target = target.clone()
    acfg = gsr.adam_config(sparse=True)
    # the loop never waits for the host: the pair capacity (and the long-list
    # passes) come from a synchronous forward; overflow is checked after
    assert not rast.check_overflow(tws)
    del tws
    rast.sync = False
    ws = rast.workspace(sc.n)
    rgb = torch.empty_like(target)

    def keyframe():
        params = [t.clone() for t in base]
        w2c = torch.tensor(np.asarray(cams[0].world_to_cam, np.float32)[None], device=dev)
        m = [torch.zeros_like(t) for t in params]
        v = [torch.zeros_like(t) for t in params]
        pm, pv = torch.zeros((1, 6), device=dev), torch.zeros((1, 6), device=dev)
        losses = []
        for it in range(1, iterations + 1):
            # forward, L1 loss and backward in one library call
            _, _, grads, _, twist = rast.step_l1(params, w2c, (0.0, 0.0, 0.0), target, ws=ws, out=rgb)
            if it == 1 or it == iterations:
                losses.append((rgb - target).abs().mean())
            gsr.adam_step(params, grads, m, v, sc.sh_degree, it, acfg, ws=ws, cams=cams, cfg=rast.cfg)
            gsr.pose_step(w2c, twist, pm, pv, it, 1e-4)
        return losses, params, grads, m, v

    keyframe()
    torch.cuda.synchronize()
    assert not rast.check_overflow(ws), "pair capacity overflowed during the keyframe optimisation"
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(repeats):
        losses, params, grads, m, v = keyframe()
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / repeats
    assert not rast.check_overflow(ws), "pair capacity overflowed during the keyframe optimisation"
    first, last = float(losses[0]), float(losses[-1])
    # the fused Adam step alone: dense (every Gaussian) and sparse (those the
    # last forward saw), HIP events on the stream it runs on
    n = sc.n
    floats = sum(int(t[0].numel()) for t in params)  # floats per Gaussian
    seen = int(gsr.query_stats(ws)["visible"])
    adam = {}
    for name, cfg_sparse in (("dense", False), ("sparse", True)):
        ac = gsr.adam_config(sparse=cfg_sparse)
        reps = 20
        for it in range(3):
            gsr.adam_step(params, grads, m, v, sc.sh_degree, 100 + it, ac, ws=ws, cams=cams, cfg=rast.cfg)
        torch.cuda.synchronize()
        a.record()
        for it in range(reps):
            gsr.adam_step(params, grads, m, v, sc.sh_degree, 200 + it, ac, ws=ws, cams=cams, cfg=rast.cfg)
        b.record()
        torch.cuda.synchronize()
        us_a = a.elapsed_time(b) / reps * 1e3
        rows = n if not cfg_sparse else seen
        # per updated float: parameter, gradient and both moments read, three written;
        # the sparse step also reads each Gaussian's per-view tile count
        nbytes = rows * floats * 28 + (n * 4 if cfg_sparse else 0)
        adam[name] = {"gaussians_updated": rows, "us": round(us_a, 2), "algorithmic_bytes": nbytes,
                      "GB_per_s": round(nbytes / us_a / 1e3, 1),
                      "frac_of_hbm_peak": round(nbytes / us_a / 1e3 / PEAK_HBM_GBS, 4)}
        log(f"[bench] adam {name}: {us_a:.1f} us, {nbytes / us_a / 1e3:.0f} GB/s")
    log(f"[bench] keyframe: {iterations} iterations in {ms:.2f} ms; L1 {first:.5f} -> {last:.5f}")
    # loop-closure relocation of all Gaussians
    rng = np.random.default_rng(0)
    kf = torch.tensor(rng.integers(0, 100, n).astype(np.int32), device=dev)
    q = rng.standard_normal((100, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    sims = torch.tensor(np.c_[rng.uniform(0.9, 1.1, 100), q, rng.standard_normal((100, 3))].astype(np.float32),
                        device=dev)
    moved = [t.clone() for t in base]
    for _ in range(3):
        gsr.sim3_relocate(moved, kf, sims)
    torch.cuda.synchronize()
    reps = 20
    a.record()
    for _ in range(reps):
        gsr.sim3_relocate(moved, kf, sims)
    b.record()
    torch.cuda.synchronize()
    us = a.elapsed_time(b) / reps * 1e3
    nbytes = n * (4 + 2 * (12 + 16 + 12))
    return {"workload": "per-keyframe optimisation of the headline view: forward, L1, backward, sparse Adam, "
                        "pose Adam + SE(3) retraction",
            "iterations": iterations, "ms_per_keyframe": round(ms, 3),
            "ms_per_iteration": round(ms / iterations, 4), "l1_first": round(first, 6), "l1_last": round(last, 6),
            "form": "host-sync-free forward (pair capacity from a synchronous forward of the start state)",
            "adam_step": adam,
            "sim3_relocation": {"gaussians": n, "keyframes": 100, "us": round(us, 2),
                                "algorithmic_bytes": nbytes, "GB_per_s": round(nbytes / us / 1e3, 1)}}


def run_lod_cut_gpu(wl, reps=10, tile_h=16):
    """The level-of-detail cut on the GPU for the street hierarchy (all nodes
    resident in HBM): cut selection (blocking: includes reading the count
    back) and the gather of the cut's rows, checked against the host cut."""
    import numpy as np
    import torch
    from paper_2607_14481_amd import gsr
    h, host_cut = wl.extra["hierarchy"], wl.extra["cut"]
    cam = wl.cameras[0]
    dev = torch.device("cuda")
    nodes = [torch.tensor(np.asarray(getattr(h.nodes, k), np.float32), device=dev)
             for k in ("means", "log_scales", "quats", "opacities", "sh")]
    parent = torch.tensor(h.parent.astype(np.int32), device=dev)
    counts = torch.tensor(h.child_count.astype(np.int32), device=dev)
    w2c = torch.tensor(np.asarray(cam.world_to_cam, np.float32), device=dev)
    scratch = torch.empty(gsr.lib().gsr_hierarchy_cut_scratch_bytes(int(h.nodes.n)), dtype=torch.uint8, device=dev)
    out = torch.empty(int(h.nodes.n), dtype=torch.int32, device=dev)
    cut = gsr.hierarchy_cut(nodes, 3, parent, counts, cam, w2c, 1.5, scratch=scratch, out=out)
    same = bool(np.array_equal(cut.cpu().numpy(), host_cut))
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        cut = gsr.hierarchy_cut(nodes, 3, parent, counts, cam, w2c, 1.5, scratch=scratch, out=out)
    ms_cut = (time.perf_counter() - t) * 1e3 / reps
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    sub = gsr.gather_gaussians(nodes, 3, cut)
    a.record()
    for _ in range(reps):
        sub = gsr.gather_gaussians(nodes, 3, cut)
    b.record()
    torch.cuda.synchronize()
    ms_gather = a.elapsed_time(b) / reps
    row = 4 * (3 + 3 + 4 + 1 + 48)
    log(f"[bench] lod cut on the GPU: {cut.numel()} of {h.nodes.n} nodes in {ms_cut:.3f} ms (same as host: {same}); "
        f"gather {ms_gather:.3f} ms")

    # the hierarchy itself built on the GPU from the Morton-ordered leaves: all
    # seven merge levels (moment-matched merges in FP64, SH means), timed
    n_leaves = int(h.level_start[1])
    levels = int(len(h.level_start) - 2)
    built = [torch.zeros_like(t) for t in nodes]
    for dst_t, src_t in zip(built, nodes):
        dst_t[:n_leaves] = src_t[:n_leaves]
    bparent, bcount = gsr.hierarchy_build(built, 3, n_leaves, levels, 8)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        gsr.hierarchy_build(built, 3, n_leaves, levels, 8, parent=bparent, child_count=bcount)
    b.record()
    torch.cuda.synchronize()
    ms_build = a.elapsed_time(b) / reps
    same_links = bool(torch.equal(bparent, parent) and torch.equal(bcount, counts))
    # algorithmic bytes: each inner node reads its children's rows and writes its own
    inner = int(h.level_start[-1]) - n_leaves
    build_bytes = (int(h.level_start[-2]) + inner) * row + 8 * int(h.level_start[-1])
    log(f"[bench] hierarchy build on the GPU: {levels} levels over {n_leaves} leaves in {ms_build:.3f} ms "
        f"(links as the host build: {same_links})")
    del built

    # the whole level-of-detail step with no host round trip: the cut writes its
    # size to a device scalar that the gather and the rasterizer read; cut,
    # gather and the one-call L1 step are captured in one graph and replayed
    from paper_2607_14481_amd.rasterizer import GaussianRasterizer
    nn = int(h.nodes.n)
    tw2c = torch.tensor(np.asarray(wl.target_cameras[0].world_to_cam, np.float32)[None], device=dev)
    target, _ = GaussianRasterizer([cam], 3).forward(sub, tw2c)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    idx = torch.empty(nn, dtype=torch.int32, device=dev)
    buf = [torch.empty_like(t) for t in nodes]
    rast = GaussianRasterizer([cam], 3, tile_h=tile_h, active_count=count)
    gsr.hierarchy_cut_async(nodes, 3, parent, counts, cam, w2c, 1.5, scratch, idx, count)
    gsr.gather_gaussians(nodes, 3, idx, count=count, dst=buf)
    rgb, ws0 = rast.forward(buf, w2c[None])  # synchronous: sizes the pair capacity and long-list passes
    assert not rast.check_overflow(ws0)
    del ws0
    rast.sync = False
    ws = rast.workspace(nn)

    def step():
        gsr.hierarchy_cut_async(nodes, 3, parent, counts, cam, w2c, 1.5, scratch, idx, count)
        gsr.gather_gaussians(nodes, 3, idx, count=count, dst=buf)
        return rast.step_l1(buf, w2c[None], (0.0, 0.0, 0.0), target, ws=ws, out=rgb)

    graph_ms = None
    try:
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            for _ in range(3):
                step()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            step()
        for _ in range(3):
            g.replay()
        torch.cuda.synchronize()
        a.record()
        for _ in range(reps):
            g.replay()
        b.record()
        torch.cuda.synchronize()
        graph_ms = a.elapsed_time(b) / reps
        assert int(count.item()) == cut.numel() and not rast.check_overflow(ws)
        log(f"[bench] lod step (cut + gather + one-call step) in one graph: {graph_ms:.3f} ms")
    except Exception as e:  # reported, never hidden
        log(f"[bench] lod step graph failed: {e!r}")
        graph_ms = repr(e)
    return {"nodes": nn, "cut": int(cut.numel()), "same_as_host_cut": same,
            "cut_ms_blocking": round(ms_cut, 4), "gather_ms": round(ms_gather, 4),
            "gather_GB_per_s": round(2 * row * cut.numel() / (ms_gather * 1e-3) / 1e9, 1),
            "hierarchy_build": {"leaves": n_leaves, "levels": levels, "inner_nodes": inner, "ms": round(ms_build, 4),
                                "links_same_as_host_build": same_links, "algorithmic_bytes": build_bytes,
                                "GB_per_s": round(build_bytes / (ms_build * 1e-3) / 1e9, 1)},
            "step_in_one_graph_ms": round(graph_ms, 4) if isinstance(graph_ms, float) else graph_ms,
            "step_in_one_graph_note": f"cut (size to a device scalar) + gather + the one-call L1 step at 16x{tile_h} tiles, arrays and "
                                      "workspace sized for all nodes, replayed from one HIP graph"}


def run_ring(steps, warmup):
    """8 cameras (mixed 640x480 / 1280x720 / 1920x1080) on a 15 m ring around
    1M Gaussians, SH degree 3: one step = fwd + L1 + bwd over all 8 views,
    gradients summed over views.  Plain = one view per launch sequence;
    batched = the autotuned launch grouping, captured in a HIP graph."""
    import numpy as np
    import torch
    from paper_2607_14481_amd import gsr
    from paper_2607_14481_amd import scenes as S
    from paper_2607_14481_amd.autotune import MultiViewStep, autotune
    from paper_2607_14481_amd.rasterizer import GaussianRasterizer
    wl = S.multi_view_ring()
    sc, cams = wl.scene, wl.cameras
    dev = torch.device("cuda")
    params = [torch.tensor(np.asarray(getattr(sc, k), np.float32), device=dev)
              for k in ("means", "log_scales", "quats", "opacities", "sh")]
    w2c = torch.tensor(np.stack([np.asarray(c.world_to_cam, np.float32) for c in cams]), device=dev)
    targets, pairs = [], []
    for v, c in enumerate(cams):
        r = GaussianRasterizer([c], sc.sh_degree)
        tw = torch.tensor(S.perturbed_pose(c.world_to_cam, 3000 + v)[None], device=dev)
        t, _ = r.forward(params, tw)
        targets.append(t.clone())
        _, ws = r.forward(params, w2c[v:v + 1])
        pairs.append(gsr.query_pairs(ws)[0])
    plain = MultiViewStep(cams, sc.sh_degree, params, w2c, targets, views_per_launch=1)
    from paper_2607_14481_amd.autotune import _time
    ms_plain = _time(plain, steps, warmup)
    log(f"[bench] ring plain (8 launch sequences): {ms_plain:.3f} ms/step")
    tuned = autotune(cams, sc.sh_degree, params, w2c, targets, cache_path=None, log=log, steps=3, warmup=1)
    best = tuned["best"]
    step = MultiViewStep(cams, sc.sh_degree, params, w2c, targets, sync=False, capacity_hint=pairs, **best)
    s_ = torch.cuda.Stream()
    s_.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s_):
        for _ in range(2):
            step(keep_workspaces=True)
    torch.cuda.current_stream().wait_stream(s_)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step(keep_workspaces=True)
    ms_graph = _time(graph.replay, steps, warmup)
    ovf = any(g[0].check_overflow(ws) for g, ws in zip(step.groups, step.ws))
    log(f"[bench] ring batched {best} graph: {ms_graph:.3f} ms/step (overflow {ovf})")
    return {"workload": "8-camera ring (r = 15 m), resolutions " + ", ".join(f"{c.width}x{c.height}" for c in cams)
                        + ", 1,000,000 Gaussians SH 3, fwd+bwd over all views, gradients summed",
            "pairs_per_view": pairs,
            "plain_ms_per_step": round(ms_plain, 4), "plain_iters_per_s": round(1000 / ms_plain, 3),
            "batched_config": best, "batched_graph_ms_per_step": round(ms_graph, 4),
            "batched_graph_iters_per_s": round(1000 / ms_graph, 3), "overflow": bool(ovf),
            "autotune_ms": tuned["ms"]}


def run_serving(seconds, rate=200.0, start=2_900_000, per_keyframe=10_000, period=0.5, seed=5,
                overload_rate=1000.0, overload_seconds=3.0):
    """Poisson arrivals (mean `rate`/s) of render / optimise requests (50/50;
    resolutions uniform over 256x256..1920x1080; optimise = 1-4 views, fwd+bwd
    vs a U(0,1) target) against a scene that grows by `per_keyframe` every
    `period` seconds.  The configured schedule grows 500k -> 3M Gaussians over
    125 s; this window is its last `seconds` (the scene starts at `start`, so
    that it ends at >= 3M).  Returns latency/throughput for one request at a
    time and for continuous batching, at the configured rate and at an
    overload rate where throughput separates the two modes."""
    import torch
    from paper_2607_14481_amd.serve import GrowingScene, Server, make_requests
    out = {"arrival_rate_per_s": rate, "window_s": seconds, "start_gaussians": start,
           "growth": f"{per_keyframe} Gaussians per {period} s keyframe",
           "window_note": "the last seconds of the 500k -> 3M schedule (scene built at its size there)"}
    runs = (("rate", rate, seconds, seed), ("overload", overload_rate, overload_seconds, seed + 7))
    for name, slots, group in (("one_at_a_time", 1, False), ("continuous_batching", 4, True)):
        for tag, lam, dur, sd in runs:
            kfs = int(dur / period) + 2
            scene = GrowingScene(capacity=start + per_keyframe * kfs, start=start, per_keyframe=per_keyframe)
            warm = make_requests(seed + 1000, rate=lam, duration=0.1)
            ws = Server(scene, slots=slots, group_renders=group)
            ws.run(warm, keyframe_period=1e9, bind_versions=True)
            torch.cuda.synchronize()
            reqs = make_requests(sd, rate=lam, duration=dur)
            # the measured server starts from the pair-count model the warm-up learned
            st = Server(scene, slots=slots, group_renders=group, pair_rate=ws.pair_rate).run(
                reqs, keyframe_period=period)
            del ws
            log(f"[bench] serving {name} at {lam:g}/s: {st['requests']} req, p50 {st['p50_ms']:.2f} ms, "
                f"p99 {st['p99_ms']:.2f} ms, {st['throughput_req_s']:.1f} req/s, final {st['final_gaussians']} "
                "Gaussians")
            res = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in st.items()}
            res["arrival_rate_per_s"] = lam
            if tag == "rate":
                out[name] = res
            else:
                out.setdefault("overload", {})[name] = res
            del scene
            torch.cuda.empty_cache()
    return out


def run_local_ba(iters=10, repeats=30, cpu_baseline=True):
    """Local bundle adjustment at the paper's timing size: 20 keyframes (4 fixed),
    10,000 landmarks seen by 2-8 consecutive keyframes each, focal length
    optimised, `iters` damped Gauss-Newton steps in FP64.  Timed from the
    device-resident start state (reset by a copy outside the timed region),
    eager launches and one captured graph."""
    import numpy as np
    import torch
    from paper_2607_14481_amd import gsr
    from paper_2607_14481_amd.ba_scenes import make_problem

    P = make_problem(0, pixel_noise=0.5)
    t0 = time.time()
    plan = gsr.BAPlan(P.free_slot, P.obs_cam)
    torch.cuda.synchronize()
    plan_ms = (time.time() - t0) * 1e3
    d = "cuda"
    init = (torch.tensor(P.init_poses, dtype=torch.float64, device=d),
            torch.tensor([P.init_focal], dtype=torch.float64, device=d),
            torch.tensor(P.init_landmarks, dtype=torch.float64, device=d))
    uv = torch.tensor(P.obs_uv, dtype=torch.float64, device=d)
    poses, focal, pts = [t.clone() for t in init]
    costs = torch.zeros(iters + 1, dtype=torch.float64, device=d)

    def reset():
        poses.copy_(init[0]); focal.copy_(init[1]); pts.copy_(init[2])

    def solve():
        gsr.ba_solve(plan, poses, focal, P.principal, pts, uv, iters, 1e-4, costs)

    for _ in range(3):
        reset(); solve()
    torch.cuda.synchronize()

    def timed(fn):
        ms = []
        for _ in range(repeats):
            reset()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(); fn(); b.record()
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
        return float(np.median(ms)), float(np.min(ms))

    eager_med, eager_min = timed(solve)
    c = costs.cpu().numpy()
    graph_med = graph_min = None
    try:
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            reset(); solve()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            solve()
        graph_med, graph_min = timed(g.replay)
        same = bool(np.array_equal(costs.cpu().numpy(), c))
    except Exception as e:  # pragma: no cover - reported, not fatal
        log(f"[bench] BA graph capture failed: {e}")
        same = None
    n_obs = int((P.obs_cam >= 0).sum())
    # algorithmic bytes of one iteration: the landmark kernel reads pose, landmark
    # and pixel per observation and writes a 608-B record per observation in a
    # free keyframe and 80 B per landmark; the assembly reads 312 B per such
    # observation (diagonal blocks) and 2 x 144 B per pair of them in one landmark
    # (off-diagonal blocks); the update reads 144 B per such observation plus
    # 48 B per landmark and writes 24 B per landmark.
    free_obs = (P.obs_cam >= 0) & (P.free_slot[np.maximum(P.obs_cam, 0)] >= 0)
    per_lm = free_obs.sum(axis=1)
    n_free_obs, n_pairs = int(per_lm.sum()), int((per_lm * (per_lm - 1) // 2).sum())
    K = P.n_landmarks
    it_bytes = (n_obs * (96 + 24 + 16) + n_free_obs * 608 + K * 80
                + n_free_obs * 312 + n_pairs * 288
                + n_free_obs * 144 + K * (48 + 24))
    it_ms = eager_med / iters
    out = {"workload": f"local BA: 20 keyframes (4 fixed), 10,000 landmarks, {n_obs} observations (2-8 consecutive "
                       f"keyframes per landmark), focal length optimised, {iters} LM iterations, FP64",
           "ms_per_solve": round(eager_med, 4), "ms_per_solve_min": round(eager_min, 4),
           "graph_ms_per_solve": round(graph_med, 4) if graph_med else None,
           "graph_ms_per_solve_min": round(graph_min, 4) if graph_min else None,
           "graph_matches_eager": same,
           "ms_per_iteration": round(eager_med / iters, 4),
           "plan_create_ms": round(plan_ms, 3),
           "cost_first_last": [float(c[0]), float(c[-1])],
           "paper_ms_rtx4090": 15.9,
           "iteration_traffic": {"algorithmic_bytes": it_bytes, "GB_per_s": round(it_bytes / (it_ms * 1e-3) / 1e9, 1),
                                 "frac_of_hbm_peak": round(it_bytes / (it_ms * 1e-3) / 8e12, 4),
                                 "note": "whole iteration (4 launches); the dominant kernel, the one-workgroup "
                                         "Cholesky of the 97-unknown reduced system, is bound by its serial "
                                         "chain, not by HBM or the FP64 units"}}
    if cpu_baseline:
        from oracle import ba as B
        lm, cam, ouv = P.flat_observations()
        pr = {"free_slot": P.free_slot, "c": np.array(P.principal), "obs_lm": lm, "obs_cam": cam, "obs_uv": ouv}
        st = {"poses": P.init_poses, "f": P.init_focal, "landmarks": P.init_landmarks}
        t = time.time()
        B.apply_step(pr, st, B.step_schur(pr, st, 1e-4))
        t_it = time.time() - t
        out["cpu_baseline"] = {"value": round(t_it * iters * 1e3, 1), "unit": "ms per solve", "cores": 1,
                               "kind": "oracle", "sample": f"one of the {iters} iterations at full size "
                                                           f"({t_it:.2f} s), times {iters}; numpy FP64"}
    log(f"[bench] local BA: {eager_med:.3f} ms eager, {graph_med} ms graph per {iters}-iteration solve")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="headline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--two-pass", action="store_true",
                    help="time the step as forward then backward_l1 instead of one fused call")
    ap.add_argument("--tile-h", type=int, default=0,
                    help="tile height 4, 8, 16 or 32 (width 16); 0: each workload's fastest, by a short timing")
    ap.add_argument("--persistent", action="store_true", help="compositing as persistent work-queue launches")
    ap.add_argument("--no-ring", action="store_true", help="skip the batched 8-view measurement")
    ap.add_argument("--no-keyframe", action="store_true",
                    help="skip the 30-iteration keyframe optimisation and relocation measurement")
    ap.add_argument("--no-other-workloads", action="store_true",
                    help="skip the small-view, 200k-at-1080p and level-of-detail measurements")
    ap.add_argument("--serve-seconds", type=float, default=5.0,
                    help="length of the Poisson request window of the serving measurement (0: skip)")
    ap.add_argument("--no-ba", action="store_true", help="skip the local bundle-adjustment measurement")
    ap.add_argument("--ba-only", action="store_true",
                    help="measure only the local bundle adjustment and print its JSON object")
    ap.add_argument("--copy-calibration", action="store_true",
                    help=f"first run {COPY_CAL_REPS} plain device copies of {COPY_CAL_MIB} MiB (the reference "
                         "kernel that scales HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: sharding the rasterizer over GPUs (one view per GPU, one "
              "gradient reduce-scatter) is not implemented; run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2607_14481_amd import gsr
    from paper_2607_14481_amd.rasterizer import GaussianRasterizer

    torch.cuda.init()
    dev = torch.device("cuda:0")
    if args.ba_only:
        print(json.dumps(run_local_ba(cpu_baseline=not args.no_cpu_baseline)), flush=True)
        return
    if args.copy_calibration:
        # reference kernels of known traffic for the HBM byte counters: a plain
        # copy (reads and writes COPY_CAL_MIB), a read-only reduction over the
        # same buffer (a sum: reads COPY_CAL_MIB), and a gather of random
        # 64-byte rows (reads and writes 64 B per row, in 64-byte pieces)
        src = torch.ones(COPY_CAL_MIB << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(COPY_CAL_REPS):
            dst.copy_(src)
        tot = torch.zeros((), device=dev)
        for _ in range(COPY_CAL_REPS):
            tot += src.sum()
        rows = src.view(-1, 16)
        pick = torch.randperm(rows.shape[0], device=dev)[: rows.shape[0] // 4]
        for _ in range(COPY_CAL_REPS):
            torch.index_select(rows, 0, pick, out=dst.view(-1, 16)[: pick.numel()])
        torch.cuda.synchronize()
        log(f"[bench] calibration: copy {COPY_CAL_MIB} MiB, sum {COPY_CAL_MIB} MiB, gather {pick.numel()} rows "
            f"of 64 B ({pick.numel() * 64 / 2**20:.0f} MiB), {COPY_CAL_REPS} times each")
        del src, dst, rows, pick
    t0 = time.time()
    wl, desc = make_workload(args.workload)
    sc, cams = wl.scene, wl.cameras
    log(f"[bench] workload {args.workload}: n={sc.n} view {cams[0].width}x{cams[0].height} "
        f"(inputs built in {time.time() - t0:.1f}s)")
    tile_h, tile_ms = (args.tile_h, None) if args.tile_h else pick_tile_h(wl, args.persistent,
                                                                           fused=not args.two_pass)
    m = measure_view(wl, args.steps, args.warmup, tile_h, args.persistent, not args.no_graph,
                     fused=not args.two_pass)
    ms_plain, ms_instrumented, stage_ms, stats = m["ms_plain"], m["ms_instrumented"], m["stage_ms"], m["stats"]
    graph_ms, graph_err = m["graph_ms"], m["graph_err"]

    copy_rate = None
    if not args.copy_calibration:  # (a counter run keeps its copies to the calibration ones)
        copy_rate = copy_rates()
        log("[bench] plain copy rate by bytes per launch: " +
            ", ".join(f"{k} {v['TB_s']} TB/s ({v['us']} us)" for k, v in copy_rate.items()))

    # ---- the other single-view workloads: small view, 200k at 1080p, the level-of-detail cut
    others = None
    if not args.no_other_workloads:
        others = {}
        for name in OTHER_WORKLOADS:
            if name == args.workload:
                continue
            t0 = time.time()
            owl, odesc = make_workload(name)
            log(f"[bench] workload {name}: n={owl.scene.n} (inputs built in {time.time() - t0:.1f}s)")
            oth, oth_ms = (args.tile_h, None) if args.tile_h else pick_tile_h(owl, args.persistent)
            om = measure_view(owl, max(10, args.steps // 2), max(3, args.warmup // 2), oth,
                              args.persistent, not args.no_graph)
            others[name] = {"workload": odesc, "n_gaussians": owl.scene.n,
                            "resolution": f"{owl.cameras[0].width}x{owl.cameras[0].height}",
                            "tile": f"16x{oth}", "tile_ms_by_height": oth_ms,
                            "plain_iters_per_s": round(1000.0 / om["ms_plain"], 3),
                            "plain_ms_per_step": round(om["ms_plain"], 4),
                            "graph_iters_per_s": round(1000.0 / om["graph_ms"], 3) if om["graph_ms"] else None,
                            "graph_ms_per_step": round(om["graph_ms"], 4) if om["graph_ms"] else None,
                            "two_pass_ms_per_step": round(om["ms_two_pass"], 4) if om["ms_two_pass"] else None,
                            "graph_error": om["graph_err"],
                            "stage_ms": {k: round(v, 4) for k, v in om["stage_ms"].items()},
                            "work": om["stats"], "meta": owl.meta, "_wl": owl}
            if name == "lod_cut":
                others[name]["gpu_cut"] = run_lod_cut_gpu(owl, tile_h=oth)
            del om
            torch.cuda.empty_cache()

    # ---- the per-keyframe optimisation loop (30 iterations) and the loop-closure relocation
    keyframe = None
    if not args.no_keyframe and wl.target_cameras is not None:
        keyframe = run_keyframe(wl)

    # ---- batched views: the 8-camera ring, plain vs autotuned + graph
    ring = None
    if not args.no_ring:
        ring = run_ring(max(5, args.steps // 5), 2)

    # ---- serving: the same seeded arrivals, one request at a time vs continuous batching
    served = None
    if args.serve_seconds > 0:
        served = run_serving(args.serve_seconds)

    # ---- the local bundle adjustment (20 keyframes x 10,000 landmarks, 10 iterations)
    local_ba = None if args.no_ba else run_local_ba(cpu_baseline=not args.no_cpu_baseline)

    # ---- roofline of the dominant kernel (compositing, ALU-bound): the fused
    # compositing of the one-call step (timed as the forward compositing stage,
    # doing the forward's and the backward's work), else the larger of the two
    fwd_flops = FLOPS_FWD_EVAL * stats["evaluations"] + FLOPS_FWD_CONTRIB * stats["contributors"]
    bwd_flops = FLOPS_BWD_EVAL * stats["replays"] + FLOPS_BWD_CONTRIB * stats["contributors"]
    if m["fused"]:
        dom, flops, dom_ms = "composite_step", fwd_flops + bwd_flops, stage_ms["composite_fwd"]
    else:
        comp = {"composite_fwd": stage_ms["composite_fwd"], "composite_bwd": stage_ms["composite_bwd"]}
        dom = max(comp, key=comp.get)
        flops, dom_ms = (bwd_flops if dom == "composite_bwd" else fwd_flops), comp[dom]
    achieved = flops / (dom_ms * 1e-3) / 1e12
    traffic = measured_traffic(args.workload, dom)
    roofline = {"kernel": dom, "bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                "traffic": traffic["bytes"] if traffic else None,
                "traffic_note": traffic["note"] if traffic else "no byte-counter profile of the current kernel sources",
                "algorithmic_flops": int(flops), "ms": round(dom_ms, 4)}

    # ---- CPU baseline: the FP64 oracle as it stands, one full iteration
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O

        def oracle_iteration(scene, cam):
            rng = np.random.default_rng(0)
            shape = (cam.height, cam.width, 3)
            g = np.sign(rng.standard_normal(shape)) / float(np.prod(shape))  # L1-shaped upstream
            t = time.time()
            O.render(scene, cam, bg=(0.0, 0.0, 0.0), dL_dimg=g)
            return time.time() - t

        oracle_iteration(sc, cams[0])  # warm-up
        runs = [oracle_iteration(sc, cams[0]) for _ in range(5)]
        tfb = float(np.median(runs))
        host = host_cpu()
        cpu = {"value": round(1.0 / tfb, 5), "unit": "iters/s", "cores": 1, "kind": "oracle",
               "sample": f"median of 5 full fwd+bwd iterations of the same view and scene after one warm-up "
                         f"({', '.join(f'{t:.2f}' for t in runs)} s), single-threaded C, FP64",
               "host_nproc": host["nproc"], "host_cpu_model": host["model"],
               "note": "the oracle is serial C: its summation order is the definition the GPU is checked "
                       "against, so it is timed on one core and not parallelised"}
        log(f"[bench] oracle fwd+bwd median {tfb:.2f}s of {runs}")
        procs = max(1, min(16, host["nproc"]))
        try:
            walls = [oracle_all_cores(procs)[0] for _ in range(3)]
            wall = float(np.median(walls))
            cpu["all_cores"] = {
                "value": round(1.0 / wall, 4), "unit": "iters/s", "cores": procs,
                "sample": f"median of 3 ({', '.join(f'{w:.2f}' for w in walls)} s wall): the same fwd+bwd "
                          f"split into {procs} bands of tile rows, one process each, each the unmodified oracle "
                          f"on its band's tiles (every process still projects all Gaussians)"}
            log(f"[bench] oracle fwd+bwd on {procs} processes: median {wall:.2f}s wall of {walls}")
        except RuntimeError as e:
            cpu["all_cores"] = {"error": str(e)}
            log(f"[bench] oracle on {procs} processes failed: {e}")
        if others:
            cpu["other_workloads_s_per_iter"] = {}
            for name, o in others.items():
                t_o = oracle_iteration(o["_wl"].scene, o["_wl"].cameras[0])
                cpu["other_workloads_s_per_iter"][name] = round(t_o, 4)
                o["oracle_s_per_iter"] = round(t_o, 4)
                log(f"[bench] oracle {name} fwd+bwd {t_o:.2f}s")

    out = {
        "metric": "fwd+bwd raster iters/s @1080p, 1M Gaussians; p50/p99 request latency",
        "value": round(1000.0 / ms_plain, 3),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_plain, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc}", "n_gaussians": sc.n,
                   "resolution": f"{cams[0].width}x{cams[0].height}", "sh_degree": sc.sh_degree,
                   "form": ("plain: one view per launch sequence, " + ("one gsr_rasterize_step_l1 call per step (compositing forward and backward fused per tile)" if m["fused"] else "forward then backward_l1") + ", no host synchronisation in the timed steps (pair capacity and long-list passes sized by synchronous warm-up steps, overflow checked after)"),
                   "tile": f"16x{tile_h}", "tile_ms_by_height": tile_ms, "persistent": bool(args.persistent)},
        "graph_form": {"iters_per_s": round(1000.0 / graph_ms, 3) if graph_ms else None,
                       "ms_per_step": round(graph_ms, 4) if graph_ms else None, "error": graph_err},
        "two_pass_form": ({"iters_per_s": round(1000.0 / m["ms_two_pass"], 3),
                           "ms_per_step": round(m["ms_two_pass"], 4),
                           "note": "the same step as gsr_rasterize_forward then gsr_rasterize_backward_l1"}
                          if m["ms_two_pass"] else None),
        "stage_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "ms_per_step_with_stage_events": round(ms_instrumented, 4),
        "work": stats,
        "roofline": roofline,
        "copy_rate_by_size": copy_rate,
        "cpu_baseline": cpu,
        "other_workloads": ({k: {a: b for a, b in v.items() if a != "_wl"} for k, v in others.items()}
                            if others else None),
        "keyframe_optimisation": keyframe,
        "batched_views": ring,
        "serving": served,
        "local_ba": local_ba,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
