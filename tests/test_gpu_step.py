"""The one-call L1 step (gsr_rasterize_step_l1): the compositing forward and
backward fused per tile must give, bit for bit, the image, the parameter and
pose gradients and the workspace state of gsr_rasterize_forward followed by
gsr_rasterize_backward_l1, at every launch configuration and whatever the
workspace held before; and the gradients of the mean absolute error must be
the FP64 oracle's."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2607_14481_amd import scenes as S

from ._util import (GRAD_KEYS, GRAD_TOL, compare_grads, compare_view, lod_workload, log, params_to_device,
                    planar_to_hwc, poses_to_device, rel_err)

pytestmark = pytest.mark.gpu


def _target_near(rgb, seed, lo=0.02, hi=0.05):
    """A target image at a seeded distance of lo..hi from rgb in every channel,
    so that sign(rgb - target) does not hang on rounding; and that sign."""
    import torch
    rng = np.random.default_rng(seed)
    s = np.where(rng.random(rgb.numel()) < 0.5, -1.0, 1.0)
    u = rng.uniform(lo, hi, rgb.numel())
    tgt = rgb.detach().cpu().numpy().astype(np.float64) + s * u
    return torch.tensor(tgt.astype(np.float32), device=rgb.device), -s


def _two_pass(rast, params, w2c, bg, target, ws=None):
    rgb, ws = rast.forward(params, w2c, bg, ws=ws)
    grads, g_w2c, g_tw = rast.backward_l1(ws, params, w2c, bg, rgb, target)
    return rgb, ws, grads, g_w2c, g_tw


def _assert_same(a, b, label):
    import torch
    torch.cuda.synchronize()
    names = ("rgb", "ws", "grads", "w2c", "twist")
    for name, x, y in zip(names, a, b):
        if name == "ws":
            continue
        xs, ys = (x, y) if isinstance(x, list) else ([x], [y])
        for i, (p, q) in enumerate(zip(xs, ys)):
            if not torch.equal(p, q):
                d = float((p - q).abs().max())
                raise AssertionError(f"{label}: {name}[{i}] differs (max |d| {d:.3e})")
    log(f"{label}: one-call step bit-identical to forward + backward_l1")


def _views(kind):
    if kind == "small_sh0":
        wl = S.small_view(seed=4, n=3000, width=200, height=136, sh_degree=0)
        return wl.scene, wl.cameras[:1]
    wl = S.multi_view_ring(seed=5, n=15_000, n_views=3)
    sizes = [(160, 120), (320, 180), (96, 72)]
    return wl.scene, [S.pinhole(w, h, c.world_to_cam) for (w, h), c in zip(sizes, wl.cameras)]


@pytest.mark.parametrize("kind,tile_h,persistent", [
    ("small_sh0", 16, False), ("small_sh0", 16, True),
    ("ring3_sh3", 4, False), ("ring3_sh3", 8, False), ("ring3_sh3", 16, False), ("ring3_sh3", 32, False),
    ("ring3_sh3", 16, True), ("ring3_sh3", 32, True)])
def test_step_matches_two_passes(kind, tile_h, persistent):
    from paper_2607_14481_amd.rasterizer import GaussianRasterizer
    sc, cams = _views(kind)
    log(f"step vs two passes: {kind}, tile 16x{tile_h}, persistent={persistent}")
    rast = GaussianRasterizer(cams, sc.sh_degree, tile_h=tile_h, persistent=persistent)
    params, w2c = params_to_device(sc), poses_to_device(cams)
    bg = (0.1, 0.2, 0.3)
    img, _ = rast.forward(params, w2c, bg)
    target, _ = _target_near(img, 11)
    a = _two_pass(rast, params, w2c, bg, target)
    b = rast.step_l1(params, w2c, bg, target)
    _assert_same(a, b, f"{kind} 16x{tile_h} p{int(persistent)}")


def test_step_schedule_hint_changes_nothing():
    """The fused compositing takes tiles in an order filed from the replay
    counts the workspace holds from its previous step: a workspace full of
    garbage, one reused after another pose, and a fresh one give the same
    results (and so does the host-sync-free form)."""
    import torch
    from paper_2607_14481_amd.rasterizer import GaussianRasterizer
    sc, cams = _views("ring3_sh3")
    rast = GaussianRasterizer(cams, sc.sh_degree)
    params, w2c = params_to_device(sc), poses_to_device(cams)
    bg = (0.0, 0.0, 0.0)
    img, ws0 = rast.forward(params, w2c, bg)
    target, _ = _target_near(img, 12)
    ref = _two_pass(rast, params, w2c, bg, target)
    nb = ws0.numel()
    garbage = torch.randint(0, 256, (nb,), dtype=torch.uint8, device="cuda",
                            generator=torch.Generator(device="cuda").manual_seed(3))
    _assert_same(ref, rast.step_l1(params, w2c, bg, target, ws=garbage), "workspace of random bytes")
    # the same workspace after a step from another pose
    w2c_b = w2c.clone()
    w2c_b[:, 0, 3] += 0.3
    rast.step_l1(params, w2c_b, bg, target, ws=garbage)
    _assert_same(ref, rast.step_l1(params, w2c, bg, target, ws=garbage), "workspace reused after another pose")
    rast.sync = False
    _assert_same(ref, rast.step_l1(params, w2c, bg, target, ws=garbage), "host-sync-free step")
    assert not rast.check_overflow(garbage)


def test_step_leaves_the_forward_state_for_a_backward():
    """After the one-call step the workspace holds the forward's state: a
    general backward with another upstream gradient on it equals the same
    backward after a plain forward."""
    import torch
    from paper_2607_14481_amd.rasterizer import GaussianRasterizer
    sc, cams = _views("ring3_sh3")
    rast = GaussianRasterizer(cams, sc.sh_degree)
    params, w2c = params_to_device(sc), poses_to_device(cams)
    bg = (0.0, 0.0, 0.0)
    img, ws_f = rast.forward(params, w2c, bg)
    target, _ = _target_near(img, 13)
    up = torch.tensor(np.random.default_rng(5).standard_normal(img.numel()).astype(np.float32), device="cuda")
    a = rast.backward(ws_f, params, w2c, bg, img, up)
    rgb, ws_s, _, _, _ = rast.step_l1(params, w2c, bg, target)
    b = rast.backward(ws_s, params, w2c, bg, rgb, up)
    torch.cuda.synchronize()
    for x, y in zip(a[0], b[0]):
        assert torch.equal(x, y)
    assert torch.equal(a[1], b[1]) and torch.equal(a[2], b[2])
    log("backward with another upstream after the one-call step: bit-identical")


def test_step_overflow_matches_two_passes():
    """Without host synchronisation a pair capacity too small makes both forms
    skip the binning alike: background image, zero gradients, overflow flagged."""
    import torch
    from paper_2607_14481_amd.rasterizer import GaussianRasterizer
    sc, cams = _views("ring3_sh3")
    rast = GaussianRasterizer(cams, sc.sh_degree, sync=False)
    rast.capacity = 1000
    params, w2c = params_to_device(sc), poses_to_device(cams)
    bg = (0.1, 0.2, 0.3)
    target = torch.full((3 * rast.total_pixels,), 0.5, device="cuda")
    a = _two_pass(rast, params, w2c, bg, target, ws=rast.workspace(sc.n, 1000))
    assert rast.check_overflow(a[1])
    b = rast.step_l1(params, w2c, bg, target, ws=rast.workspace(sc.n, 1000))
    assert rast.check_overflow(b[1])
    _assert_same(a, b, "overflow")
    assert all(float(g.abs().max()) == 0.0 for g in b[2])


def test_step_stats_flag_runs_the_two_passes():
    from paper_2607_14481_amd import gsr
    from paper_2607_14481_amd.rasterizer import GaussianRasterizer
    sc, cams = _views("small_sh0")
    rast = GaussianRasterizer(cams, sc.sh_degree)
    params, w2c = params_to_device(sc), poses_to_device(cams)
    img, _ = rast.forward(params, w2c)
    target, _ = _target_near(img, 14)
    a = _two_pass(rast, params, w2c, (0.0, 0.0, 0.0), target)
    rast.stats = True
    b = rast.step_l1(params, w2c, (0.0, 0.0, 0.0), target)
    _assert_same(a, b, "stats flag")
    st = gsr.query_stats(b[1])
    assert st["evaluations"] > 0 and st["replays"] > 0 and st["contributors"] > 0


def test_step_target_must_not_be_null():
    import torch
    from paper_2607_14481_amd import gsr
    from paper_2607_14481_amd.rasterizer import GaussianRasterizer
    sc, cams = _views("small_sh0")
    rast = GaussianRasterizer(cams, sc.sh_degree)
    params, w2c = params_to_device(sc), poses_to_device(cams)
    ws = rast.workspace(sc.n)
    rgb = torch.empty(3 * rast.total_pixels, device="cuda")
    grads = [torch.empty_like(p) for p in params]
    with pytest.raises(gsr.GsrError):
        gsr.rasterize_step_l1(ws, params, sc.sh_degree, cams, w2c.reshape(-1, 16), (0.0, 0.0, 0.0), None, rgb,
                              grads)
    assert "target" in gsr.last_error()


@pytest.mark.parametrize("kind", ["small_sh0", "ring3_sh3"])
def test_step_l1_gradients_match_the_oracle(kind):
    """The oracle's image, a target at 0.02..0.05 from it (so that the sign of
    C - target is the same on both sides), and the oracle's backward of the
    mean absolute error: dL/dC = sign(C - target) / (3 sum H W)."""
    from paper_2607_14481_amd.rasterizer import GaussianRasterizer
    import torch
    sc, cams = _views(kind)
    bg = (0.05, 0.1, 0.15)
    refs = [O.render(sc, c, bg=bg) for c in cams]
    imgs = np.concatenate([np.ascontiguousarray(r["img"].transpose(2, 0, 1)).reshape(-1) for r in refs])
    rng = np.random.default_rng(21)
    s = np.where(rng.random(imgs.size) < 0.5, -1.0, 1.0)
    tgt = imgs + s * rng.uniform(0.02, 0.05, imgs.size)
    count = 3.0 * sum(c.width * c.height for c in cams)
    outs, o = [], 0
    tot = {k: 0.0 for k in GRAD_KEYS}
    for c in cams:
        npx = 3 * c.width * c.height
        up = (-s[o:o + npx] / count).reshape(3, c.height, c.width).transpose(1, 2, 0)
        r = O.render(sc, c, bg=bg, dL_dimg=up)
        outs.append(r)
        for k in GRAD_KEYS:
            tot[k] = tot[k] + r[k]
        o += npx
    rast = GaussianRasterizer(cams, sc.sh_degree)
    params, w2c = params_to_device(sc), poses_to_device(cams)
    rgb, _, grads, g_w2c, g_tw = rast.step_l1(params, w2c, bg, torch.tensor(tgt.astype(np.float32), device="cuda"))
    torch.cuda.synchronize()
    for v, (img, r) in enumerate(zip(planar_to_hwc(rgb, cams), outs)):
        compare_view(img, r, f"{kind} view {v}")
        assert rel_err(g_w2c[v].cpu().numpy(), r["w2c"]) <= GRAD_TOL
        assert rel_err(g_tw[v].cpu().numpy(), r["twist"]) <= GRAD_TOL
    gpu = {k: t.cpu().numpy().astype(np.float64) for k, t in zip(GRAD_KEYS, grads)}
    compare_grads(gpu, tot, f"{kind} one-call L1 step vs oracle")


_BIG = {}


def _big(name):
    if name not in _BIG:
        _BIG[name] = S.headline_view() if name == "headline" else lod_workload()
    return _BIG[name]


@pytest.mark.parametrize("name,tile_h", [("headline", 16), ("lod_cut", 16), ("lod_cut", 8)])
def test_step_full_size_matches_two_passes(name, tile_h):
    """The 1080p, 1M-Gaussian headline view as the benchmark runs it (a
    synchronous step sizes the capacity, then steps without host
    synchronisation reuse one workspace), and the level-of-detail view whose
    longest tile lists need seven merge passes at 16x16 tiles (six at the
    16x8 tiles the benchmark picks for it)."""
    import torch
    from paper_2607_14481_amd.rasterizer import GaussianRasterizer
    wl = _big(name)
    sc, cams = wl.scene, wl.cameras[:1]
    rast = GaussianRasterizer(cams, sc.sh_degree, tile_h=tile_h)
    params, w2c = params_to_device(sc), poses_to_device(cams)
    bg = (0.0, 0.0, 0.0)
    img, ws0 = rast.forward(params, w2c, bg)
    target, _ = _target_near(img, 31)
    assert not rast.check_overflow(ws0)
    del ws0
    rast.sync = False
    ws = rast.workspace(sc.n)
    ref = _two_pass(rast, params, w2c, bg, target, ws=ws)
    ref = [x.clone() if isinstance(x, torch.Tensor) else ([g.clone() for g in x] if isinstance(x, list) else x)
           for x in ref]
    for k in range(2):  # the second step's schedule comes from the first's replay counts
        got = rast.step_l1(params, w2c, bg, target, ws=ws)
        _assert_same(ref, got, f"{name} 16x{tile_h} step {k}")
    assert not rast.check_overflow(ws)


@pytest.mark.parametrize("persistent", [False, True])
def test_step_ring_8_views_as_autotuned_matches_two_passes(persistent):
    """The 8-view ring at full size in the configuration the autotuner picks
    (all views in one call, 16x32 tiles, the one-call step)."""
    import torch
    from paper_2607_14481_amd.rasterizer import GaussianRasterizer
    if "ring" not in _BIG:
        _BIG["ring"] = S.multi_view_ring()
    wl = _BIG["ring"]
    sc, cams = wl.scene, wl.cameras
    rast = GaussianRasterizer(cams, sc.sh_degree, tile_h=32, persistent=persistent)
    params, w2c = params_to_device(sc), poses_to_device(cams)
    bg = (0.0, 0.0, 0.0)
    img, _ = rast.forward(params, w2c, bg)
    target, _ = _target_near(img, 41)
    ref = _two_pass(rast, params, w2c, bg, target)
    got = rast.step_l1(params, w2c, bg, target)
    _assert_same(ref, got, f"8-view ring, 16x32 tiles, persistent={persistent}")
    torch.cuda.synchronize()


@pytest.mark.parametrize("persistent", [False, True])
def test_step_graph_replays_match_eager(persistent):
    """The one-call step captured in a HIP graph, as the benchmark's graph form
    runs it (no host synchronisation, capacity from an eager step): every
    replay, with other eager work through the library between replays, gives
    the eager step's image and gradients bit for bit.  The replays carry the
    fused kernel's schedule (the previous step's replay counts) and, with
    persistent compositing, its work-queue counters from one to the next."""
    import torch
    from paper_2607_14481_amd.rasterizer import GaussianRasterizer
    sc, cams = _views("ring3_sh3")
    bg = (0.0, 0.0, 0.0)
    params, w2c = params_to_device(sc), poses_to_device(cams)
    eager = GaussianRasterizer(cams, sc.sh_degree, persistent=persistent)
    img, _ = eager.forward(params, w2c, bg)
    target, _ = _target_near(img, 31)
    ref = eager.step_l1(params, w2c, bg, target)
    torch.cuda.synchronize()
    assert not eager.check_overflow(ref[1])  # records the pair count
    g = GaussianRasterizer(cams, sc.sh_degree, persistent=persistent, sync=False)
    g.capacity = int(eager.last_pairs * 1.2) + 1024
    ws = g.workspace(sc.n)
    out = torch.empty_like(img)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(2):
            g.step_l1(params, w2c, bg, target, ws=ws, out=out)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        got = g.step_l1(params, w2c, bg, target, ws=ws, out=out)
    for rep in range(4):
        junk = GaussianRasterizer(cams, sc.sh_degree)
        junk.step_l1([params[0] * 1.01] + params[1:], w2c, bg, target)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert not g.check_overflow(ws)
        _assert_same(ref, got, f"graph replay {rep} (persistent {persistent})")
