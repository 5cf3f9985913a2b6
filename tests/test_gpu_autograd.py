"""The autograd front-end (torch.autograd.Function over the C ABI):
gradients against the FP64 oracle, against central finite differences of the
GPU forward itself, the 6-DoF pose twist, repeated forwards before a backward,
and graph capture (replays compared with eager results)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2607_14481_amd import scenes as S

from ._util import log, rel_err

pytestmark = pytest.mark.gpu


def _params(scene, requires_grad=True):
    import torch
    return [torch.tensor(np.asarray(getattr(scene, k), np.float32), device="cuda", requires_grad=requires_grad)
            for k in ("means", "log_scales", "quats", "opacities", "sh")]


def _planar(up):
    return np.ascontiguousarray(np.asarray(up, np.float32).transpose(2, 0, 1)).reshape(-1)


def _fd_scene():
    # the oracle's finite-difference scene: no pixel near a decision boundary
    rng = np.random.default_rng(48)
    n = 6
    cam = S.Camera(28, 22, 30.0, 30.0, 14.0, 11.0,
                   S.look_at([0.3, -0.2, -4.0], target=[0, 0, 0.5], up=[0, -1, 0]).astype(np.float32))
    sc = S.Scene(np.c_[rng.uniform(-0.4, 0.4, (n, 2)), rng.uniform(-0.3, 0.8, n)].astype(np.float32),
                 rng.normal(-1.9, 0.2, (n, 3)).astype(np.float32), rng.standard_normal((n, 4)).astype(np.float32),
                 rng.uniform(0.3, 0.9, n).astype(np.float32), rng.normal(0, 0.3, (n, 4, 3)).astype(np.float32), 1)
    return sc, cam


def test_autograd_matches_oracle_gradients():
    import torch
    from paper_2607_14481_amd.rasterizer import GaussianRasterizer, rasterize
    wl = S.small_view(seed=9, n=800, width=120, height=90, sh_degree=3, z_range=(1.0, 5.0), xy_half=1.5)
    sc, cam = wl.scene, wl.cameras[0]
    params = _params(sc)
    w2c = torch.tensor(np.asarray(S.look_at([0.2, 0.1, -1.0], target=[0, 0, 3.0], up=[0, -1, 0]), np.float32)[None],
                       device="cuda", requires_grad=True)
    cam = cam.copy_with_pose(w2c[0].detach().cpu().numpy())
    rast = GaussianRasterizer([cam], 3)
    bg = (0.2, 0.3, 0.1)
    up = S.random_upstream(5, (90, 120, 3))
    rgb = rasterize(*params, w2c, rasterizer=rast, bg=bg)
    (rgb * torch.tensor(_planar(up), device="cuda")).sum().backward()
    ref = O.render(sc, cam, bg=bg, dL_dimg=up)
    for k, p in zip(("means", "log_scales", "quats", "opacities", "sh"), params):
        e = rel_err(p.grad.cpu().numpy(), ref[k])
        log(f"autograd d{k}: {e:.2e}")
        assert e <= 1e-3
    assert rel_err(w2c.grad[0].cpu().numpy(), ref["w2c"]) <= 1e-3
    assert rel_err(rast.last_twist_grad[0].cpu().numpy(), ref["twist"]) <= 1e-3


# Central differences of the FP32 forward carry its rounding: the loss (a sum
# of ~1.8e3 weighted pixels) moves by ~1e-6 between the two evaluations
# independently of the step, i.e. ~5e-4 after division by 2h = 2e-3; the
# absolute slack below covers that noise floor.  The same directions are also
# differenced on the FP64 oracle forward, which has no such floor, and the GPU's
# analytic derivative must match that to 1e-3 relative.
FD_H = 1e-3
FD32_REL, FD32_ABS = 1e-2, 1e-3
FD64_REL, FD64_ABS = 1e-3, 1e-5


def _oracle_loss(sc, cam, g, key=None, value=None, pose=None):
    keys = ("means", "log_scales", "quats", "opacities", "sh")
    kw = {k: getattr(sc, k) for k in keys}
    if key is not None:
        kw[key] = value
    scene = S.Scene(kw["means"], kw["log_scales"], kw["quats"], kw["opacities"], kw["sh"], sc.sh_degree)
    c = cam if pose is None else cam.copy_with_pose(pose)
    return float((O.render(scene, c)["img"] * g).sum())


def test_autograd_matches_finite_differences_fp32():
    import torch
    from scipy.linalg import expm
    from paper_2607_14481_amd.rasterizer import GaussianRasterizer, rasterize
    sc, cam = _fd_scene()
    rast = GaussianRasterizer([cam], sc.sh_degree)
    up = S.random_upstream(2, (22, 28, 3))
    g = torch.tensor(_planar(up), device="cuda")
    params = _params(sc)
    w2c = torch.tensor(np.asarray(cam.world_to_cam, np.float32)[None], device="cuda", requires_grad=True)
    (rasterize(*params, w2c, rasterizer=rast) * g).sum().backward()
    grads = [p.grad.detach().clone() for p in params]
    twist = rast.last_twist_grad[0].detach().cpu().numpy().astype(np.float64)

    def loss(ps, pose):
        with torch.no_grad():
            return float((rasterize(*ps, pose, rasterizer=rast).double() * g.double()).sum())

    rng = np.random.default_rng(0)
    h = FD_H
    keys = ("means", "log_scales", "quats", "opacities", "sh")
    for k, (p, gr) in enumerate(zip(params, grads)):
        d = torch.tensor(rng.standard_normal(tuple(p.shape)).astype(np.float32), device="cuda")
        d /= d.norm()
        base = [q.detach() for q in params]
        plus = list(base)
        minus = list(base)
        plus[k] = base[k] + h * d
        minus[k] = base[k] - h * d
        fd = (loss(plus, w2c.detach()) - loss(minus, w2c.detach())) / (2 * h)
        an = float((gr * d).sum())
        fd64 = (_oracle_loss(sc, cam, up, keys[k], plus[k].cpu().numpy())
                - _oracle_loss(sc, cam, up, keys[k], minus[k].cpu().numpy())) / (2 * h)
        log(f"fd param {k}: analytic {an:.6f} fd fp32 {fd:.6f} fd oracle {fd64:.6f}")
        assert abs(an - fd) <= FD32_REL * max(abs(fd), abs(an)) + FD32_ABS
        assert abs(an - fd64) <= FD64_REL * abs(fd64) + FD64_ABS
    T0 = np.asarray(cam.world_to_cam, np.float64)
    d = rng.standard_normal(6)
    d /= np.linalg.norm(d)
    vals, vals64 = [], []
    for sgn in (1, -1):
        xi = sgn * h * d
        X = np.zeros((4, 4))
        X[:3, :3] = [[0, -xi[5], xi[4]], [xi[5], 0, -xi[3]], [-xi[4], xi[3], 0]]
        X[:3, 3] = xi[:3]
        pose = (expm(X) @ T0).astype(np.float32)
        vals.append(loss([q.detach() for q in params], torch.tensor(pose[None], device="cuda")))
        vals64.append(_oracle_loss(sc, cam, up, pose=pose))
    fd = (vals[0] - vals[1]) / (2 * h)
    fd64 = (vals64[0] - vals64[1]) / (2 * h)
    an = float(twist @ d)
    log(f"fd pose twist: analytic {an:.6f} fd fp32 {fd:.6f} fd oracle {fd64:.6f}")
    assert abs(an - fd) <= FD32_REL * max(abs(fd), abs(an)) + FD32_ABS
    assert abs(an - fd64) <= FD64_REL * abs(fd64) + FD64_ABS


def test_several_forwards_before_backward():
    import torch
    from paper_2607_14481_amd.rasterizer import GaussianRasterizer, rasterize
    wl = S.small_view(seed=10, n=600, width=80, height=64, sh_degree=1)
    sc, cam = wl.scene, wl.cameras[0]
    rast = GaussianRasterizer([cam], 1)
    params = _params(sc)
    w2c = torch.tensor(np.asarray(cam.world_to_cam, np.float32)[None], device="cuda", requires_grad=True)
    g1 = torch.tensor(_planar(S.random_upstream(1, (64, 80, 3))), device="cuda")
    g2 = torch.tensor(_planar(S.random_upstream(2, (64, 80, 3))), device="cuda")
    # two renders share the rasterizer; each keeps its own workspace until its backward
    a = rasterize(*params, w2c, rasterizer=rast)
    shifted = [params[0] + 0.01] + params[1:]
    b = rasterize(*shifted, w2c, rasterizer=rast)
    ((a * g1).sum() + (b * g2).sum()).backward()
    got = params[0].grad.cpu().numpy()
    ref1 = O.render(sc, cam, dL_dimg=S.random_upstream(1, (64, 80, 3)))
    ref2 = O.render(sc.with_means(np.asarray(sc.means) + 0.01), cam, dL_dimg=S.random_upstream(2, (64, 80, 3)))
    assert rel_err(got, ref1["means"] + ref2["means"]) <= 1e-3


def test_graph_capture_replays_match_eager():
    import torch
    from paper_2607_14481_amd.rasterizer import GaussianRasterizer
    from ._util import params_to_device, poses_to_device
    wl = S.small_view(seed=11, n=3000, width=160, height=120, sh_degree=2)
    sc, cams = wl.scene, wl.cameras
    params = params_to_device(sc)
    w2c = poses_to_device(cams)
    up = torch.tensor(_planar(S.random_upstream(3, (120, 160, 3))), device="cuda")
    eager = GaussianRasterizer(cams, 2)
    rgb_e, ws_e = eager.forward(params, w2c)
    grads_e, gw_e, _ = eager.backward(ws_e, params, w2c, (0, 0, 0), rgb_e, up)
    torch.cuda.synchronize()
    assert not eager.check_overflow(ws_e)  # records the pair count
    g = GaussianRasterizer(cams, 2, sync=False)
    g.capacity = int(eager.last_pairs * 1.2) + 1024
    ws = g.workspace(sc.n)
    out = torch.empty_like(rgb_e)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        g.forward(params, w2c, ws=ws, out=out)
        g.backward(ws, params, w2c, (0, 0, 0), out, up)
    torch.cuda.current_stream().wait_stream(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        rgb_g, _ = g.forward(params, w2c, ws=ws, out=out)
        grads_g, gw_g, _ = g.backward(ws, params, w2c, (0, 0, 0), rgb_g, up)
    for rep in range(4):
        # eager work between replays: a different render through the same library
        junk = GaussianRasterizer(cams, 2)
        junk.forward([params[0] * 1.01] + params[1:], w2c)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert not g.check_overflow(ws)
        assert torch.equal(rgb_g, rgb_e), rep
        for a, b in zip(grads_g, grads_e):
            assert torch.equal(a, b), rep
        assert torch.equal(gw_g, gw_e), rep


@pytest.mark.parametrize("multi", [False, True])
def test_l1_backward_matches_explicit_upstream(multi):
    """The backward of the mean absolute error, with dL/dC formed inside the
    library, against the general backward given sign(C - target) / (3 sum HW)
    computed by torch: the same upstream values, so bit-identical results."""
    import torch
    from paper_2607_14481_amd.rasterizer import GaussianRasterizer
    from ._util import params_to_device, poses_to_device
    if multi:
        wl = S.multi_view_ring(seed=6, n=20_000, n_views=3, radius=15.0)
        cams = [S.pinhole(c.width // 4, c.height // 4, c.world_to_cam) for c in wl.cameras]
        sc = wl.scene
    else:
        wl = S.small_view(seed=8, n=1500, width=96, height=80, sh_degree=2)
        sc, cams = wl.scene, wl.cameras
    rast = GaussianRasterizer(cams, sc.sh_degree)
    params = params_to_device(sc)
    w2c = poses_to_device(cams)
    rgb, ws = rast.forward(params, w2c)
    target = torch.rand(rgb.shape, generator=torch.Generator(device="cuda").manual_seed(3), device="cuda")
    ga, wa, ta = rast.backward_l1(ws, params, w2c, (0.0, 0.0, 0.0), rgb, target)
    gb, wb, tb = rast.backward(ws, params, w2c, (0.0, 0.0, 0.0), rgb, torch.sign(rgb - target) / rgb.numel())
    torch.cuda.synchronize()
    for x, y in zip(list(ga) + [wa, ta], list(gb) + [wb, tb]):
        assert torch.equal(x, y)
    log(f"l1 backward (multi={multi}): bit-identical; |dmeans| {float(ga[0].abs().max()):.3e}")



def test_multi_view_step_same_for_every_grouping():
    """The batched step's loss is the mean absolute error over all views'
    pixels: all views in one call (upstream formed inside the library, as two
    passes or as the fused one-call step) and one view per call (upstream
    formed by torch, gradients summed) agree, and the step's gradient matches
    the oracle's for the loss against targets the oracle's own images fix."""
    import torch
    from paper_2607_14481_amd.autotune import MultiViewStep
    from paper_2607_14481_amd.rasterizer import GaussianRasterizer
    wl = S.multi_view_ring(seed=6, n=12_000, n_views=3)
    sc = wl.scene
    sizes = [(144, 96), (96, 80), (200, 120)]
    cams = [S.pinhole(w, h, c.world_to_cam) for (w, h), c in zip(sizes, wl.cameras)]
    params = _params(sc, requires_grad=False)
    w2c = torch.tensor(np.stack([np.asarray(c.world_to_cam, np.float32) for c in cams]), device="cuda")
    targets = []
    for v, c in enumerate(cams):
        r = GaussianRasterizer([c], sc.sh_degree)
        tw = torch.tensor(S.perturbed_pose(c.world_to_cam, 70 + v)[None], device="cuda")
        targets.append(r.forward(params, tw)[0].clone())
    log("multi-view step, 3 views, n=12000: one call vs one call per view")
    one, g_one = MultiViewStep(cams, sc.sh_degree, params, w2c, targets, views_per_launch=3)()
    fus, g_fus = MultiViewStep(cams, sc.sh_degree, params, w2c, targets, views_per_launch=3, fused=True)()
    per, g_per = MultiViewStep(cams, sc.sh_degree, params, w2c, targets, views_per_launch=1)()
    for a, b in zip(one + [g_one], fus + [g_fus]):
        assert torch.equal(a, b)
    for k, a, b in zip(("means", "log_scales", "quats", "opacities", "sh"), one, per):
        e = rel_err(a.cpu().numpy(), b.cpu().numpy())
        log(f"  d{k}: rel diff {e:.2e}")
        assert e <= 1e-5, k
    assert rel_err(g_one.cpu().numpy(), g_per.cpu().numpy()) <= 1e-5
    # against the oracle: targets at 0.02..0.05 from the oracle's images, so
    # that sign(C - target) is the same on both sides
    refs = [O.render(sc, c) for c in cams]
    rng = np.random.default_rng(77)
    numel = sum(3 * c.width * c.height for c in cams)
    otargets, ups = [], []
    for c, r in zip(cams, refs):
        s_ = np.where(rng.random((c.height, c.width, 3)) < 0.5, -1.0, 1.0)
        t = r["img"] + s_ * rng.uniform(0.02, 0.05, s_.shape)
        otargets.append(torch.tensor(np.ascontiguousarray(t.transpose(2, 0, 1)).reshape(-1).astype(np.float32),
                                     device="cuda"))
        ups.append(-s_ / numel)
    outs, tot = O.render_views(sc, cams, dL_dimgs=ups)
    got, _ = MultiViewStep(cams, sc.sh_degree, params, w2c, otargets, views_per_launch=3, fused=True)()
    for k, a in zip(("means", "log_scales", "quats", "opacities", "sh"), got):
        e = rel_err(a.cpu().numpy(), tot[k])
        log(f"  d{k} vs oracle: {e:.2e}")
        assert e <= 1e-3, k
