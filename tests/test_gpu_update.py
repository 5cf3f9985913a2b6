"""Parameter updates through the C ABI against the FP64 update oracle: the
fused Adam step (dense and restricted to the Gaussians the last forward saw),
the pose step with SE(3) retraction, and the Sim(3) relocation."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import update as U
from paper_2607_14481_amd import scenes as S

from ._util import log

pytestmark = pytest.mark.gpu

LRS = dict(means=1.6e-4, log_scales=5e-3, quats=1e-3, opacities=5e-2, sh_dc=2.5e-3, sh_rest=1.25e-4)
KEYS = U.KEYS


def _random_state(rng, n, deg):
    K = (deg + 1) ** 2
    shapes = dict(means=(n, 3), log_scales=(n, 3), quats=(n, 4), opacities=(n,), sh=(n, K, 3))
    p = {k: rng.standard_normal(s).astype(np.float32) for k, s in shapes.items()}
    p["opacities"] = rng.uniform(0.05, 0.95, n).astype(np.float32)
    return p, shapes


def _dev(d):
    import torch
    return [torch.tensor(np.ascontiguousarray(d[k], np.float32), device="cuda") for k in KEYS]


def _host(ts):
    return {k: t.cpu().numpy().astype(np.float64) for k, t in zip(KEYS, ts)}


def _compare(gpu, ref, what, rtol=2e-5, atol=1e-6):
    for k in KEYS:
        err = np.abs(gpu[k] - ref[k]) - (atol + rtol * np.abs(ref[k]))
        log(f"{what} {k}: max |d| {np.abs(gpu[k] - ref[k]).max():.3e}")
        assert err.max() <= 0, (what, k)


def _acfg(gsr, sparse=False, eps=1e-8):
    return gsr.adam_config(lr_means=LRS["means"], lr_log_scales=LRS["log_scales"], lr_quats=LRS["quats"],
                           lr_opacities=LRS["opacities"], lr_sh_dc=LRS["sh_dc"], lr_sh_rest=LRS["sh_rest"],
                           eps=eps, sparse=sparse)


@pytest.mark.parametrize("deg,n", [(3, 1000), (2, 777), (0, 65)])
def test_adam_dense_matches_oracle(deg, n):
    import torch
    from paper_2607_14481_amd import gsr
    rng = np.random.default_rng(10 + deg)
    p, shapes = _random_state(rng, n, deg)
    zero = {k: np.zeros(s, np.float32) for k, s in shapes.items()}
    P, M, V = _dev(p), _dev(zero), _dev(zero)
    refP, refM, refV = p, zero, zero
    for step in (1, 2, 3):
        g = {k: rng.standard_normal(s).astype(np.float32) for k, s in shapes.items()}
        gsr.adam_step(P, _dev(g), M, V, deg, step, _acfg(gsr))
        refP, refM, refV = U.adam(refP, g, refM, refV, step, LRS, 0.9, 0.999, 1e-8)
    torch.cuda.synchronize()
    _compare(_host(P), refP, f"adam deg {deg} params")
    _compare(_host(M), refM, f"adam deg {deg} exp_avg")
    _compare(_host(V), refV, f"adam deg {deg} exp_avg_sq", rtol=1e-4, atol=1e-9)


def test_sparse_adam_updates_only_what_the_forward_saw():
    import torch
    from paper_2607_14481_amd import gsr
    from paper_2607_14481_amd.rasterizer import GaussianRasterizer
    from ._util import params_to_device, poses_to_device
    wl = S.small_view(seed=12, n=1500, width=96, height=80, sh_degree=1, xy_half=2.5)
    sc, cams = wl.scene, wl.cameras
    vis = O.project(sc, cams[0])["visible"]
    log(f"sparse adam: {int(vis.sum())} of {sc.n} visible (oracle)")
    assert 0 < vis.sum() < sc.n
    rast = GaussianRasterizer(cams, sc.sh_degree)
    params = params_to_device(sc)
    _, ws = rast.forward(params, poses_to_device(cams))
    assert gsr.query_stats(ws)["visible"] == int(vis.sum())
    rng = np.random.default_rng(5)
    host = {k: np.asarray(getattr(sc, k), np.float32) for k in KEYS}
    g = {k: rng.standard_normal(host[k].shape).astype(np.float32) for k in KEYS}
    zero = {k: np.zeros_like(host[k]) for k in KEYS}
    M, V = _dev(zero), _dev(zero)
    gsr.adam_step(params, _dev(g), M, V, sc.sh_degree, 1, _acfg(gsr, sparse=True), ws=ws, cams=cams,
                  cfg=rast.cfg)
    torch.cuda.synchronize()
    refP, refM, refV = U.adam(host, g, zero, zero, 1, LRS, 0.9, 0.999, 1e-8, visible=vis)
    got = _host(params)
    for k in KEYS:
        np.testing.assert_array_equal(got[k][~vis], host[k][~vis])  # untouched, bit for bit
    _compare(got, refP, "sparse adam params")
    _compare(_host(M), refM, "sparse adam exp_avg")


@pytest.mark.parametrize("deg,n_views", [(0, 1), (1, 3), (2, 2), (3, 1), (3, 4)])
def test_sparse_adam_is_the_dense_step_on_the_seen_rows(deg, n_views):
    """Every SH row width, one view and several overlapping ones: the sparse
    step (which walks the visible-item list, each Gaussian by the first view
    that saw it) leaves unseen rows untouched bit for bit, gives the seen rows
    exactly what the dense step gives them, two steps running, and matches the
    oracle restricted to the union of the views' visible sets."""
    import torch
    from paper_2607_14481_amd import gsr
    from paper_2607_14481_amd.rasterizer import GaussianRasterizer
    from ._util import params_to_device, poses_to_device
    wl = S.small_view(seed=20 + deg, n=3000 + 17 * deg, width=96, height=72, sh_degree=deg, xy_half=2.5)
    sc, cam = wl.scene, wl.cameras[0]
    # further views: the first pose turned and moved a little (overlapping sets)
    cams = [cam] + [cam.copy_with_pose(S.perturbed_pose(cam.world_to_cam, seed=40 + v, degrees=12.0, metres=0.4))
                    for v in range(1, n_views)]
    vis = np.zeros(sc.n, bool)
    per_view = []
    for c in cams:
        pv = O.project(sc, c)["visible"]
        per_view.append(int(pv.sum()))
        vis |= pv
    log(f"sparse adam deg {deg}, {n_views} views: {int(vis.sum())} of {sc.n} seen (per view {per_view})")
    assert 0 < vis.sum() < sc.n
    if n_views > 1:
        assert sum(per_view) > vis.sum()  # the views overlap: some Gaussians are listed more than once
    rast = GaussianRasterizer(cams, sc.sh_degree)
    params = params_to_device(sc)
    _, ws = rast.forward(params, poses_to_device(cams))
    rng = np.random.default_rng(30 + deg)
    host = {k: np.asarray(getattr(sc, k), np.float32) for k in KEYS}
    grads = [{k: rng.standard_normal(host[k].shape).astype(np.float32) for k in KEYS} for _ in range(2)]
    zero = {k: np.zeros_like(host[k]) for k in KEYS}
    P_s, M_s, V_s = _dev(host), _dev(zero), _dev(zero)
    P_d, M_d, V_d = _dev(host), _dev(zero), _dev(zero)
    refP, refM, refV = host, zero, zero
    for step, g in enumerate(grads, start=1):
        gsr.adam_step(P_s, _dev(g), M_s, V_s, sc.sh_degree, step, _acfg(gsr, sparse=True), ws=ws, cams=cams,
                      cfg=rast.cfg)
        gsr.adam_step(P_d, _dev(g), M_d, V_d, sc.sh_degree, step, _acfg(gsr))
        refP, refM, refV = U.adam(refP, g, refM, refV, step, LRS, 0.9, 0.999, 1e-8, visible=vis)
    torch.cuda.synchronize()
    for got, dense, base in ((P_s, P_d, host), (M_s, M_d, zero), (V_s, V_d, zero)):
        hs, hd = _host(got), _host(dense)
        for k in KEYS:
            np.testing.assert_array_equal(hs[k][~vis], base[k][~vis].astype(np.float64), err_msg=k)
            np.testing.assert_array_equal(hs[k][vis], hd[k][vis], err_msg=k)
    _compare(_host(P_s), refP, "sparse adam params")
    _compare(_host(M_s), refM, "sparse adam exp_avg")
    _compare(_host(V_s), refV, "sparse adam exp_avg_sq", rtol=1e-4, atol=1e-9)


@pytest.mark.parametrize("deg", [1, 3])
def test_keyframe_loop_matches_the_oracle_step_by_step(deg):
    """The keyframe optimisation as timed (the one-call L1 step on a reused
    workspace with no host synchronisation, the sparse Adam step on that
    workspace, the pose step on the twist gradient), three iterations.  Each
    iteration is checked from the state the GPU reached before it: the image,
    Gaussian and twist gradients against the oracle's render of that state,
    then the parameters and the pose against the oracle's update applied to
    the GPU's gradients.  The target lies 0.05..0.1 from the start image, so
    the sign of C - target, the L1 gradient, is the same on both sides."""
    import torch
    from paper_2607_14481_amd import gsr
    from paper_2607_14481_amd.rasterizer import GaussianRasterizer
    from ._util import (GRAD_KEYS, GRAD_TOL, compare_grads, compare_view, params_to_device, planar_to_hwc,
                        poses_to_device, rel_err)
    wl = S.small_view(seed=50 + deg, n=2500, width=96, height=72, sh_degree=deg, xy_half=2.0)
    sc, cam = wl.scene, wl.cameras[0]
    bg = (0.0, 0.0, 0.0)
    img0 = O.render(sc, cam, bg=bg)["img"]
    rng = np.random.default_rng(60 + deg)
    sgn = np.where(rng.random(img0.shape) < 0.5, -1.0, 1.0)
    tgt = img0 + sgn * rng.uniform(0.05, 0.1, img0.shape)
    up = -sgn / float(img0.size)  # dL/dC = sign(C - target) / (3 H W) while |C - C0| < 0.05
    target = torch.tensor(np.ascontiguousarray(tgt.transpose(2, 0, 1)).reshape(-1).astype(np.float32), device="cuda")

    rast = GaussianRasterizer([cam], sc.sh_degree)
    params, w2c = params_to_device(sc), poses_to_device([cam])
    rast.forward(params, w2c, bg)  # a synchronous forward sizes the pair capacity
    rast.sync = False
    ws = rast.workspace(sc.n)
    rgb = torch.empty_like(target)
    m = [torch.zeros_like(t) for t in params]
    v = [torch.zeros_like(t) for t in params]
    pm, pv = torch.zeros((1, 6), device="cuda"), torch.zeros((1, 6), device="cuda")
    acfg, lr_pose = _acfg(gsr, sparse=True), 1e-4
    def host(ts):
        return {k: t.cpu().numpy().astype(np.float64) for k, t in zip(KEYS, ts)}

    for it in (1, 2, 3):
        P, M, V = host(params), host(m), host(v)
        T, PM, PV = w2c.cpu().numpy()[0].astype(np.float64), pm.cpu().numpy(), pv.cpu().numpy()
        _, _, grads, _, twist = rast.step_l1(params, w2c, bg, target, ws=ws, out=rgb)
        G = {k: t.cpu().numpy() for k, t in zip(KEYS, grads)}
        tw = twist.cpu().numpy()
        gsr.adam_step(params, grads, m, v, sc.sh_degree, it, acfg, ws=ws, cams=[cam], cfg=rast.cfg)
        gsr.pose_step(w2c, twist, pm, pv, it, lr_pose, eps=1e-8)
        torch.cuda.synchronize()
        assert not rast.check_overflow(ws)
        # the step against the oracle at the state before it
        state = S.Scene(*(P[k].astype(np.float32) for k in KEYS), sc.sh_degree)
        c_t = cam.copy_with_pose(T.astype(np.float32))
        ref = O.render(state, c_t, bg=bg, dL_dimg=up)
        compare_view(planar_to_hwc(rgb, [c_t])[0], ref, f"keyframe deg {deg} it {it}")
        compare_grads({k: G[k].astype(np.float64) for k in GRAD_KEYS}, {k: ref[k] for k in GRAD_KEYS},
                      f"keyframe deg {deg} it {it}")
        assert rel_err(tw[0], ref["twist"]) <= GRAD_TOL
        # the updates against the oracle's, from the GPU's gradients
        seen = O.project(state, c_t)["visible"]
        refP, refM, refV = U.adam(P, G, M, V, it, LRS, 0.9, 0.999, 1e-8, visible=seen)
        _compare(host(params), refP, f"keyframe it {it} params")
        _compare(host(m), refM, f"keyframe it {it} exp_avg")
        refT, _, _ = U.pose_step(T[None], tw, PM, PV, it, lr_pose, 0.9, 0.999, 1e-8)
        np.testing.assert_allclose(w2c.cpu().numpy()[0], refT[0], atol=2e-6, rtol=0)
        moved = np.abs(refT[0] - T).max()
        log(f"keyframe deg {deg} it {it}: {int(seen.sum())} of {sc.n} seen, pose moved {moved:.2e}")
        assert 0 < seen.sum() < sc.n and moved > 1e-5  # a real sparse step, a real pose step


def test_pose_step_matches_oracle():
    import torch
    from paper_2607_14481_amd import gsr
    rng = np.random.default_rng(6)
    V = 3
    T = np.stack([U.se3_exp(rng.standard_normal(6) * 0.5) for _ in range(V)]).astype(np.float32)
    w2c = torch.tensor(T, device="cuda")
    m = torch.zeros((V, 6), device="cuda")
    v = torch.zeros((V, 6), device="cuda")
    refT, refm, refv = T.astype(np.float64), np.zeros((V, 6)), np.zeros((V, 6))
    for step in (1, 2):
        g = rng.standard_normal((V, 6)).astype(np.float32)
        lr = 0.05 if step == 1 else 1e-6  # a large and a tiny rotation (series branch)
        gsr.pose_step(w2c, torch.tensor(g, device="cuda"), m, v, step, lr)
        refT, refm, refv = U.pose_step(refT.astype(np.float32), g, refm, refv, step, lr, 0.9, 0.999, 1e-15)
    torch.cuda.synchronize()
    err = np.abs(w2c.cpu().numpy() - refT).max()
    log(f"pose step: max |d T| {err:.3e}")
    assert err <= 2e-6
    np.testing.assert_allclose(m.cpu().numpy(), refm, rtol=1e-5, atol=1e-7)


def test_sim3_relocation_matches_oracle():
    import torch
    from paper_2607_14481_amd import gsr
    rng = np.random.default_rng(7)
    n, K = 5000, 6
    p, _ = _random_state(rng, n, 1)
    p["quats"] /= np.linalg.norm(p["quats"], axis=1, keepdims=True)
    kf = rng.integers(-2, K + 2, n).astype(np.int32)  # some ids outside [0, K): not moved
    sims = []
    for k in range(K):
        q = rng.standard_normal(4)
        q /= np.linalg.norm(q)
        sims.append(np.r_[rng.uniform(0.5, 2.0), q, rng.standard_normal(3) * 3])
    sims = np.array(sims, np.float32)
    P = _dev(p)
    gsr.sim3_relocate(P, torch.tensor(kf, device="cuda"), torch.tensor(sims, device="cuda"))
    torch.cuda.synchronize()
    got = _host(P)
    kf_valid = np.where(kf < K, kf, -1)
    mu, q, ls = U.sim3_relocate(p["means"], p["quats"], p["log_scales"], kf_valid, sims)
    for name, a, b in (("means", got["means"], mu), ("quats", got["quats"], q), ("log_scales", got["log_scales"], ls)):
        err = np.abs(a - b).max()
        log(f"sim3 {name}: max |d| {err:.3e}")
        assert err <= 1e-5 * max(1.0, np.abs(b).max())
    np.testing.assert_array_equal(got["opacities"], p["opacities"])
    np.testing.assert_array_equal(got["sh"], p["sh"])
    np.testing.assert_array_equal(got["means"][kf_valid < 0], p["means"][kf_valid < 0])
