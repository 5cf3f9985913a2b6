"""Dense brute-force FP64 oracle (PyTorch CPU, autograd gradients).

TEST INFRASTRUCTURE ONLY.  Only tests, the package smoke check and the
benchmark's CPU-baseline leg may import this module.  It does not import the GPU
package and shares nothing with the C oracle either: it is a second, independent
statement of the same definition, used to pin the C oracle.

Definition (per pixel, no tiles): every Gaussian that survives projection is
evaluated at the pixel centre in (float32 depth bits, index) order; alpha =
min(0.99, o * exp(-sigma)); Gaussians with sigma < 0 or alpha < 1/255 are
skipped; compositing stops, without adding, at the first Gaussian that would
take the transmittance below 1e-4.  Gradients come from autograd on that
expression, with the discrete decisions (skip, stop, culling) held fixed, so
they are the true derivatives of the forward wherever it is differentiable.
Follows the 3DGS lineage that the paper's renderer builds on (Sec. 5.2).
"""
from __future__ import annotations

import math

import numpy as np
import torch

ALPHA_MAX = 0.99
ALPHA_MIN = 1.0 / 255.0
T_MIN = 1e-4


def _sh_basis(degree, d):
    """Real SH basis (3DGS order and signs) at unit directions d [N, 3]."""
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    pi = math.pi
    out = [torch.full_like(x, 1.0 / (2.0 * math.sqrt(pi)))]
    if degree >= 1:
        k1 = math.sqrt(3.0 / (4.0 * pi))
        out += [-k1 * y, k1 * z, -k1 * x]
    if degree >= 2:
        a = math.sqrt(15.0 / pi) / 2.0
        b = math.sqrt(5.0 / pi) / 4.0
        c = math.sqrt(15.0 / pi) / 4.0
        out += [a * x * y, -a * y * z, b * (2 * z * z - x * x - y * y),
                -a * x * z, c * (x * x - y * y)]
    if degree >= 3:
        a = math.sqrt(35.0 / (2.0 * pi)) / 4.0
        b = math.sqrt(105.0 / pi) / 2.0
        c = math.sqrt(21.0 / (2.0 * pi)) / 4.0
        e = math.sqrt(7.0 / pi) / 4.0
        f = math.sqrt(105.0 / pi) / 4.0
        out += [-a * y * (3 * x * x - y * y), b * x * y * z, -c * y * (4 * z * z - x * x - y * y),
                e * z * (2 * z * z - 3 * x * x - 3 * y * y), -c * x * (4 * z * z - x * x - y * y),
                f * z * (x * x - y * y), -a * x * (x * x - 3 * y * y)]
    return torch.stack(out, dim=1)


def _rot(q):
    w, x, y, z = q.unbind(1)
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], 1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], 1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], 1),
    ], 1)


def _project(means, log_scales, quats, opac, sh, w2c, cam, degree):
    W = w2c[:3, :3]
    t = w2c[:3, 3]
    p = means @ W.T + t
    z = p[:, 2]
    qn = quats.norm(dim=1, keepdim=True)
    q = quats / qn.clamp_min(1e-300)
    R = _rot(q)
    s = torch.exp(log_scales)
    M = R * s[:, None, :]
    Sig = M @ M.transpose(1, 2)
    fx, fy, cx, cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    zs = torch.where(z > 0, z, torch.ones_like(z))
    rx = p[:, 0] / zs
    ry = p[:, 1] / zs
    limx = 1.3 * cam.width / (2.0 * fx)
    limy = 1.3 * cam.height / (2.0 * fy)
    rxc = rx.clamp(-limx, limx)
    ryc = ry.clamp(-limy, limy)
    n = means.shape[0]
    zero = torch.zeros_like(zs)
    J = torch.stack([torch.stack([fx / zs, zero, -fx * rxc / zs], 1),
                     torch.stack([zero, fy / zs, -fy * ryc / zs], 1)], 1)
    Tm = J @ W
    cov = Tm @ Sig @ Tm.transpose(1, 2)
    a = cov[:, 0, 0] + 0.3
    b = cov[:, 0, 1]
    c = cov[:, 1, 1] + 0.3
    det = a * c - b * b
    dets = torch.where(det > 0, det, torch.ones_like(det))
    A, B, Cc = c / dets, -b / dets, a / dets
    u = fx * rx + cx
    v = fy * ry + cy
    campos = -(W.T @ t)
    dv = means - campos
    dirs = dv / dv.norm(dim=1, keepdim=True)
    Y = _sh_basis(degree, dirs)
    col = (sh * Y[:, :, None]).sum(1) + 0.5
    rgb = col.clamp_min(0.0)
    with torch.no_grad():
        o = opac
        ok = (z > cam.near) & (qn[:, 0] > 0) & (det > 0) & (o >= ALPHA_MIN)
        k2 = 2.0 * torch.log((255.0 * o).clamp_min(1e-300))
        ex = torch.sqrt((k2 * a).clamp_min(0))
        ey = torch.sqrt((k2 * c).clamp_min(0))
        x0 = torch.ceil(u - ex - 0.5).clamp_min(0)
        x1 = torch.floor(u + ex - 0.5).clamp_max(cam.width - 1)
        y0 = torch.ceil(v - ey - 0.5).clamp_min(0)
        y1 = torch.floor(v + ey - 0.5).clamp_max(cam.height - 1)
        ok &= (x0 <= x1) & (y0 <= y1)
    return dict(u=u, v=v, z=z, A=A, B=B, C=Cc, rgb=rgb, o=opac, ok=ok)


def _zkey(z):
    return np.asarray(z.detach().numpy(), np.float32).view(np.uint32)


def render(scene, cam, bg=(0.0, 0.0, 0.0), dL_dimg=None, chunk=2048) -> dict:
    """Forward (and with dL_dimg, autograd backward) of one view in float64."""
    dt = torch.float64
    leaves = dict(
        means=torch.tensor(np.asarray(scene.means, np.float64), dtype=dt),
        log_scales=torch.tensor(np.asarray(scene.log_scales, np.float64), dtype=dt),
        quats=torch.tensor(np.asarray(scene.quats, np.float64), dtype=dt),
        opacities=torch.tensor(np.asarray(scene.opacities, np.float64), dtype=dt),
        sh=torch.tensor(np.asarray(scene.sh, np.float64), dtype=dt),
        w2c=torch.tensor(np.asarray(cam.world_to_cam, np.float64), dtype=dt),
    )
    need = dL_dimg is not None
    for t in leaves.values():
        t.requires_grad_(need)
    pr = _project(leaves["means"], leaves["log_scales"], leaves["quats"], leaves["opacities"],
                  leaves["sh"], leaves["w2c"], cam, int(scene.sh_degree))
    idx = np.nonzero(pr["ok"].numpy())[0]
    zk = _zkey(pr["z"])[idx]
    order = idx[np.lexsort((idx, zk))]
    sel = torch.as_tensor(order, dtype=torch.long)
    u, v = pr["u"][sel], pr["v"][sel]
    A, B, Cc = pr["A"][sel], pr["B"][sel], pr["C"][sel]
    o, rgb = pr["o"][sel], pr["rgb"][sel]
    H, W = int(cam.height), int(cam.width)
    ys, xs = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    pxc = torch.tensor(xs.reshape(-1) + 0.5, dtype=dt)
    pyc = torch.tensor(ys.reshape(-1) + 0.5, dtype=dt)
    bgt = torch.tensor(np.asarray(bg, np.float64), dtype=dt)
    P = H * W
    img = np.zeros((P, 3))
    Tf = np.zeros(P)
    ncon = np.zeros(P, np.int64)
    g = None if dL_dimg is None else torch.tensor(np.asarray(dL_dimg, np.float64).reshape(P, 3))
    for s0 in range(0, P, chunk):
        s1 = min(P, s0 + chunk)
        dx = u[None, :] - pxc[s0:s1, None]
        dy = v[None, :] - pyc[s0:s1, None]
        sig = 0.5 * (A[None] * dx * dx + Cc[None] * dy * dy) + B[None] * dx * dy
        araw = o[None] * torch.exp(-sig)
        alpha = araw.clamp(max=ALPHA_MAX)
        with torch.no_grad():
            valid = (sig >= 0) & (alpha >= ALPHA_MIN)
            av = torch.where(valid, alpha, torch.zeros_like(alpha))
            Tb = torch.cumprod(torch.cat([torch.ones_like(av[:, :1]), 1 - av[:, :-1]], 1), 1)
            stop = valid & (Tb * (1 - av) < T_MIN)
            first = torch.where(stop.any(1), stop.to(torch.int8).argmax(1),
                                torch.full((s1 - s0,), stop.shape[1], dtype=torch.long))
            ar = torch.arange(stop.shape[1])[None, :]
            contrib = valid & (ar < first[:, None])
        ac = torch.where(contrib, alpha, torch.zeros_like(alpha))
        one_m = 1 - ac
        Tbefore = torch.cumprod(torch.cat([torch.ones_like(one_m[:, :1]), one_m[:, :-1]], 1), 1)
        wgt = ac * Tbefore
        col = wgt @ rgb
        Tfin = torch.prod(one_m, 1)
        out = col + Tfin[:, None] * bgt[None, :]
        img[s0:s1] = out.detach().numpy()
        Tf[s0:s1] = Tfin.detach().numpy()
        ncon[s0:s1] = contrib.sum(1).numpy()
        if g is not None:
            (out * g[s0:s1]).sum().backward(retain_graph=True)
    res = dict(img=img.reshape(H, W, 3), T=Tf.reshape(H, W), n_contributors=ncon.reshape(H, W))
    if g is not None:
        for k, t in leaves.items():
            res[k] = t.grad.numpy().copy() if t.grad is not None else np.zeros(t.shape)
    return res
