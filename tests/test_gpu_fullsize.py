"""Parity at the full benchmark sizes, in the launch configuration bench.py
times: the GPU renders and differentiates the whole 1920x1080 view; the FP64
oracle computes a random sample of tiles exactly (its tile-mask mode, pinned
against the full render on the CPU).  The upstream gradient is non-zero only on
the sampled tiles, so the oracle's parameter and pose gradients are exact for
the whole scene and are compared tensor by tensor.  The pair count is compared
with the oracle's FP64 projection of every Gaussian."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2607_14481_amd import scenes as S

from ._util import GRAD_KEYS, gpu_render, log, oracle_bin_from_gpu_state, rel_err

pytestmark = pytest.mark.gpu


def _sampled_parity(wl, n_tiles, seed, bg=(0.0, 0.0, 0.0)):
    sc, cam = wl.scene, wl.cameras[0]
    tx, ty = O.tile_grid(cam)
    rng = np.random.default_rng(seed)
    mask = np.zeros(tx * ty, np.uint8)
    mask[rng.choice(tx * ty, n_tiles, replace=False)] = 1
    pix = np.zeros((cam.height, cam.width), bool)
    for t in np.nonzero(mask)[0]:
        pix[(t // tx) * 16:(t // tx + 1) * 16, (t % tx) * 16:(t % tx + 1) * 16] = True
    up = S.random_upstream(seed, (cam.height, cam.width, 3)) * pix[..., None]
    log(f"{wl.name}: GPU fwd+bwd n={sc.n} {cam.width}x{cam.height}")
    gpu = gpu_render(sc, [cam], bg=bg, upstream=[up])
    log(f"{wl.name}: oracle on {n_tiles} tiles")
    ref = O.render(sc, cam, bg=bg, dL_dimg=up, tile_mask=mask)
    amb = ref["ambig"] & pix
    d = np.abs(gpu["imgs"][0].astype(np.float64) - ref["img"])
    ok = pix & ~amb
    worst = float(d[ok].max())
    log(f"{wl.name}: max|d img| over {ok.sum()} sampled px = {worst:.3e}; ambiguous {int(amb.sum())}")
    assert worst <= 1e-4
    for k in GRAD_KEYS:
        e = rel_err(gpu[k], ref[k])
        log(f"{wl.name}: rel err d{k} = {e:.3e}")
        assert e <= 1e-3
    ew = rel_err(gpu["w2c"][0], ref["w2c"])
    et = rel_err(gpu["twist"][0], ref["twist"])
    log(f"{wl.name}: rel err pose 4x4 {ew:.3e}, twist {et:.3e}")
    assert ew <= 1e-3 and et <= 1e-3
    pr = O.project(sc, cam)
    m_ref = int(((pr["trect"][:, 2] - pr["trect"][:, 0] + 1) * (pr["trect"][:, 3] - pr["trect"][:, 1] + 1))[pr["visible"]].sum())
    log(f"{wl.name}: pairs gpu {gpu['stats']['pairs']} oracle {m_ref}; visible gpu {gpu['stats']['visible']} "
        f"oracle {int(pr['visible'].sum())}")
    assert gpu["stats"]["pairs"] == m_ref
    assert gpu["stats"]["visible"] == int(pr["visible"].sum())


def test_headline_1080p_1M_sampled_parity():
    _sampled_parity(S.headline_view(), n_tiles=24, seed=101)


def test_headline_1080p_1M_binning_bit_exact():
    """The whole tile list of the benchmark view (5M+ pairs, lists up to ~2000
    entries) against the oracle's integer binning fed the GPU's boxes and
    depth bits."""
    wl = S.headline_view()
    sc, cams = wl.scene, wl.cameras
    st = gpu_render(sc, cams, export=True)["state"]
    tiles, items, ranges = oracle_bin_from_gpu_state(st, cams, sc.n)
    lens = ranges[:, 1].astype(np.int64) - ranges[:, 0]
    log(f"headline binning: M gpu={st['M']} oracle={len(tiles)}; longest list {int(lens.max())}")
    assert st["M"] == len(tiles)
    np.testing.assert_array_equal(st["pair_tiles"].astype(np.uint64), tiles)
    np.testing.assert_array_equal(st["pair_items"].astype(np.uint64), items)


def test_single_view_1080p_200k_sampled_parity():
    _sampled_parity(S.single_view_1080p(), n_tiles=24, seed=102, bg=(0.1, 0.1, 0.1))


def test_lod_cut_1080p_sampled_parity():
    from paper_2607_14481_amd import hierarchy
    wl = hierarchy.lod_workload()
    log(f"lod cut: {wl.meta}")
    _sampled_parity(wl, n_tiles=24, seed=103)
