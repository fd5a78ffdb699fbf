"""GPU parity for the region of interest (only the rows [roi_y0, H) are rendered and
enter the loss, Sec. III-C image cropping) and for the scale regulariser L_scale."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2403_11577_amd import binding as B
from paper_2403_11577_amd import pipeline as pl

from gpu_util import compare_images, gpu_render, rel_close, say

pytestmark = pytest.mark.gpu


def _scene():
    return synth.small_drive(7, n_frames=2)   # 96 x 40 views


@pytest.mark.parametrize("tile, roi", [((16, 16), 20), ((16, 16), 23), ((8, 8), 23), ((16, 32), 31)])
def test_roi_render_vs_oracle_and_vs_full_render(tile, roi):
    say(f"case: roi render tile={tile} roi_y0={roi}")
    s = _scene()
    g = gpu_render(s, tile=tile, roi_y0=roi)
    full = gpu_render(s, tile=tile)
    w2c, _, _ = oracle.pose(s.traj, s.rig, s.xi, s.delta, s.views)
    orc = oracle.render(s.gauss, w2c, oracle.view_intr(s.rig, s.views), s.rig.W, s.rig.H,
                        oracle.Settings(roi_y0=roi), alternatives=True)
    nbad, nfl, nex, mx = compare_images(g, orc)
    say(f"  flagged={nfl} excluded={nex} max_err={mx:.3g} slots {g['slots']} vs {full['slots']}")
    assert nbad == 0 and g["status"] == 0
    # the region of interest is bitwise the full render; above it nothing is rendered
    assert np.array_equal(g["img"][:, :, roi:], full["img"][:, :, roi:])
    assert np.array_equal(g["T"][:, roi:], full["T"][:, roi:])
    assert np.array_equal(g["last_id"][:, roi:], full["last_id"][:, roi:])
    assert np.all(g["img"][:, :, :roi] == 0.0) and np.all(g["T"][:, :roi] == 1.0)
    assert np.all(g["last_pos"][:, :roi] == -1)
    assert g["inst"] < full["inst"]


def test_roi_tile_lists_vs_oracle():
    say("case: roi bin_sort")
    s, tile, roi = _scene(), (16, 16), 21
    w2c, _, _ = oracle.pose(s.traj, s.rig, s.xi, s.delta, s.views)
    g = gpu_render(s, tile=tile, w2c=w2c, roi_y0=roi)
    fr = g["frame"]
    ns, ni = g["slots"], g["inst"]
    vals = fr.sorted_vals(ni).cpu().numpy().astype(np.int64)
    meta = fr.meta(ns).cpu().numpy()
    ranges = fr.ranges().cpu().numpy().astype(np.int64)
    proj = oracle.project_all(s.gauss, w2c, oracle.view_intr(s.rig, s.views), s.rig.W, s.rig.H,
                              oracle.Settings(roi_y0=roi))
    T = int(fr.plan.tiles_per_view)
    for v in range(s.views.n):
        off, gid, margin = oracle.tile_lists(proj, s.rig.W, s.rig.H, tile[0], tile[1], view=v)
        mset = set(gid[margin])
        for t in range(T):
            a, b = ranges[v * T + t]
            mine = [int(x) for x in meta[vals[a:b], 0]] if b > a else []
            ref = [int(x) for x in gid[off[t]:off[t + 1]]]
            assert [x for x in mine if x not in mset] == [x for x in ref if x not in mset], (v, t)


@pytest.mark.parametrize("split_len, split_fwd, faint", [(0, 0, False), (64, 1, False), (64, 1, True)])
def test_roi_gradients_vs_oracle(split_len, split_fwd, faint):
    # also with the lists walked as chunks of 64 and the joined forward, which must leave the
    # rows above the region untouched (their pixels never composite)
    say(f"case: roi gradients split_len={split_len} split_fwd={split_fwd} faint={faint}")
    s, roi = _scene(), 19
    if faint:
        s.gauss.opacity = (s.gauss.opacity * np.float32(0.1)).astype(np.float32)
    w2c_ref, _, _ = oracle.pose(s.traj, s.rig, s.xi, s.delta, s.views)
    intr = oracle.view_intr(s.rig, s.views)
    target = oracle.render_scene(s, xi=s.xi_gt, delta=s.delta_gt)["img"]
    g = gpu_render(s, roi_y0=roi, split_len=split_len, split_fwd=split_fwd)
    if split_len:
        cnt = g["frame"].buf("counts", torch.int32, 8).cpu().numpy()
        assert int(cnt[4]) > int(cnt[3]) > 0  # lists were split
        orc_img = oracle.render(s.gauss, w2c_ref, intr, s.rig.W, s.rig.H, oracle.Settings(roi_y0=roi),
                                alternatives=True)
        nbad, _, _, _ = compare_images(g, orc_img)
        assert nbad == 0
        assert np.all(g["T"][:, :roi] == 1.0) and np.all(g["last_pos"][:, :roi] == -1)
    mset = oracle.Settings(margin=1e-2, roi_y0=roi)
    orc = oracle.render(s.gauss, w2c_ref, intr, s.rig.W, s.rig.H, mset)
    mask = (orc["nflag"] > 0) | (orc["kink"] > 0)
    _, dimg = oracle.l1_loss(orc["img"], target, mask, roi_y0=roi)
    gr = pl.alloc_grads(g["ds"], with_mean=True)
    pl.backward(g["frame"], g["ds"], g["xi"], g["delta"], torch.as_tensor(dimg, dtype=torch.float32, device="cuda"), gr)
    torch.cuda.synchronize()
    ref = oracle.grad(s.gauss, w2c_ref, intr, s.rig.W, s.rig.H, dimg.astype(np.float32).astype(np.float64),
                      oracle.Settings(roi_y0=roi), mask=mask.astype(np.int8))
    rxi, rdl = oracle.pose_bwd(s.traj, s.rig, s.xi, s.delta, s.views, ref["w2c"])
    for name in ("quat", "scale", "opacity", "color", "mean", "w2c"):
        ok, err = rel_close(getattr(gr, name).cpu().numpy(), ref[name], 1e-3)
        say(f"  {name} {err:.2e}")
        assert ok, (name, err)
    for name, a, b in (("xi", gr.xi.cpu().numpy(), rxi), ("delta", gr.delta.cpu().numpy(), rdl)):
        e = float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-12)))
        say(f"  {name} {e:.2e}")
        assert e <= 1e-3


def test_roi_l1_kernel_vs_oracle():
    say("case: roi l1")
    rng = np.random.default_rng(3)
    V, H, W, roi = 3, 37, 50, 13
    img = rng.uniform(size=(V, 3, H, W)).astype(np.float32)
    tgt = rng.uniform(size=(V, 3, H, W)).astype(np.float32)
    tgt[0, 1, 20, 5] = img[0, 1, 20, 5]                   # a zero difference inside the region
    loss, dimg = pl.l1_loss_grad(torch.as_tensor(img, device="cuda"), torch.as_tensor(tgt, device="cuda"),
                                 roi_y0=roi)
    L, g = oracle.l1_loss(img.astype(np.float64), tgt.astype(np.float64), roi_y0=roi)
    assert float(loss.item()) == pytest.approx(L, rel=1e-6)
    np.testing.assert_array_equal(dimg.cpu().numpy(), g.astype(np.float32))


def test_scale_reg_kernel_vs_oracle():
    say("case: scale regulariser")
    rng = np.random.default_rng(4)
    G = 10007
    sc = np.exp(rng.normal(np.log(0.1), 0.5, size=(3, G))).astype(np.float32)
    sc[:, :100] = sc[0, :100]            # isotropic ones: exactly zero gradient
    sc[1, 100:200] = sc[0, 100:200]      # two equal axes
    lam = 1e-3
    dsc = torch.zeros((3, G), dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    st = torch.as_tensor(sc, device="cuda")
    B.splat_scale_reg(st, lam, dsc, loss)
    L, g = oracle.scale_reg(sc.astype(np.float64), lam)
    assert float(loss.item()) == pytest.approx(L, rel=1e-12)
    once = dsc.cpu().numpy()
    np.testing.assert_array_equal(once, g.astype(np.float32))   # float64 signs and mean, one rounding
    assert np.all(once[:, :100] == 0.0)
    B.splat_scale_reg(st, lam, dsc, None)                          # accumulates
    np.testing.assert_array_equal(dsc.cpu().numpy(), 2 * once)
