"""GPU parity of every stage of the HIP path against the FP64 CPU oracle.

Bars: float64 poses to 1e-12; depth keys, visibility, tile lists and sort order
bit-exact (Gaussians whose footprint edge sits on a rounding step excepted);
images within 1e-4 per channel and last contributors bit-exact, with the
oracle's alternatives at threshold-margin pixels; gradients within 1e-3
relative.  All through the C ABI.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2403_11577_amd import binding as B
from paper_2403_11577_amd import pipeline as pl

from gpu_util import use_instance_sort, compare_images, gpu_render, rel_close, say

pytestmark = pytest.mark.gpu

TILES = [(16, 16), (8, 8), (16, 32), (32, 16)]


def _dev(a, dt=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def test_library_loads_and_abi_matches():
    say("case: abi")
    assert B.splat_version().startswith("splat")


@pytest.mark.parametrize("seed", [0, 1])
def test_pose_fwd_bwd_vs_oracle(seed):
    say(f"case: pose seed={seed}")
    s = synth.small_drive(seed, n_frames=3)
    ds = pl.DeviceScene.from_scene(s)
    xi, dl = _dev(s.xi), _dev(s.delta)
    w2c = torch.empty((s.views.n, 12), dtype=torch.float64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    B.splat_pose_interp_fwd(ds.knot_t, ds.knot_q, ds.knot_p, ds.R0, ds.t0, xi, dl, ds.view_cam, ds.view_t,
                            w2c, status)
    ref, _, _ = oracle.pose(s.traj, s.rig, s.xi, s.delta, s.views)
    np.testing.assert_allclose(w2c.cpu().numpy(), ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    assert int(status.item()) == 0
    G = np.random.default_rng(seed).normal(size=(s.views.n, 12))
    dxi = torch.zeros((2, 6), dtype=torch.float64, device="cuda")
    ddl = torch.zeros(2, dtype=torch.float64, device="cuda")
    B.splat_pose_interp_bwd(ds.knot_t, ds.knot_q, ds.knot_p, ds.R0, ds.t0, xi, dl, ds.view_cam, ds.view_t,
                            _dev(G), dxi, ddl)
    rxi, rdl = oracle.pose_bwd(s.traj, s.rig, s.xi, s.delta, s.views, G)
    np.testing.assert_allclose(dxi.cpu().numpy(), rxi, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(ddl.cpu().numpy(), rdl, rtol=1e-10, atol=1e-12)


def test_pose_extrapolation_flag():
    say("case: pose extrapolation")
    s = synth.small_drive(0, n_frames=1)
    ds = pl.DeviceScene.from_scene(s)
    vt = torch.tensor([s.traj.t[-1] + 0.3, s.traj.t[0] - 0.2], dtype=torch.float64, device="cuda")
    cam = torch.tensor([0, 1], dtype=torch.int32, device="cuda")
    w2c = torch.empty((2, 12), dtype=torch.float64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    B.splat_pose_interp_fwd(ds.knot_t, ds.knot_q, ds.knot_p, ds.R0, ds.t0, _dev(s.xi), _dev(s.delta), cam, vt,
                            w2c, status)
    views = synth.Views(np.array([0, 1], np.int32), vt.cpu().numpy())
    ref, _, _ = oracle.pose(s.traj, s.rig, s.xi, s.delta, views)
    np.testing.assert_allclose(w2c.cpu().numpy(), ref, atol=1e-9)
    assert int(status.item()) & B.ST_EXTRAPOLATED


def _project_check(scene, tile):
    w2c, _, _ = oracle.pose(scene.traj, scene.rig, scene.xi, scene.delta, scene.views)
    intr = oracle.view_intr(scene.rig, scene.views)
    W, H = scene.rig.W, scene.rig.H
    g = gpu_render(scene, tile=tile, w2c=w2c)
    fr = g["frame"]
    ns, ni = g["slots"], g["inst"]
    proj = oracle.project_all(scene.gauss, w2c, intr, W, H)
    meta = fr.meta(ns).cpu().numpy()
    rec = fr.records(ns).cpu().numpy()
    view_off = fr.buf("view_off", torch.int32, scene.views.n + 1).cpu().numpy()
    for v in range(scene.views.n):
        sl = slice(view_off[v], view_off[v + 1])
        gids = meta[sl, 0]
        assert np.all(meta[sl, 1] == v)
        assert np.all(np.diff(gids) > 0)  # compaction keeps Gaussian order
        vis = np.nonzero(proj["cull"][v] == 0)[0]
        rm = proj["rect_margin"][v].astype(bool)
        assert set(gids) ^ set(vis) <= set(np.nonzero(rm)[0])
        common = np.intersect1d(gids, vis)
        idx = np.searchsorted(gids, common)
        r = rec[sl][idx]
        # depth key: bit-exact by specification
        assert np.array_equal(r[:, 11].view(np.uint32), proj["depth32"][v][common].view(np.uint32))
        mu = r[:, 0:2].astype(np.float64) + r[:, 2:4].astype(np.float64)
        np.testing.assert_allclose(mu, proj["mu"][v][common], rtol=0, atol=1e-5)
        np.testing.assert_allclose(r[:, 4:7], proj["conic"][v][common], rtol=2e-6,
                                   atol=2e-6 * np.abs(proj["conic"][v][common]).max())
    return g, proj, w2c


@pytest.mark.parametrize("tile", [(16, 16), (8, 8)])
def test_project_vs_oracle(tile):
    say(f"case: project tile={tile}")
    _project_check(synth.tiny_scene(0), tile)
    _project_check(synth.small_drive(1, n_frames=2), tile)


def _edge_scene(seed, n=3000, roi_y0=0):
    """Small, faint Gaussians whose means project within a few pixels of the image borders
    (and of the first row of the region of interest): the projection's visibility test is
    decided there by its exact float64 path or by its float32 bounds, and the opacities span
    the value below which a footprint's half-width can fall under half a pixel."""
    s = synth.tiny_scene(seed)
    rng = np.random.default_rng(seed)
    W, H = s.rig.W, s.rig.H
    fx, fy, cx, cy = s.rig.intr[0]
    u = rng.uniform(-3.0, 3.0, n)
    v = rng.uniform(-3.0, 3.0, n)
    side = rng.integers(0, 4, n)
    u = np.where(side == 1, W + u, u)                       # left / right edges
    ys = rng.choice([0.0, float(H), float(roi_y0)], n)
    v = np.where(side >= 2, ys + v, rng.uniform(0, H, n))   # top / bottom / region-of-interest row
    u = np.where(side >= 2, rng.uniform(0, W, n), u)
    z = rng.uniform(2.0, 20.0, n)
    mean = np.stack([(u - cx) / fx * z, (v - cy) / fy * z, z])
    g = s.gauss.subset(np.arange(n) % s.gauss.n)
    g.mean = mean.astype(np.float32)
    g.scale = np.exp(rng.uniform(np.log(1e-4), np.log(0.05), size=(3, n))).astype(np.float32)
    g.opacity = (rng.choice([1.0, 1.1, 1.25, 1.3, 1.35, 1.5, 3.0, 50.0, 250.0], n) / 255.0).astype(np.float32)
    s.gauss = g
    return s


@pytest.mark.parametrize("pad_px, roi_y0", [(0.1, 0), (0.6, 0), (0.1, 23)])
def test_projection_visibility_at_image_edges(pad_px, roi_y0):
    """Pairs whose footprints touch the image border: the visible set, the float32 depth
    and the float64 mean and conic match the oracle, whichever test decided visibility."""
    say(f"case: projection at the image edges pad_px={pad_px} roi_y0={roi_y0}")
    scene = _edge_scene(3, roi_y0=roi_y0)
    w2c, _, _ = oracle.pose(scene.traj, scene.rig, scene.xi, scene.delta, scene.views)
    intr = oracle.view_intr(scene.rig, scene.views)
    W, H = scene.rig.W, scene.rig.H
    ds = pl.DeviceScene.from_scene(scene)
    xi = torch.as_tensor(scene.xi, dtype=torch.float64, device="cuda")
    dl = torch.as_tensor(scene.delta, dtype=torch.float64, device="cuda")
    w2c_t = torch.as_tensor(np.ascontiguousarray(w2c), dtype=torch.float64, device="cuda")
    st = pl.make_settings(tile=(16, 16), pad_px=pad_px, roi_y0=roi_y0)
    fr = pl.fit_frame(ds, xi, dl, st, w2c=w2c_t)
    pl.forward(fr, ds, xi, dl, w2c=w2c_t)
    torch.cuda.synchronize()
    ns, _ = fr.counts()
    meta = fr.meta(ns).cpu().numpy()
    rec = fr.records(ns).cpu().numpy()
    proj = oracle.project_all(scene.gauss, w2c, intr, W, H, oracle.Settings(pad_px=pad_px, roi_y0=roi_y0))
    gids = meta[:, 0]
    vis = np.nonzero(proj["cull"][0] == 0)[0]
    rm = set(np.nonzero(proj["rect_margin"][0])[0])
    say(f"  visible {len(gids)} of {scene.gauss.n} (oracle {len(vis)}, {len(rm)} at a rounding step)")
    assert 200 < len(vis) < scene.gauss.n - 200   # both kinds of pair are present
    assert set(gids) ^ set(vis) <= rm
    common = np.intersect1d(gids, vis)
    idx = np.searchsorted(gids, common)
    r = rec[idx]
    assert np.array_equal(r[:, 11].view(np.uint32), proj["depth32"][0][common].view(np.uint32))
    mu = r[:, 0:2].astype(np.float64) + r[:, 2:4].astype(np.float64)
    np.testing.assert_allclose(mu, proj["mu"][0][common], rtol=0, atol=1e-5)
    np.testing.assert_allclose(r[:, 4:7], proj["conic"][0][common], rtol=2e-6,
                               atol=2e-6 * np.abs(proj["conic"][0][common]).max())


@pytest.mark.parametrize("path", ["slot_first", "instance_keys"])
@pytest.mark.parametrize("tile", TILES)
def test_bin_sort_vs_oracle(tile, path):
    say(f"case: bin_sort tile={tile} path={path}")
    scene = synth.small_drive(2, n_frames=2)
    g, proj, w2c = _project_check(scene, tile)
    fr = g["frame"]
    assert int(fr.plan.slot_sort) == 1  # the default where the payload fits 64 bits
    if path == "instance_keys":
        use_instance_sort(fr)
        pl.forward(fr, g["ds"], g["xi"], g["delta"], w2c=torch.as_tensor(w2c, device="cuda"))
        torch.cuda.synchronize()
        assert fr.status() == 0
    ns, ni = fr.counts()
    assert (ns, ni) == (g["slots"], g["inst"])
    vals = fr.sorted_vals(ni).cpu().numpy().astype(np.int64)
    meta = fr.meta(ns).cpu().numpy()
    ranges = fr.ranges().cpu().numpy().astype(np.int64)
    # the lists tile the sorted instances in (view, tile) order, each instance once
    nz = ranges[ranges[:, 1] > ranges[:, 0]]
    assert nz[0, 0] == 0 and nz[-1, 1] == ni and np.all(nz[1:, 0] == nz[:-1, 1])
    if path == "instance_keys":  # the per-slot tile counts were scanned in place to instance offsets
        per_slot = np.diff(fr.buf("ntiles", torch.int32, ns + 1).cpu().numpy().astype(np.int64))
    else:  # every slot payload (slot | first tile | w - 1 | h - 1), in the order a sort pass left
        pay = fr.buf("spay", torch.int64, ns).cpu().numpy().view(np.uint64)
        b0, b1, b2 = (int(x) for x in fr.plan.pack_bits)
        s1 = b0 + int(fr.plan.tile_bits)
        field = lambda sh, b: (pay >> np.uint64(sh)) & np.uint64((1 << b) - 1) if sh < 64 else np.zeros_like(pay)
        slot_of = field(0, b0).astype(np.int64)
        assert np.array_equal(np.sort(slot_of), np.arange(ns))
        per_slot = np.zeros(ns, np.int64)
        per_slot[slot_of] = ((field(s1, b1) + np.uint64(1)) * (field(s1 + b1, b2) + np.uint64(1))).astype(np.int64)
    assert per_slot.sum() == ni and np.array_equal(np.bincount(vals, minlength=ns), per_slot)
    # the sorted keys are the (view, tile) of every instance
    keys = fr.sorted_keys(ni).cpu().numpy().astype(np.int64)
    if int(fr.plan.key_shift) >= 0:
        tile_of = keys >> (int(fr.plan.depth_bits) - int(fr.plan.key_shift))
    else:
        tile_of = keys >> int(fr.plan.depth_bits)
    for t in np.nonzero(ranges[:, 1] > ranges[:, 0])[0][:: 7]:
        assert np.all(tile_of[ranges[t, 0]:ranges[t, 1]] == t)
    T = int(fr.plan.tiles_per_view)
    W, H = scene.rig.W, scene.rig.H
    for v in range(scene.views.n):
        off, gid, margin = oracle.tile_lists(proj, W, H, tile[0], tile[1], view=v)
        mset = set(gid[margin])
        for t in range(T):
            a, b = ranges[v * T + t]
            mine = [int(x) for x in meta[vals[a:b], 0]] if b > a else []
            ref = [int(x) for x in gid[off[t]:off[t + 1]]]
            if mset:
                mine = [x for x in mine if x not in mset]
                ref = [x for x in ref if x not in mset]
            assert mine == ref, (v, t)


@pytest.mark.parametrize("tile", [(16, 16), (32, 16)])
@pytest.mark.parametrize("path", ["slot_first", "instance_keys"])
def test_bin_sort_long_lists_vs_oracle(tile, path):
    """Tile lists far longer than one radix-sort tile of 4096 keys: 40,000 small Gaussians in
    front of a 64x32 camera put 5,000-10,000 instances in a tile; every list must still be the
    oracle's (depth32, Gaussian id) order, and the image its image, with either bin sort."""
    say(f"case: bin_sort long lists tile={tile} path={path}")
    scene = synth.tiny_scene(9, n=40000, W=64, H=32, f=10.0)
    g, proj, w2c = _project_check(scene, tile)
    fr = g["frame"]
    if path == "instance_keys":
        use_instance_sort(fr)
        img, T, last = pl.forward(fr, g["ds"], g["xi"], g["delta"], w2c=torch.as_tensor(w2c, device="cuda"))
        torch.cuda.synchronize()
        assert fr.status() == 0
        g = dict(g, img=img.cpu().numpy().astype(np.float64), T=T.cpu().numpy().astype(np.float64))
        lastp = last.cpu().numpy().astype(np.int64)
        vals0 = fr.sorted_vals(g["inst"]).cpu().numpy().astype(np.int64)
        meta0 = fr.meta(g["slots"]).cpu().numpy()
        gid = np.full(lastp.shape, -1, np.int64)
        gid[lastp >= 0] = meta0[vals0[lastp[lastp >= 0]], 0]
        g["last_pos"], g["last_id"] = lastp, gid
    ns, ni = g["slots"], g["inst"]
    vals = fr.sorted_vals(ni).cpu().numpy().astype(np.int64)
    meta = fr.meta(ns).cpu().numpy()
    ranges = fr.ranges().cpu().numpy().astype(np.int64)
    L = ranges[:, 1] - ranges[:, 0]
    say(f"  list lengths: max {L.max()}, lists over 4096: {int((L > 4096).sum())} of {L.size}")
    assert L.max() > 2 * 4096
    off, gid, margin = oracle.tile_lists(proj, scene.rig.W, scene.rig.H, tile[0], tile[1], view=0)
    mset = set(gid[margin])
    for t in range(int(fr.plan.tiles_per_view)):
        a, b = ranges[t]
        mine = [int(x) for x in meta[vals[a:b], 0] if int(x) not in mset]
        ref = [int(x) for x in gid[off[t]:off[t + 1]] if int(x) not in mset]
        assert mine == ref, t
    orc = oracle.render(scene.gauss, w2c, oracle.view_intr(scene.rig, scene.views), scene.rig.W, scene.rig.H,
                        alternatives=True)
    nbad, nfl, nex, mx = compare_images(g, orc)
    assert nbad == 0 and nex <= 0.001 * orc["nflag"].size


SCENES = {
    "tiny": lambda: synth.tiny_scene(0),
    "tiny_ragged": lambda: synth.tiny_scene(4, n=700, W=100, H=37, f=80.0),
    "small_drive": lambda: synth.small_drive(3, n_frames=2),
}


@pytest.mark.parametrize("name", list(SCENES))
@pytest.mark.parametrize("tile", TILES)
def test_render_fwd_vs_oracle(name, tile):
    say(f"case: render_fwd scene={name} tile={tile}")
    scene = SCENES[name]()
    g = gpu_render(scene, tile=tile)
    ref_w2c, _, _ = oracle.pose(scene.traj, scene.rig, scene.xi, scene.delta, scene.views)
    orc = oracle.render(scene.gauss, ref_w2c, oracle.view_intr(scene.rig, scene.views), scene.rig.W,
                        scene.rig.H, alternatives=True)
    np.testing.assert_allclose(g["w2c"], ref_w2c, atol=1e-12 * np.abs(ref_w2c).max())
    nbad, nfl, nex, mx = compare_images(g, orc)
    say(f"  flagged={nfl} excluded={nex} max_err={mx:.3g} slots={g['slots']} inst={g['inst']}")
    assert g["status"] == 0
    assert nbad == 0
    assert nex <= 0.001 * orc["nflag"].size


def test_render_invariant_across_launch_shapes():
    say("case: launch-shape invariance")
    scene = synth.small_drive(4, n_frames=2)
    base = gpu_render(scene, tile=(16, 16), batch=64, persistent=True)
    for tile in TILES:
        for batch in (32, 64, 128, 256):
            for pers in (True, False):
                o = gpu_render(scene, tile=tile, batch=batch, persistent=pers)
                assert np.array_equal(o["img"], base["img"]), (tile, batch, pers)
                assert np.array_equal(o["T"], base["T"])
                assert np.array_equal(o["last_id"], base["last_id"])


def _read_blend_masks(o):
    """The blend masks the adjoint reads: in every tile list, the instances up to the last
    contributor of any pixel of the tile (the forward leaves the rest of a list unwritten once
    every pixel of the tile has stopped)."""
    fr = o["frame"]
    V, H, W = o["T"].shape
    TW, TH = int(fr.plan.s.tile_w), int(fr.plan.s.tile_h)
    tx_n, nt = int(fr.plan.tiles_x), int(fr.plan.tiles_per_view)
    rg = fr.ranges().cpu().numpy().astype(np.int64)
    lp = o["last_pos"]
    yy, xx = np.mgrid[0:H, 0:W]
    tile = (yy // TH) * tx_n + xx // TW
    maxlp = np.full(V * nt, -1, np.int64)
    for v in range(V):
        np.maximum.at(maxlp, v * nt + tile.ravel(), lp[v].ravel())
    bm = fr.buf("bmask", torch.uint8, int(o["inst"])).cpu().numpy()
    pos = np.arange(bm.size)
    owner = np.repeat(np.arange(rg.shape[0]), np.maximum(rg[:, 1] - rg[:, 0], 0))
    starts = np.repeat(rg[:, 0], np.maximum(rg[:, 1] - rg[:, 0], 0))
    assert np.array_equal(starts + (pos - np.repeat(np.cumsum(np.maximum(rg[:, 1] - rg[:, 0], 0)) -
                                                    np.maximum(rg[:, 1] - rg[:, 0], 0),
                                                    np.maximum(rg[:, 1] - rg[:, 0], 0))), pos)
    return np.where(pos <= maxlp[owner], bm, 0)


@pytest.mark.parametrize("split_len, split_fwd", [(64, 0), (64, 1), (256, 1)])
def test_batch_size_invariance_with_split_lists(split_len, split_fwd):
    """Gaussians per LDS batch (32, 64, 128, 256; at most the split length) change only the
    staging: images, T and last ids are bitwise those of batch 64 (also for lists split into
    chunks and joined), the blend masks the adjoint reads are the same, and the gradients agree
    to float-atomic ordering."""
    say(f"case: batch invariance, split_len={split_len} split_fwd={split_fwd}")
    scene = synth.small_drive(4, n_frames=2)
    outs = {}
    for batch in (64, 32, 128, 256):
        o = gpu_render(scene, tile=(8, 8), batch=batch, persistent=False, split_len=split_len,
                       split_fwd=split_fwd)
        fr = o["frame"]
        dimg = torch.as_tensor(np.sign(o["img"] - 0.4).astype(np.float32) * 1e-3, device="cuda")
        gr = pl.alloc_grads(o["ds"])
        pl.backward(fr, o["ds"], o["xi"], o["delta"], dimg, gr)
        torch.cuda.synchronize()
        outs[batch] = (o, _read_blend_masks(o),
                       {n: getattr(gr, n).cpu().numpy() for n in ("quat", "scale", "opacity", "color", "xi", "delta")})
    ref, ref_bm, ref_g = outs[64]
    for batch, (o, bm, g) in outs.items():
        assert np.array_equal(o["img"], ref["img"]), batch
        assert np.array_equal(o["T"], ref["T"]), batch
        assert np.array_equal(o["last_id"], ref["last_id"]), batch
        assert np.array_equal(bm, ref_bm), batch
        for n in g:
            ok, err = rel_close(g[n], ref_g[n], 1e-5)
            assert ok, (batch, n, err)


def _grad_case(scene, tile, seed=0, split_len=0, persistent=True, keep=None, split_fwd=0):
    w2c_ref, _, _ = oracle.pose(scene.traj, scene.rig, scene.xi, scene.delta, scene.views)
    target = oracle.render_scene(scene, xi=scene.xi_gt, delta=scene.delta_gt)["img"]
    g = gpu_render(scene, tile=tile, split_len=split_len, persistent=persistent, split_fwd=split_fwd)
    if keep is not None:
        keep["render"] = g
    fr, ds = g["frame"], g["ds"]
    # pixels with a threshold decision or an alpha_max kink near the margin are left out on both sides
    mset = oracle.Settings(margin=1e-2)
    orc_m = oracle.render(scene.gauss, w2c_ref, oracle.view_intr(scene.rig, scene.views), scene.rig.W,
                          scene.rig.H, mset)
    mask = (orc_m["nflag"] > 0) | (orc_m["kink"] > 0)
    # dL/dimg from the oracle's own image, handed to both sides
    L, dimg = oracle.l1_loss(orc_m["img"], target, mask)
    gr = pl.alloc_grads(ds, with_mean=True)
    pl.backward(fr, ds, g["xi"], g["delta"], torch.as_tensor(dimg, dtype=torch.float32, device="cuda"), gr)
    torch.cuda.synchronize()
    ref = oracle.grad(scene.gauss, w2c_ref, oracle.view_intr(scene.rig, scene.views), scene.rig.W, scene.rig.H,
                      dimg.astype(np.float32).astype(np.float64), mask=mask.astype(np.int8))
    rxi, rdl = oracle.pose_bwd(scene.traj, scene.rig, scene.xi, scene.delta, scene.views, ref["w2c"])
    out = {}
    if keep is not None:
        keep["grads"] = {n: getattr(gr, n).cpu().numpy() for n in ("quat", "scale", "opacity", "color", "mean", "w2c")}
    for name in ("quat", "scale", "opacity", "color", "mean"):
        ok, err = rel_close(getattr(gr, name).cpu().numpy(), ref[name], 1e-3)
        out[name] = (ok, err)
    ok, err = rel_close(gr.w2c.cpu().numpy(), ref["w2c"], 1e-3, floor_frac=0)
    out["w2c"] = (ok, err)
    for name, a, b in (("xi", gr.xi.cpu().numpy(), rxi), ("delta", gr.delta.cpu().numpy(), rdl)):
        e = float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-12)))
        out[name] = (e <= 1e-3, e)
    return out, float(mask.mean())


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (16, 32)])
def test_gradients_vs_oracle(tile):
    say(f"case: gradients tile={tile}")
    out, mfrac = _grad_case(synth.small_drive(5, n_frames=2), tile)
    say("  masked frac %.4f " % mfrac + " ".join(f"{k}={v[1]:.2e}" for k, v in out.items()))
    for k, (ok, err) in out.items():
        assert ok, (k, err)


@pytest.mark.parametrize("jitter", [0.8, 1.2])
def test_gradients_thin_rotated_gaussians_vs_oracle(jitter):
    """Thin, randomly rotated footprints (per-axis scales times exp(N(0, jitter)), axis ratios up
    to about 100 and 900 here) are where the 2-D covariance is nearly singular and the conic's adjoint
    amplifies rounding most; every gradient still meets the 1e-3 bar against the float64 oracle.
    This is what keeps the projection adjoint's chain rule in float64: in float32 (the
    projection still formed in float64) the quaternion and mean gradients of this scene were off
    by 1.4e-3 and 3.8e-3."""
    say(f"case: gradients of thin rotated Gaussians, jitter {jitter}")
    scene = synth.anisotropic(synth.small_drive(5, n_frames=2), seed=11, jitter=jitter)
    g = scene.gauss
    ratio = (g.scale.max(axis=0) / g.scale.min(axis=0)).astype(np.float64)
    say(f"  axis ratio median {np.median(ratio):.1f}, max {ratio.max():.1f}")
    out, mfrac = _grad_case(scene, (16, 16))
    say("  masked frac %.4f " % mfrac + " ".join(f"{k}={v[1]:.2e}" for k, v in out.items()))
    for k, (ok, err) in out.items():
        assert ok, (k, err)


@pytest.mark.parametrize("tile, persistent", [((16, 16), True), ((8, 8), True), ((16, 16), False), ((8, 8), False)])
def test_gradients_split_lists_vs_oracle(tile, persistent):
    # every tile list of 64 instances or more is walked by the adjoint as chunks of 64, each
    # started from the forward's checkpoint where the next chunk starts
    say(f"case: gradients with split lists tile={tile} persistent={persistent}")
    scene = synth.small_drive(5, n_frames=2)
    kept, base = {}, {}
    out, _ = _grad_case(scene, tile, split_len=64, persistent=persistent, keep=kept)
    fr = kept["render"]["frame"]
    cnt = fr.buf("counts", torch.int32, 8).cpu().numpy()
    nT = fr.plan.n_views * fr.plan.tiles_per_view
    rg = fr.buf("ranges", torch.int32, 2 * nT).view(nT, 2).cpu().numpy().astype(np.int64)
    L = rg[:, 1] - rg[:, 0]
    nsplit, nchunk, nitems = int(cnt[3]), int(cnt[4]), int(cnt[5])
    say(f"  split lists {nsplit}, chunks {nchunk}, adjoint items {nitems}, longest list {L.max()}")
    assert nsplit == int((L >= 64).sum()) and nsplit > 0
    assert nchunk == int(((L[L >= 64] + 63) // 64).sum())
    assert nitems == nchunk + nT - nsplit
    say("  " + " ".join(f"{k}={v[1]:.2e}" for k, v in out.items()))
    for k, (ok, err) in out.items():
        assert ok, (k, err)
    # the same adjoint without splitting: the forward is identical, the gradients agree to rounding
    _grad_case(scene, tile, split_len=1 << 24, persistent=persistent, keep=base)
    for k in ("img", "T", "last_id"):
        assert np.array_equal(kept["render"][k], base["render"][k]), k
    for k, a in kept["grads"].items():
        b = base["grads"][k]
        err = float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))
        say(f"  split vs unsplit {k}: {err:.2e}")
        assert err <= 1e-4, (k, err)


def _faint(scene, factor=0.1):
    # the regime at the start of a calibration: faint Gaussians, few pixels reach t_min
    scene.gauss.opacity = (scene.gauss.opacity * np.float32(factor)).astype(np.float32)
    return scene


@pytest.mark.parametrize("faint", [False, True])
@pytest.mark.parametrize("tile, persistent", [((16, 16), True), ((8, 8), False), ((16, 32), True)])
def test_render_joined_chunks_vs_oracle(tile, persistent, faint):
    # chunks of 64 composited on their own and joined per pixel, or walked in order where a
    # pixel could reach t_min: the same images, T and last contributors as the oracle
    say(f"case: joined chunks tile={tile} persistent={persistent} faint={faint}")
    scene = synth.small_drive(6, n_frames=2)
    if faint:
        scene = _faint(scene)
    g = gpu_render(scene, tile=tile, persistent=persistent, split_len=64, split_fwd=1)
    ref_w2c, _, _ = oracle.pose(scene.traj, scene.rig, scene.xi, scene.delta, scene.views)
    orc = oracle.render(scene.gauss, ref_w2c, oracle.view_intr(scene.rig, scene.views), scene.rig.W,
                        scene.rig.H, alternatives=True)
    nbad, nfl, nex, mx = compare_images(g, orc)
    fr = g["frame"]
    cnt = fr.buf("counts", torch.int32, 8).cpu().numpy()
    say(f"  split lists {int(cnt[3])} chunks {int(cnt[4])} flagged={nfl} excluded={nex} max_err={mx:.3g} "
        f"min T {g['T'].min():.3g}")
    assert int(cnt[4]) > int(cnt[3]) > 0
    assert g["status"] == 0
    assert nbad == 0
    assert nex <= 0.001 * orc["nflag"].size
    # and within rounding of the walk in order (pixels with a decision at the threshold margin aside)
    o = gpu_render(scene, tile=tile, persistent=persistent, split_len=64, split_fwd=0)
    plain = orc["nflag"] == 0
    assert np.array_equal(o["last_id"][plain], g["last_id"][plain])
    assert float(np.abs(o["img"] - g["img"]).max(axis=1)[plain].max()) <= 1e-5
    assert float(np.abs(o["T"] - g["T"])[plain].max()) <= 1e-5


@pytest.mark.parametrize("tile", [(16, 16), (8, 8)])
def test_gradients_joined_chunks_vs_oracle(tile):
    say(f"case: gradients with joined chunks tile={tile}")
    out, _ = _grad_case(_faint(synth.small_drive(5, n_frames=2)), tile, split_len=64, split_fwd=1)
    say("  " + " ".join(f"{k}={v[1]:.2e}" for k, v in out.items()))
    for k, (ok, err) in out.items():
        assert ok, (k, err)


def test_gradients_tiny_vs_oracle():
    say("case: gradients tiny")
    s = synth.tiny_scene(2)
    out, _ = _grad_case(s, (16, 16))
    for k in ("quat", "scale", "opacity", "color", "mean"):
        assert out[k][0], (k, out[k][1])


def test_empty_and_degenerate_inputs():
    say("case: empty / degenerate")
    s = synth.tiny_scene(0, n=64)
    # every Gaussian behind the camera
    s.gauss.mean[2] = -5.0
    g = gpu_render(s)
    assert g["slots"] == 0 and g["inst"] == 0
    assert np.all(g["img"] == 0) and np.all(g["T"] == 1) and np.all(g["last_pos"] == -1)
    # a NaN parameter and a zero quaternion are culled and flagged
    s = synth.tiny_scene(0, n=64)
    s.gauss.scale[0, 3] = np.nan
    s.gauss.quat[:, 5] = 0.0
    g = gpu_render(s)
    assert g["status"] & B.ST_NONFINITE and g["status"] & B.ST_DEGENERATE
    w2c_ref, _, _ = oracle.pose(s.traj, s.rig, s.xi, s.delta, s.views)
    orc = oracle.render(s.gauss, w2c_ref, oracle.view_intr(s.rig, s.views), s.rig.W, s.rig.H, alternatives=True)
    assert compare_images(g, orc)[0] == 0


def test_capacity_overflow_is_flagged_not_fatal():
    say("case: capacity overflow")
    s = synth.tiny_scene(0)
    ds = pl.DeviceScene.from_scene(s)
    xi, dl = _dev(s.xi), _dev(s.delta)
    fr = pl.Frame(pl.make_settings(), 1, s.gauss.n, s.rig.W, s.rig.H, 100, 200)
    pl.forward(fr, ds, xi, dl)
    torch.cuda.synchronize()
    assert fr.status() & B.ST_CAPACITY
    ns, ni = fr.counts()
    assert ns <= 100 and ni <= 200


@pytest.mark.parametrize("path", ["slot_first", "instance_keys"])
def test_instance_capacity_overflow_keeps_the_longest_prefix(path):
    """With too few instance slots the bin sort emits exactly the instances of the longest prefix
    of slots that fits, in emission order (depth order with the slot-first sort, slot order with
    the 64-bit keys), and flags SPLAT_ST_CAPACITY."""
    say(f"case: instance capacity overflow path={path}")
    scene = synth.small_drive(4, n_frames=2)
    ds = pl.DeviceScene.from_scene(scene)
    xi, dl = _dev(scene.xi), _dev(scene.delta)
    ref = pl.fit_frame(ds, xi, dl, pl.make_settings())
    if path == "instance_keys":
        use_instance_sort(ref)
    pl.forward(ref, ds, xi, dl)
    torch.cuda.synchronize()
    ns, ni = ref.counts()
    assert ref.status() == 0 and ni > 3000
    per_slot = np.bincount(ref.sorted_vals(ni).cpu().numpy().astype(np.int64), minlength=ns)
    if path == "slot_first":  # emission order: (depth32, slot)
        depth = ref.records(ns)[:, 11].contiguous().cpu().numpy().view(np.uint32)
        order = np.lexsort((np.arange(ns), depth))
    else:
        order = np.arange(ns)
    ends = np.cumsum(per_slot[order])
    for cap in (ni // 3, ni // 2 + 17, ni - 1):
        fr = pl.Frame(ref.settings, ref.V, ref.G, ref.W, ref.H, int(ref.plan.slot_cap), cap)
        if path == "instance_keys":
            use_instance_sort(fr)
        pl.forward(fr, ds, xi, dl)
        torch.cuda.synchronize()
        assert fr.status() == B.ST_CAPACITY
        ns2, ni2 = fr.counts()
        k = int(np.searchsorted(ends, cap, side="right"))   # slots order[:k] fit
        assert ns2 == ns and ni2 == (int(ends[k - 1]) if k else 0), cap
        got = np.bincount(fr.sorted_vals(ni2).cpu().numpy().astype(np.int64), minlength=ns)
        want = np.zeros(ns, np.int64)
        want[order[:k]] = per_slot[order[:k]]
        assert np.array_equal(got, want), cap


def test_invalid_arguments_rejected():
    say("case: invalid args")
    st = pl.make_settings()
    with pytest.raises(B.SplatError):
        B.splat_plan_make(st, 0, 10, 64, 64, 10, 10)
    bad = pl.make_settings(tile=(12, 12))
    with pytest.raises(B.SplatError):
        B.splat_plan_make(bad, 1, 10, 64, 64, 10, 10)


def test_l1_kernel_vs_numpy():
    say("case: l1 kernel")
    rng = np.random.default_rng(0)
    img = rng.uniform(size=(3, 3, 17, 29)).astype(np.float32)
    tgt = img.copy()
    tgt[:, :, ::2] = rng.uniform(size=tgt[:, :, ::2].shape)
    mask = np.zeros((3, 17, 29), np.uint8)
    mask[1, 3:7, 2:9] = 1
    it, tt, mt = (torch.as_tensor(a, device="cuda") for a in (img, tgt, mask))
    loss, dimg = pl.l1_loss_grad(it, tt, mt.bool())
    ref_L, ref_d = oracle.l1_loss(img.astype(np.float64), tgt.astype(np.float64), mask)
    # the kernel subtracts in float32 (exact sign, rounded magnitude) and sums in float64
    np.testing.assert_allclose(float(loss.item()), ref_L, rtol=1e-6)
    np.testing.assert_array_equal(dimg.cpu().numpy(), ref_d.astype(np.float32))


@pytest.mark.parametrize("tile, roi, masked", [((16, 16), 0, False), ((8, 8), 9, True), ((32, 16), 17, False),
                                                ((16, 32), 0, True)])
def test_render_fwd_l1_matches_the_separate_calls(tile, roi, masked):
    """The forward with the L1 term in the same launch writes the forward's outputs and the loss
    kernel's gradient bit for bit, and the loss up to the order of its float64 sum (Eq. 4's L1 term
    over the region of interest, with and without a mask)."""
    say(f"case: render_fwd_l1 tile={tile} roi={roi} masked={masked}")
    scene = synth.small_drive(4, n_frames=2)
    ds = pl.DeviceScene.from_scene(scene)
    xi, dl = _dev(scene.xi), _dev(scene.delta)
    st = pl.make_settings(tile=tile, roi_y0=roi)
    fr = pl.fit_frame(ds, xi, dl, st)
    V, H, W = fr.V, fr.H, fr.W
    rng = np.random.default_rng(roi)
    tgt = torch.as_tensor(rng.uniform(size=(V, 3, H, W)).astype(np.float32), device="cuda")
    mask = None
    if masked:
        m = np.zeros((V, H, W), np.uint8)
        m[:, H // 3:H // 2, W // 4:W // 2] = 1
        mask = torch.as_tensor(m, device="cuda")
    img, T, last = (t.clone() for t in pl.forward(fr, ds, xi, dl))
    ref_loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    ref_d = torch.empty_like(img)
    B.splat_l1_loss_grad(img, tgt, mask, ref_d, ref_loss, roi, 0.8)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    d = torch.full_like(img, float("nan"))
    img2, T2, last2 = pl.forward(fr, ds, xi, dl, l1=(tgt, mask, d, loss, 0.8))
    torch.cuda.synchronize()
    assert torch.equal(img2, img) and torch.equal(T2, T) and torch.equal(last2, last)
    assert torch.equal(d, ref_d)
    say(f"  loss {loss.item():.12f} vs {ref_loss.item():.12f}")
    assert float(loss.item()) == pytest.approx(float(ref_loss.item()), rel=1e-12)


def test_slot_meta_matches_the_projections_own_and_a_host_count():
    """splat_slot_meta: the (Gaussian id, view) of every slot, formed from the visibility words,
    equals what the projection writes itself for the 64-bit instance sort, and on the slot-first
    path (where the projection leaves it out) the slots of each view are its visible Gaussians
    in increasing order, as many as the view's slot range holds."""
    say("case: splat_slot_meta against the projection's own meta")
    scene = synth.small_drive(5, n_frames=2)
    ds = pl.DeviceScene.from_scene(scene)
    xi, dl = _dev(scene.xi), _dev(scene.delta)
    fr = pl.fit_frame(ds, xi, dl, pl.make_settings())
    pl.forward(fr, ds, xi, dl)
    torch.cuda.synchronize()
    ns = int(fr.counts()[0])
    assert ns > 0 and fr.status() == 0
    slot_meta = fr.meta(ns).cpu().numpy().copy()
    view_off = fr.buf("view_off", torch.int32, scene.views.n + 1).cpu().numpy()
    for v in range(scene.views.n):
        sl = slot_meta[view_off[v]:view_off[v + 1]]
        assert np.all(sl[:, 1] == v) and np.all(np.diff(sl[:, 0]) > 0)
        assert np.all((sl[:, 0] >= 0) & (sl[:, 0] < ds.n_gauss))
    use_instance_sort(fr)
    raw = fr.buf("meta", torch.int32, 2 * ns)
    raw.fill_(-7)
    pl.forward(fr, ds, xi, dl)   # the projection for the instance keys writes meta itself
    torch.cuda.synchronize()
    assert fr.status() == 0 and int(fr.counts()[0]) == ns
    own = raw.cpu().numpy().reshape(ns, 2).copy()
    assert np.array_equal(own, slot_meta)
    B.splat_slot_meta(fr.plan, fr.ws)
    torch.cuda.synchronize()
    assert np.array_equal(raw.cpu().numpy().reshape(ns, 2), own)


def test_bin_sort_after_a_projection_for_the_other_sort_bins_nothing():
    """A projection writes the per-slot inputs of the plan's bin sort only; binning with the other
    sort before projecting again flags SPLAT_ST_SEQUENCE and leaves every tile list empty (the
    image is the background), and a new projection makes it whole again."""
    say("case: bin_sort after a projection for the other sort")
    scene = synth.small_drive(3, n_frames=2)
    ds = pl.DeviceScene.from_scene(scene)
    xi, dl = _dev(scene.xi), _dev(scene.delta)
    fr = pl.fit_frame(ds, xi, dl, pl.make_settings())
    slot_fields = (int(fr.plan.slot_sort), int(fr.plan.sorted_buf), int(fr.plan.key_shift))
    assert slot_fields[0] == 1
    ref = [t.clone() for t in pl.forward(fr, ds, xi, dl)]
    torch.cuda.synchronize()
    assert fr.status() == 0 and fr.counts()[1] > 0
    for switch in ("to_instance_keys", "to_slot_first"):
        if switch == "to_instance_keys":
            use_instance_sort(fr)
        else:
            pl.forward(fr, ds, xi, dl)   # projected for the instance keys
            fr.plan.slot_sort, fr.plan.sorted_buf, fr.plan.key_shift = slot_fields
        fr.clear_status()
        B.splat_bin_sort(fr.plan, fr.ws)
        torch.cuda.synchronize()
        assert fr.status() == B.ST_SEQUENCE, switch
        assert fr.counts() == (0, 0), switch
        assert int((fr.ranges()[:, 1] - fr.ranges()[:, 0]).sum()) == 0
        fr.clear_status()
        img = pl.forward(fr, ds, xi, dl)[0]
        torch.cuda.synchronize()
        assert fr.status() == 0
        assert torch.equal(img, ref[0]), switch


def test_render_fwd_l1_sum_over_many_work_items_is_reproducible():
    """16,544 work items (8x8 tiles of four 704x376 views): the forward's per-item partial sums of
    |C - target| are added in a fixed order over five groups, so the loss equals the loss kernel's
    up to the order of the float64 sum, a second call adds bit for bit the same value, and the
    loss accumulates into what the caller passed (Eq. 4's L1 term)."""
    say("case: render_fwd_l1 704x376 8x8, 4 views")
    scene = synth.small_drive(5, n_points=20000, W=704, H=376, f=276.0, n_frames=2)
    ds = pl.DeviceScene.from_scene(scene)
    xi, dl = _dev(scene.xi), _dev(scene.delta)
    fr = pl.fit_frame(ds, xi, dl, pl.make_settings(tile=(8, 8)))
    assert fr.V * fr.plan.tiles_per_view > 4 * 4096
    rng = np.random.default_rng(5)
    tgt = torch.as_tensor(rng.uniform(size=(fr.V, 3, fr.H, fr.W)).astype(np.float32), device="cuda")
    img = pl.forward(fr, ds, xi, dl)[0].clone()
    ref_loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    ref_d = torch.empty_like(img)
    B.splat_l1_loss_grad(img, tgt, None, ref_d, ref_loss, 0, 1.0)
    losses = []
    for start in (0.0, 0.0, 2.5):
        loss = torch.full((1,), start, dtype=torch.float64, device="cuda")
        d = torch.full_like(img, float("nan"))
        pl.forward(fr, ds, xi, dl, l1=(tgt, None, d, loss, 1.0))
        torch.cuda.synchronize()
        assert torch.equal(d, ref_d)
        losses.append(float(loss.item()) - start)
    say(f"  loss {losses} vs {ref_loss.item():.12f}")
    assert losses[0] == pytest.approx(float(ref_loss.item()), rel=1e-12)
    assert losses[0] == losses[1]
    assert losses[2] == pytest.approx(losses[0], rel=1e-14)


def _step_for(scene, tile=(16, 16)):
    ds = pl.DeviceScene.from_scene(scene)
    xi, dl = _dev(scene.xi), _dev(scene.delta)
    tgt = torch.as_tensor(oracle.render_scene(scene, xi=scene.xi_gt, delta=scene.delta_gt)["img"],
                          dtype=torch.float32, device="cuda")
    return pl.BatchedStep(ds, xi, dl, tgt, pl.make_settings(tile=tile))


def test_graph_replay_matches_eager():
    say("case: hipGraph replay")
    step = _step_for(synth.small_drive(6, n_frames=2))
    step.run()
    torch.cuda.synchronize()
    ref = [t.clone() for t in (step.fr.img, step.gr.quat, step.gr.color, step.gr.xi, step.gr.delta, step.loss)]
    step.capture()
    for rep in range(3):
        step.fr.img.fill_(-1.0)      # eager work between replays
        step.gr.color.fill_(123.0)
        torch.cuda.synchronize()
        step.replay()
        torch.cuda.synchronize()
        got = (step.fr.img, step.gr.quat, step.gr.color, step.gr.xi, step.gr.delta, step.loss)
        assert torch.equal(got[0], ref[0]), rep
        # float atomics may sum in another order: compare to the gradient bar's metric, 100x tighter
        for a, b in zip(got[1:], ref[1:]):
            ok, err = rel_close(a.cpu().numpy(), b.cpu().numpy(), 1e-5)
            assert ok, (rep, err)


def test_autograd_function_matches_kernels():
    say("case: autograd")
    scene = synth.small_drive(7, n_frames=2)
    step = _step_for(scene)
    step.run()
    torch.cuda.synchronize()
    ds = step.ds
    q = ds.quat.clone().requires_grad_(True)
    sc = ds.scale.clone().requires_grad_(True)
    op = ds.opacity.clone().requires_grad_(True)
    co = ds.color.clone().requires_grad_(True)
    xi = step.xi.clone().requires_grad_(True)
    dl = step.delta.clone().requires_grad_(True)
    img = pl.SplatRender.apply(q, sc, op, co, xi, dl, step.fr, ds)
    loss = (img - step.targets).abs().mean()
    loss.backward()
    for a, b in ((co.grad, step.gr.color), (xi.grad, step.gr.xi), (dl.grad, step.gr.delta), (q.grad, step.gr.quat)):
        ok, err = rel_close(a.detach().cpu().numpy(), b.cpu().numpy(), 1e-4)
        assert ok, err
    # a second render into the same Frame before the first node's backward: that backward would
    # read the second render's lists, so it must refuse
    img1 = pl.SplatRender.apply(q, sc, op, co, xi, dl, step.fr, ds)
    img2 = pl.SplatRender.apply(q, sc * 1.01, op, co, xi, dl, step.fr, ds)
    with pytest.raises(B.SplatError, match="rendered into again"):
        (img1 - step.targets).abs().mean().backward()
    (img2 - step.targets).abs().mean().backward()   # the latest render still differentiates


def test_binding_rejects_undersized_and_misplaced_buffers():
    """The wrappers check element types, contiguity, device and sizes before any launch: the
    kernels trust the sizes the plan implies, so a wrong buffer must not reach them."""
    say("case: binding argument checks")
    scene = synth.small_drive(7, n_frames=2)
    step = _step_for(scene)
    fr = step.fr
    with pytest.raises(B.SplatError, match="elements"):
        B.splat_render_fwd(fr.plan, fr.ws, fr.img[:1], fr.T, fr.last)
    with pytest.raises(B.SplatError, match="dtype"):
        B.splat_render_bwd(fr.plan, fr.ws, step.dimg.double(), fr.T, fr.last)
    with pytest.raises(B.SplatError, match="contiguous"):
        B.splat_render_fwd(fr.plan, fr.ws, fr.img.transpose(2, 3), fr.T, fr.last)
    with pytest.raises(B.SplatError, match="device"):
        B.splat_render_fwd(fr.plan, fr.ws, fr.img.cpu(), fr.T, fr.last)
    with pytest.raises(B.SplatError, match="plan needs"):
        B.splat_bin_sort(fr.plan, fr.ws[:16])
    with pytest.raises(B.SplatError, match="elements"):
        B.splat_project(fr.plan, fr.ws, step.ds.gaussians(), fr.w2c[:1], step.ds.intr)


def test_per_view_plain_matches_batched():
    say("case: per-view plain vs batched")
    scene = synth.small_drive(8, n_frames=2)
    step = _step_for(scene)
    step.run()
    torch.cuda.synchronize()
    pv = pl.PerViewPlain(step.ds, step.xi, step.delta, pl.make_settings())
    gr = pl.alloc_grads(step.ds)
    pv.step(step.xi, step.delta, step.targets, gr)
    torch.cuda.synchronize()
    for v, (dv, fr, _) in enumerate(pv.views):
        assert torch.equal(fr.img[0], step.fr.img[v])
        assert torch.equal(fr.T[0], step.fr.T[v])
    for a, b in ((gr.color, step.gr.color), (gr.xi, step.gr.xi), (gr.delta, step.gr.delta)):
        ok, err = rel_close(a.cpu().numpy(), b.cpu().numpy(), 1e-4)
        assert ok, err
