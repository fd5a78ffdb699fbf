"""The C ABI on the host: the library loads without a GPU, exports every symbol that
include/splat.h declares, its struct mirrors match, and argument checks reject bad
calls synchronously (nothing is launched, so no device is needed)."""
import ctypes as C
import os
import re

import pytest

from paper_2403_11577_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "splat.h")).read()
    return sorted(set(re.findall(r"SPLAT_API\s+[\w\s\*]+?\b(splat_\w+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = declared_symbols()
    assert len(names) >= 15
    L = B.lib()
    for n in names:
        assert hasattr(L, n), n


def test_struct_sizes_match_library():
    L = B.lib()
    assert L.splat_struct_size(0) == C.sizeof(B.splat_settings)
    assert L.splat_struct_size(1) == C.sizeof(B.splat_gaussians)
    assert L.splat_struct_size(2) == C.sizeof(B.splat_plan)


def test_default_settings_are_the_documented_readings():
    s = B.default_settings()
    assert (s.near_z, s.far_z, s.eps2d, s.alpha_max, s.t_min, s.guard) == (0.2, 256.0, 0.3, 0.99, 1e-4, 0.15)
    assert abs(s.alpha_min - 1 / 255) < 1e-15
    assert (s.tile_w, s.tile_h) == (16, 16)


def test_plan_layout_is_aligned_and_disjoint():
    s = B.default_settings()
    p = B.splat_plan_make(s, 3, 1000, 100, 37, 2000, 9000)
    names = [n for n in B._PLAN_OFFS if n != "ws_bytes"] + ["off_bqueue", "off_bqoff", "off_chk", "off_chklast",
                                                           "off_bmask", "off_dkey", "off_spay", "off_skeys", "off_soff",
                                                           "off_l1part"]
    offs = sorted((getattr(p, n), n) for n in names)
    assert all(o % 256 == 0 for o, _ in offs)
    assert len({o for o, _ in offs}) == len(offs)
    assert offs[-1][0] < p.ws_bytes
    # split lists: a list of L >= split_len instances needs ceil(L / split_len) <= 2 L / split_len
    # checkpoint slots, so 2 inst_cap / split_len (+1) bound them; the adjoint items add the tiles
    assert p.split_len == 1024
    assert p.chk_cap == 2 * -(-9000 // 1024) + 1 and p.bq_cap == 63 + p.chk_cap
    assert p.off_chklast - p.off_chk >= p.chk_cap * 16 * 16 * 16
    assert p.off_bmask - p.off_chklast >= p.chk_cap * 16 * 16 * 4
    assert p.off_dkey - p.off_bmask >= 9000 and p.off_spay - p.off_dkey >= 2000 * 4
    assert p.off_skeys - p.off_spay >= 2000 * 16 and p.off_soff - p.off_skeys >= 2000 * 4
    assert p.off_l1part - p.off_soff >= (-(-2000 // 64) + 1) * 4
    assert p.ws_bytes - p.off_l1part >= (63 + 1) * 8   # 63 work-item partials, one group sum
    assert p.tiles_x == 7 and p.tiles_y == 3 and p.tiles_per_view == 21
    # key = (view*T + tile) << depth_bits | depth: 63 items need 6 bits, the 0.2..256 m window 27
    assert p.tile_bits == 6 and p.depth_bits == 27
    rb = p.radix_bits
    assert 4 <= rb <= 12
    # slot-first bin sort: payload = slot (11 bits for 2000 slots) | first tile (6) | w - 1 (3, 7
    # tiles) | h - 1 (2, 3 tiles), 22 bits; the instance keys are the tile field (key >> 27)
    assert p.slot_sort == 1 and list(p.pack_bits) == [11, 3, 2]
    assert p.sorted_buf == ((p.tile_bits + rb - 1) // rb) % 2 and p.key_shift == p.depth_bits


def test_plan_sort_fields_are_checked():
    """The plan may be switched from the slot-first bin sort to one 64-bit key per instance (the
    GPU parity tests run both), but only with the sorted-buffer and key-shift fields of that
    sort; inconsistent sort fields are refused before anything is launched."""
    L = B.lib()
    p = B.splat_plan_make(B.default_settings(), 3, 1000, 100, 37, 2000, 9000)
    rb = p.radix_bits
    p.slot_sort = 0   # the 64-bit sort needs sorted_buf = passes mod 2 and key_shift = 9 here
    assert L.splat_bin_sort(C.byref(p), C.c_void_p(16), None) == -1
    assert b"sort fields are inconsistent" in L.splat_last_error()
    p.sorted_buf = ((p.tile_bits + p.depth_bits + rb - 1) // rb) % 2
    p.key_shift = -1
    assert L.splat_render_fwd(C.byref(p), C.c_void_p(16), C.c_void_p(16), C.c_void_p(16), C.c_void_p(16), None) == -1
    assert b"sort fields are inconsistent" in L.splat_last_error()
    p.slot_sort = 2
    assert L.splat_bin_sort(C.byref(p), C.c_void_p(16), None) == -1
    assert b"sort fields are inconsistent" in L.splat_last_error()
    # the payload must fit: 2^40 slots would need 40 bits for the slot id alone
    q = B.splat_plan_make(B.default_settings(), 3, 1000, 100, 37, 2000, 9000)
    q.pack_bits[0] = 1
    assert L.splat_bin_sort(C.byref(q), C.c_void_p(16), None) == -1
    assert b"sort fields are inconsistent" in L.splat_last_error()


@pytest.mark.parametrize("kw, msg", [
    (dict(n_views=0), "n_views"),
    (dict(width=0), "image size"),
    (dict(slot_cap=0), "capacities"),
    (dict(inst_cap=1 << 31), "capacities"),
])
def test_plan_make_rejects_bad_shapes(kw, msg):
    args = dict(n_views=2, n_gauss=100, width=64, height=48, slot_cap=100, inst_cap=1000)
    args.update(kw)
    with pytest.raises(B.SplatError, match=msg):
        B.splat_plan_make(B.default_settings(), **args)


@pytest.mark.parametrize("field, value", [
    ("tile_w", 12), ("batch", 8), ("batch", 300), ("batch", 16), ("batch", 48), ("near_z", 0.0), ("far_z", 0.1),
    ("alpha_min", 0.0), ("alpha_max", 1.0), ("t_min", 0.0), ("eps2d", -1.0), ("persistent", 2),
    ("split_len", 32), ("split_len", 96), ("split_len", 1 << 25), ("split_len", -64), ("split_fwd", 2),
])
def test_plan_make_rejects_bad_settings(field, value):
    s = B.default_settings()
    setattr(s, field, value)
    with pytest.raises(B.SplatError):
        B.splat_plan_make(s, 1, 10, 64, 64, 10, 10)


def test_entry_points_reject_an_edited_split_length():
    # the checkpoint capacity is sized for the plan's split_len: editing it is an error, not a fault
    L = B.lib()
    p = B.splat_plan_make(B.default_settings(), 1, 10, 64, 64, 10, 100)
    p.split_len = 64
    assert L.splat_render_fwd(C.byref(p), C.c_void_p(16), C.c_void_p(16), C.c_void_p(16), C.c_void_p(16), None) == -1
    assert b"split fields" in L.splat_last_error()
    assert L.splat_bin_sort(C.byref(p), C.c_void_p(16), None) == -1


def test_render_fwd_l1_rejects_bad_arguments_before_launching():
    L = B.lib()
    s = B.default_settings()
    p = B.splat_plan_make(s, 1, 10, 64, 37, 10, 100)
    buf = C.c_void_p(16)
    # a NULL target or gradient is refused
    assert L.splat_render_fwd_l1(C.byref(p), buf, buf, buf, buf, None, None, 1.0, buf, None, None) == -1
    assert b"NULL argument" in L.splat_last_error()
    # the region of interest must leave rows (N > 0; splat_plan_make already refuses such a plan,
    # an edited one is refused here), and the weight must be finite
    q = B.splat_plan_make(s, 1, 10, 64, 37, 10, 100)
    q.s.roi_y0 = 37
    assert L.splat_render_fwd_l1(C.byref(q), buf, buf, buf, buf, buf, None, 1.0, buf, None, None) == -1
    assert b"leaves no rows" in L.splat_last_error()
    assert L.splat_render_fwd_l1(C.byref(p), buf, buf, buf, buf, buf, None, float("inf"), buf, None, None) == -1
    assert b"finite" in L.splat_last_error()


def test_too_many_work_items_is_unsupported():
    # 1023 views of 2048 x 2048 8x8 tiles exceed the 2^31 (view, tile) items the key and queue allow
    s = B.default_settings()
    s.far_z = 1e30   # 30 depth bits: with at most 31 tile bits the key stays within 64 bits
    s.tile_w = s.tile_h = 8
    rc = B.lib().splat_plan_make(C.byref(s), 1023, 10, 16384, 16384, 10, 10, C.byref(B.splat_plan()))
    assert rc == -2
    assert b"too many" in B.lib().splat_last_error()
    p = B.splat_plan_make(s, 1, 10, 1408, 376, 10, 10)
    assert p.depth_bits == 30


def test_entry_points_reject_null_arguments_without_a_device():
    L = B.lib()
    s = B.default_settings()
    p = B.splat_plan_make(s, 1, 10, 64, 64, 10, 100)
    g = B.splat_gaussians()
    g.n = 10
    assert L.splat_project(None, None, None, None, None, None) == -1
    assert L.splat_project(C.byref(p), None, C.byref(g), None, None, None) == -1
    assert L.splat_project(C.byref(p), C.c_void_p(16), C.byref(g), None, None, None) == -1  # NULL planes
    g.n = 11
    assert L.splat_project(C.byref(p), C.c_void_p(16), C.byref(g), C.c_void_p(16), C.c_void_p(16), None) == -1
    assert b"plan was made for" in L.splat_last_error()
    assert L.splat_bin_sort(C.byref(p), None, None) == -1
    assert L.splat_render_fwd(C.byref(p), C.c_void_p(16), None, None, None, None) == -1
    assert L.splat_render_bwd(C.byref(p), C.c_void_p(16), None, None, None, None) == -1
    assert L.splat_pose_interp_fwd(1, *([None] * 3), 1, *([None] * 4), 1, None, None, None, None, None) == -1
    assert b"2 trajectory knots" in L.splat_last_error()
    assert L.splat_l1_loss_grad(None, None, None, 1, 4, 4, 0, 1.0, None, None, None) == -1
    bad = B.splat_plan()  # all zeros: not made by splat_plan_make
    assert L.splat_bin_sort(C.byref(bad), C.c_void_p(16), None) == -1
    assert b"not initialised" in L.splat_last_error()


def test_region_of_interest_is_validated():
    s = B.default_settings()
    assert s.roi_y0 == 0
    s.roi_y0 = -1
    with pytest.raises(B.SplatError, match="roi_y0"):
        B.splat_plan_make(s, 1, 10, 64, 48, 10, 10)
    s.roi_y0 = 48
    with pytest.raises(B.SplatError, match="roi_y0"):
        B.splat_plan_make(s, 1, 10, 64, 48, 10, 10)
    s.roi_y0 = 47
    assert B.splat_plan_make(s, 1, 10, 64, 48, 10, 10).s.roi_y0 == 47
    L = B.lib()
    assert L.splat_l1_loss_grad(None, None, None, 1, 4, 4, 4, 1.0, None, None, None) == -1


def test_scale_reg_rejects_bad_arguments_without_a_device():
    L = B.lib()
    assert L.splat_scale_reg(None, 0, 1e-3, None, None, None) == 0   # nothing to do
    assert L.splat_scale_reg(None, 5, 1e-3, None, None, None) == -1
    assert b"NULL" in L.splat_last_error()
    assert L.splat_scale_reg(None, -1, 1e-3, None, None, None) == -1


def test_dssim_workspace_and_argument_checks_without_a_device():
    L = B.lib()
    assert L.splat_dssim_workspace_size(2, 10, 8, 3) == 3 * 6 * 5 * 10 * 4
    assert L.splat_dssim_workspace_size(2, 10, 8, 8) == 0
    assert L.splat_dssim_loss_grad(None, None, 1, 4, 4, 0, 0.2, None, 0, None, None, None) == -1
    assert b"NULL" in L.splat_last_error()


def test_voxel_downsample_argument_checks_without_a_device():
    L = B.lib()
    lo = (C.c_double * 3)(0.0, 0.0, 0.0)
    assert L.splat_voxel_workspace_size(-1) == 0
    assert L.splat_voxel_workspace_size(1000) >= 1000 * (16 + 8 + 4)  # two key, value and flag buffers
    assert L.splat_voxel_downsample(None, 10, lo, 0.1, None, 0, None, None, None, None) == -1
    assert b"NULL" in L.splat_last_error()
    n_keep = C.c_void_p(16)
    for voxel in (0.0, -1.0, float("inf"), float("nan")):
        assert L.splat_voxel_downsample(C.c_void_p(16), 10, lo, voxel, C.c_void_p(16), 1 << 20, C.c_void_p(16),
                                        n_keep, C.c_void_p(16), None) == -1
    assert b"voxel size" in L.splat_last_error()
    assert L.splat_voxel_downsample(C.c_void_p(16), 10, lo, 0.1, C.c_void_p(16), 8, C.c_void_p(16), n_keep,
                                    C.c_void_p(16), None) == -1
    assert b"workspace" in L.splat_last_error()
    bad = (C.c_double * 3)(0.0, float("nan"), 0.0)
    assert L.splat_voxel_downsample(C.c_void_p(16), 10, bad, 0.1, C.c_void_p(16), 1 << 20, C.c_void_p(16), n_keep,
                                    C.c_void_p(16), None) == -1


def test_ngp_index_argument_checks_without_a_device():
    L = B.lib()
    m = B.splat_ngp(16, 2, 19, 16, 4096, 64, 0.05, (C.c_double * 3)(0, 0, 0), (C.c_double * 3)(1, 1, 1),
                    *([C.c_void_p(16)] * 7))
    n = 1000
    assert L.splat_ngp_index_size(C.byref(m), n) >= 16 * 8 * n * 8      # (Gaussian, weight) pairs
    assert L.splat_ngp_index_workspace_size(C.byref(m), n) >= 16 * 8 * n * 24
    assert L.splat_ngp_index_size(None, n) == 0
    assert L.splat_ngp_index_size(C.byref(m), (1 << 24) + 1) == 0
    assert b"2^24" in L.splat_last_error()
    assert L.splat_ngp_index_build(C.byref(m), None, n, None, 0, None, 0, None) == -1
    assert L.splat_ngp_index_build(C.byref(m), C.c_void_p(16), n, C.c_void_p(16), 8, C.c_void_p(16), 1 << 40,
                                   None) == -1
    assert b"index of" in L.splat_last_error()
    args = [C.c_void_p(16)] * 14
    assert L.splat_ngp_bwd_indexed(C.byref(m), C.c_void_p(16), n, C.c_void_p(16), 1 << 40, *args[:4],
                                   C.c_void_p(16), 8, *args[:7], None) == -1
    assert b"workspace" in L.splat_last_error()


def test_ngp_training_pair_argument_checks_without_a_device():
    L = B.lib()
    m = B.splat_ngp(16, 2, 19, 16, 4096, 64, 0.05, (C.c_double * 3)(0, 0, 0), (C.c_double * 3)(1, 1, 1),
                    *([C.c_void_p(16)] * 7))
    p = C.c_void_p(16)
    assert L.splat_ngp_fwd_train(C.byref(m), p, 100, p, p, p, p, None, 0, None) == -1
    assert b"NULL" in L.splat_last_error()
    assert L.splat_ngp_fwd_train(C.byref(m), p, 100, p, p, p, p, p, 16, None) == -1
    assert b"workspace" in L.splat_last_error()
    assert L.splat_ngp_bwd_saved(C.byref(m), 100, None, 0, *([p] * 4), p, 1 << 40, *([p] * 7), None) == -1
    assert L.splat_ngp_bwd_saved(C.byref(m), 100, p, 1 << 40, *([p] * 4), p, 16, *([p] * 7), None) == -1
    assert b"workspace" in L.splat_last_error()
    assert L.splat_ngp_bwd_saved(C.byref(m), 0, None, 0, *([None] * 4), None, 0, *([None] * 7), None) == 0


def test_header_is_plain_c99(tmp_path):
    """include/splat.h compiles as strict C99 (no C++ or torch types in the ABI)."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "use.c"
    src.write_text('#include "splat.h"\nint main(void) { splat_settings s; return (int)sizeof(s) == 0; }\n')
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    r = subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-fsyntax-only", f"-I{inc}",
                        str(src)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_adam_step_rejects_bad_groups_without_a_device():
    L = B.lib()
    g = (B.splat_adam_group * 2)()
    for a in g:
        a.n, a.act = 4, B.ACT_IDENTITY
        a.param = a.exp_avg = a.exp_avg_sq = a.grad = a.lr = C.c_void_p(16)
    step = C.c_void_p(16)
    assert L.splat_adam_step(None, 1, 0.9, 0.999, 1e-15, step, None) == -1
    assert L.splat_adam_step(g, 0, 0.9, 0.999, 1e-15, step, None) == -1
    assert L.splat_adam_step(g, B.ADAM_MAX_GROUPS + 1, 0.9, 0.999, 1e-15, step, None) == -1
    assert L.splat_adam_step(g, 2, 1.0, 0.999, 1e-15, step, None) == -1
    g[1].act = B.ACT_SIGMOID  # needs the value array
    assert L.splat_adam_step(g, 2, 0.9, 0.999, 1e-15, step, None) == -1
    assert b"NULL" in L.splat_last_error()
    g[1].act = 7
    assert L.splat_adam_step(g, 2, 0.9, 0.999, 1e-15, step, None) == -1
    assert b"activation" in L.splat_last_error()


def test_binding_checks_buffers_before_the_library():
    """The wrappers refuse host tensors, wrong element types and undersized buffers on the host,
    before anything reaches the library (which cannot see tensor sizes)."""
    import torch
    p = B.splat_plan_make(B.default_settings(), 2, 10, 32, 16, 20, 100)
    ws = torch.empty(int(p.ws_bytes), dtype=torch.uint8)
    img = torch.empty((2, 3, 16, 32))
    T = torch.empty((2, 16, 32))
    last = torch.empty((2, 16, 32), dtype=torch.int32)
    with pytest.raises(B.SplatError, match="device"):
        B.splat_render_fwd(p, ws, img, T, last)
    with pytest.raises(B.SplatError, match="device"):
        B.splat_bin_sort(p, ws)
    with pytest.raises(B.SplatError, match="device"):
        B.splat_l1_loss_grad(img, img, None, img)


def test_device_scene_rejects_bad_trajectories_and_cameras():
    """Knot times must increase strictly and view cameras must exist: checked once on the host,
    since the pose kernels read these only on the device."""
    import dataclasses
    import numpy as np
    import synth
    from paper_2403_11577_amd import pipeline as pl
    s = synth.small_drive(0, n_frames=1)
    pl.DeviceScene.from_scene(s, device="cpu")
    t = np.asarray(s.traj.t, np.float64).copy()
    t[3] = t[2]
    bad = dataclasses.replace(s, traj=dataclasses.replace(s.traj, t=t))
    with pytest.raises(B.SplatError, match="strictly increasing"):
        pl.DeviceScene.from_scene(bad, device="cpu")
    cam = np.asarray(s.views.cam).copy()
    cam[0] = 2
    bad = dataclasses.replace(s, views=dataclasses.replace(s.views, cam=cam))
    with pytest.raises(B.SplatError, match="camera indices"):
        pl.DeviceScene.from_scene(bad, device="cpu")


def test_noalloc_dssim_rejects_oversized_inputs_on_the_host():
    """The allocation-free D-SSIM call checks its size against the fixed array before it
    touches a device: nothing is launched, so no GPU is needed."""
    L = B.lib()
    big = B.DSSIM_NOALLOC_MAX_PX // (3 * 64 * 64) + 1
    assert L.splat_dssim_loss_grad_noalloc(C.c_void_p(16), C.c_void_p(16), big, 64, 64, 0, 0.2, C.c_void_p(16),
                                           None, None) == -1
    assert b"exceed the maximum" in L.splat_last_error()
    assert L.splat_dssim_loss_grad_noalloc(None, None, 1, 8, 8, 0, 0.2, None, None, None) == -1


def test_status_bits_and_return_codes_match_the_header():
    """The binding's copies of the status bits and return codes are the header's values."""
    text = open(os.path.join(ROOT, "include", "splat.h")).read()
    defs = {m.group(1): int(m.group(2)) for m in re.finditer(r"#define SPLAT_(\w+) \(?(-?\d+)u?\)?", text)}
    for name in ("CAPACITY", "NONFINITE", "DEGENERATE", "EXTRAPOLATED", "RANGE", "SEQUENCE"):
        assert getattr(B, "ST_" + name) == defs["ST_" + name], name
    assert len({defs[k] for k in defs if k.startswith("ST_")}) == sum(k.startswith("ST_") for k in defs)
