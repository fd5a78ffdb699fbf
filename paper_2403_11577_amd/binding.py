"""ctypes binding of libsplat.so with the names of include/splat.h.

Argument marshalling only: every function takes torch device tensors (or ints
for sizes), passes their data pointers and the current HIP stream to the C ABI
and raises on a negative return code.  No arithmetic of the method happens here.
The library is loaded from this package directory; if it is missing the import
fails loudly (there is no fallback path).
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsplat.so")

ST_CAPACITY, ST_NONFINITE, ST_DEGENERATE, ST_EXTRAPOLATED, ST_RANGE, ST_SEQUENCE = 1, 2, 4, 8, 16, 32


class SplatError(RuntimeError):
    pass


class splat_settings(C.Structure):
    _fields_ = [("near_z", C.c_double), ("far_z", C.c_double), ("eps2d", C.c_double),
                ("alpha_min", C.c_double), ("alpha_max", C.c_double), ("t_min", C.c_double),
                ("guard", C.c_double), ("bg", C.c_double * 3), ("pad_px", C.c_double),
                ("pad_rel", C.c_double), ("tile_w", C.c_int32), ("tile_h", C.c_int32),
                ("batch", C.c_int32), ("persistent", C.c_int32), ("roi_y0", C.c_int32), ("split_len", C.c_int32),
                ("split_fwd", C.c_int32), ("reserved0", C.c_int32)]


class splat_gaussians(C.Structure):
    _fields_ = [("mean", C.c_void_p), ("quat", C.c_void_p), ("scale", C.c_void_p),
                ("opacity", C.c_void_p), ("color", C.c_void_p), ("n", C.c_int64)]


_PLAN_OFFS = ["ws_bytes", "off_status", "off_counts", "off_view_off", "off_blockcnt", "off_rec",
              "off_meta", "off_rect", "off_ntiles", "off_keys", "off_vals", "off_ranges",
              "off_queue", "off_hist", "off_scan", "off_grad2d", "off_visbits", "off_dwpart", "off_cam"]


class splat_plan(C.Structure):
    _fields_ = ([("s", splat_settings)] +
                [(n, C.c_int32) for n in ("n_views", "width", "height", "tiles_x", "tiles_y",
                                          "tiles_per_view", "depth_bits", "tile_bits",
                                          "n_blocks_proj", "n_sort_blocks")] +
                [(n, C.c_int64) for n in ("n_gauss", "slot_cap", "inst_cap")] +
                [(n, C.c_size_t) for n in _PLAN_OFFS] +
                [("sorted_buf", C.c_int32), ("radix_bits", C.c_int32), ("split_len", C.c_int32),
                 ("key_shift", C.c_int32), ("chk_cap", C.c_int64), ("bq_cap", C.c_int64)] +
                [(n, C.c_size_t) for n in ("off_bqueue", "off_bqoff", "off_chk", "off_chklast", "off_bmask",
                                                      "off_dkey")] +
                [("slot_sort", C.c_int32), ("pack_bits", C.c_int32 * 3)] +
                [(n, C.c_size_t) for n in ("off_spay", "off_skeys", "off_soff", "off_l1part")])


ADAM_MAX_GROUPS = 8
ACT_IDENTITY, ACT_SIGMOID, ACT_EXP = 0, 1, 2


class splat_adam_group(C.Structure):
    _fields_ = [("param", C.c_void_p), ("exp_avg", C.c_void_p), ("exp_avg_sq", C.c_void_p), ("grad", C.c_void_p),
                ("value", C.c_void_p), ("lr", C.c_void_p), ("n", C.c_int64), ("act", C.c_int32),
                ("reserved", C.c_int32)]


class splat_ngp(C.Structure):
    _fields_ = ([(n, C.c_int32) for n in ("levels", "feat", "log2_table", "n_min", "n_max", "hidden")] +
                [("scale_max", C.c_double), ("lo", C.c_double * 3), ("hi", C.c_double * 3)] +
                [(n, C.c_void_p) for n in ("tables", "w1", "b1", "w2", "b2", "w3", "b3")])


_lib = None


def lib():
    """Load libsplat.so once and declare the signatures of include/splat.h."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise SplatError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                         "or python -m paper_2403_11577_amd.build")
    L = C.CDLL(LIB_PATH)
    P, I32, I64 = C.c_void_p, C.c_int32, C.c_int64
    L.splat_default_settings.argtypes = [C.POINTER(splat_settings)]
    L.splat_default_settings.restype = None
    L.splat_plan_make.argtypes = [C.POINTER(splat_settings), I32, I64, I32, I32, I64, I64,
                                  C.POINTER(splat_plan)]
    L.splat_pose_interp_fwd.argtypes = [I32, P, P, P, I32, P, P, P, P, I32, P, P, P, P, P]
    L.splat_pose_interp_bwd.argtypes = [I32, P, P, P, I32, P, P, P, P, I32, P, P, P, P, P, P]
    L.splat_project.argtypes = [C.POINTER(splat_plan), P, C.POINTER(splat_gaussians), P, P, P]
    L.splat_bin_sort.argtypes = [C.POINTER(splat_plan), P, P]
    L.splat_slot_meta.argtypes = [C.POINTER(splat_plan), P, P]
    L.splat_render_fwd.argtypes = [C.POINTER(splat_plan), P, P, P, P, P]
    L.splat_render_bwd.argtypes = [C.POINTER(splat_plan), P, P, P, P, P]
    L.splat_project_bwd.argtypes = [C.POINTER(splat_plan), P, C.POINTER(splat_gaussians), P, P,
                                    P, P, P, P, P, P, P]
    L.splat_render_fwd_stats.argtypes = [C.POINTER(splat_plan), P, P, P, P, P, P]
    L.splat_render_fwd_l1.argtypes = [C.POINTER(splat_plan), P, P, P, P, P, P, C.c_double, P, P, P]
    L.splat_render_bwd_stats.argtypes = [C.POINTER(splat_plan), P, P, P, P, P, P]
    L.splat_l1_loss_grad.argtypes = [P, P, P, I32, I32, I32, I32, C.c_double, P, P, P]
    L.splat_dssim_workspace_size.argtypes = [I32, I32, I32, I32]
    L.splat_dssim_workspace_size.restype = C.c_size_t
    L.splat_dssim_loss_grad.argtypes = [P, P, I32, I32, I32, I32, C.c_double, P, C.c_size_t, P, P, P]
    L.splat_dssim_loss_grad_noalloc.argtypes = [P, P, I32, I32, I32, I32, C.c_double, P, P, P]
    L.splat_scale_reg.argtypes = [P, I64, C.c_double, P, P, P]
    L.splat_adam_step.argtypes = [C.POINTER(splat_adam_group), I32, C.c_double, C.c_double, C.c_double, P, P]
    L.splat_last_error.restype = C.c_char_p
    L.splat_version.restype = C.c_char_p
    L.splat_struct_size.argtypes = [I32]
    L.splat_struct_size.restype = C.c_size_t
    L.splat_ngp_fwd.argtypes = [C.POINTER(splat_ngp), P, I64, P, P, P, P, P]
    L.splat_ngp_workspace_size.argtypes = [I64]
    L.splat_ngp_workspace_size.restype = C.c_size_t
    L.splat_ngp_bwd.argtypes = [C.POINTER(splat_ngp), P, I64, P, P, P, P, P, C.c_size_t, P, P, P, P, P, P, P, P]
    L.splat_ngp_index_size.argtypes = [C.POINTER(splat_ngp), I64]
    L.splat_ngp_index_size.restype = C.c_size_t
    L.splat_ngp_index_workspace_size.argtypes = [C.POINTER(splat_ngp), I64]
    L.splat_ngp_index_workspace_size.restype = C.c_size_t
    L.splat_ngp_index_build.argtypes = [C.POINTER(splat_ngp), P, I64, P, C.c_size_t, P, C.c_size_t, P]
    L.splat_ngp_bwd_indexed.argtypes = [C.POINTER(splat_ngp), P, I64, P, C.c_size_t, P, P, P, P, P, C.c_size_t,
                                        P, P, P, P, P, P, P, P]
    L.splat_ngp_fwd_train.argtypes = [C.POINTER(splat_ngp), P, I64, P, P, P, P, P, C.c_size_t, P]
    L.splat_ngp_bwd_saved.argtypes = [C.POINTER(splat_ngp), I64, P, C.c_size_t, P, P, P, P, P, C.c_size_t,
                                      P, P, P, P, P, P, P, P]
    L.splat_voxel_workspace_size.argtypes = [I64]
    L.splat_voxel_workspace_size.restype = C.c_size_t
    L.splat_voxel_downsample.argtypes = [P, I64, C.POINTER(C.c_double), C.c_double, P, C.c_size_t, P, P, P, P]
    for w, st in ((0, splat_settings), (1, splat_gaussians), (2, splat_plan), (3, splat_ngp), (4, splat_adam_group)):
        if L.splat_struct_size(w) != C.sizeof(st):
            raise SplatError(f"ABI mismatch: {st.__name__} is {L.splat_struct_size(w)} bytes in the "
                             f"library, {C.sizeof(st)} in the binding")
    _lib = L
    return L


def _check(rc: int, what: str):
    if rc != 0:
        msg = lib().splat_last_error().decode()
        raise SplatError(f"{what} failed ({rc}): {msg}")


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


_DT = {"f32": "torch.float32", "f64": "torch.float64", "i32": "torch.int32", "i64": "torch.int64",
       "u8": "torch.uint8"}


def _arg(t, name, dt, numel=None, at_least=False, optional=False):
    """Pointer of a device tensor after checking what the C ABI cannot: that it is a
    contiguous device tensor of the element type the call reads or writes, with the
    number of elements the call touches (or at least that many).  The kernels trust
    these sizes, so an undersized buffer must not reach them."""
    if t is None:
        if optional:
            return None
        raise SplatError(f"{name}: a device tensor is required")
    if not getattr(t, "is_cuda", False):
        raise SplatError(f"{name}: must be a device tensor")
    if str(t.dtype) not in (_DT[dt],) and not (dt == "i32" and str(t.dtype) == "torch.uint32"):
        raise SplatError(f"{name}: dtype {t.dtype}, expected {_DT[dt]}")
    if not t.is_contiguous():
        raise SplatError(f"{name}: must be contiguous")
    if numel is not None:
        n = t.numel()
        if (n < numel) if at_least else (n != numel):
            raise SplatError(f"{name}: {n} elements, expected {'at least ' if at_least else ''}{numel}")
    return C.c_void_p(t.data_ptr())


def _ws(plan, ws):
    if ws is None or not getattr(ws, "is_cuda", False) or not ws.is_contiguous():
        raise SplatError("ws: a contiguous device tensor is required")
    if ws.numel() * ws.element_size() < int(plan.ws_bytes):
        raise SplatError(f"ws: {ws.numel() * ws.element_size()} bytes, the plan needs {int(plan.ws_bytes)}")
    return C.c_void_p(ws.data_ptr())


def _img_sizes(plan):
    V, H, W = int(plan.n_views), int(plan.height), int(plan.width)
    return V * 3 * H * W, V * H * W


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def default_settings(**overrides) -> splat_settings:
    s = splat_settings()
    lib().splat_default_settings(C.byref(s))
    for k, v in overrides.items():
        if k == "bg":
            s.bg = (C.c_double * 3)(*v)
        else:
            setattr(s, k, v)
    return s


def splat_plan_make(settings: splat_settings, n_views: int, n_gauss: int, width: int, height: int,
                    slot_cap: int, inst_cap: int) -> splat_plan:
    p = splat_plan()
    _check(lib().splat_plan_make(C.byref(settings), int(n_views), int(n_gauss), int(width),
                                 int(height), int(slot_cap), int(inst_cap), C.byref(p)),
           "splat_plan_make")
    return p


def gaussians_struct(mean, quat, scale, opacity, color) -> splat_gaussians:
    n = int(opacity.numel())
    return splat_gaussians(_arg(mean, "mean", "f32", 3 * n), _arg(quat, "quat", "f32", 4 * n),
                           _arg(scale, "scale", "f32", 3 * n), _arg(opacity, "opacity", "f32", n),
                           _arg(color, "color", "f32", 3 * n), n)


def _pose_args(knot_t, knot_q, knot_p, R0, t0, xi, delta, view_cam, view_t):
    K, Cn, V = int(knot_t.numel()), int(delta.numel()), int(view_cam.numel())
    return [K, _arg(knot_t, "knot_t", "f64", K), _arg(knot_q, "knot_q", "f64", 4 * K),
            _arg(knot_p, "knot_p", "f64", 3 * K), Cn, _arg(R0, "R0", "f64", 9 * Cn), _arg(t0, "t0", "f64", 3 * Cn),
            _arg(xi, "xi", "f64", 6 * Cn), _arg(delta, "delta", "f64", Cn), V,
            _arg(view_cam, "view_cam", "i32", V), _arg(view_t, "view_t", "f64", V)], V, Cn


def splat_pose_interp_fwd(knot_t, knot_q, knot_p, R0, t0, xi, delta, view_cam, view_t, w2c,
                          status=None, stream=None):
    a, V, _ = _pose_args(knot_t, knot_q, knot_p, R0, t0, xi, delta, view_cam, view_t)
    _check(lib().splat_pose_interp_fwd(*a, _arg(w2c, "w2c", "f64", 12 * V),
                                       _arg(status, "status", "i32", 1, at_least=True, optional=True),
                                       _stream(stream)), "splat_pose_interp_fwd")


def splat_pose_interp_bwd(knot_t, knot_q, knot_p, R0, t0, xi, delta, view_cam, view_t, dw2c, dxi,
                          ddelta, stream=None):
    a, V, Cn = _pose_args(knot_t, knot_q, knot_p, R0, t0, xi, delta, view_cam, view_t)
    _check(lib().splat_pose_interp_bwd(*a, _arg(dw2c, "dw2c", "f64", 12 * V), _arg(dxi, "dxi", "f64", 6 * Cn),
                                       _arg(ddelta, "ddelta", "f64", Cn), _stream(stream)), "splat_pose_interp_bwd")


def _check_gauss(plan, gauss: splat_gaussians):
    if int(gauss.n) != int(plan.n_gauss):
        raise SplatError(f"Gaussians: {int(gauss.n)}, the plan was made for {int(plan.n_gauss)}")


def splat_project(plan, ws, gauss: splat_gaussians, w2c, intr, stream=None):
    _check_gauss(plan, gauss)
    V = int(plan.n_views)
    _check(lib().splat_project(C.byref(plan), _ws(plan, ws), C.byref(gauss), _arg(w2c, "w2c", "f64", 12 * V),
                               _arg(intr, "intr", "f64", 4 * V), _stream(stream)), "splat_project")


def splat_slot_meta(plan, ws, stream=None):
    _check(lib().splat_slot_meta(C.byref(plan), _ws(plan, ws), _stream(stream)), "splat_slot_meta")


def splat_bin_sort(plan, ws, stream=None):
    _check(lib().splat_bin_sort(C.byref(plan), _ws(plan, ws), _stream(stream)), "splat_bin_sort")


def _render_out(plan, img, T_final, last_pos, img_name="img"):
    n3, n1 = _img_sizes(plan)
    return (_arg(img, img_name, "f32", n3), _arg(T_final, "T_final", "f32", n1),
            _arg(last_pos, "last_pos", "i32", n1))


def splat_render_fwd(plan, ws, img, T_final, last_pos, stream=None):
    _check(lib().splat_render_fwd(C.byref(plan), _ws(plan, ws), *_render_out(plan, img, T_final, last_pos),
                                  _stream(stream)), "splat_render_fwd")


def splat_render_fwd_l1(plan, ws, img, T_final, last_pos, target, mask, dL_dimg, loss=None, weight=1.0,
                        stream=None):
    V, H, W = int(plan.n_views), int(plan.height), int(plan.width)
    out = _render_out(plan, img, T_final, last_pos)
    _check(lib().splat_render_fwd_l1(C.byref(plan), _ws(plan, ws), *out, _arg(target, "target", "f32", V * 3 * H * W),
                                     _arg(mask, "mask", "u8", V * H * W, optional=True), float(weight),
                                     _arg(dL_dimg, "dL_dimg", "f32", V * 3 * H * W),
                                     _arg(loss, "loss", "f64", 1, at_least=True, optional=True), _stream(stream)),
           "splat_render_fwd_l1")


def splat_render_bwd(plan, ws, dL_dimg, T_final, last_pos, stream=None):
    _check(lib().splat_render_bwd(C.byref(plan), _ws(plan, ws),
                                  *_render_out(plan, dL_dimg, T_final, last_pos, "dL_dimg"), _stream(stream)),
           "splat_render_bwd")


def splat_project_bwd(plan, ws, gauss: splat_gaussians, w2c, intr, dquat, dscale, dopacity, dcolor,
                      dmean, dw2c, stream=None):
    _check_gauss(plan, gauss)
    V, G = int(plan.n_views), int(plan.n_gauss)
    _check(lib().splat_project_bwd(C.byref(plan), _ws(plan, ws), C.byref(gauss), _arg(w2c, "w2c", "f64", 12 * V),
                                   _arg(intr, "intr", "f64", 4 * V), _arg(dquat, "dquat", "f32", 4 * G),
                                   _arg(dscale, "dscale", "f32", 3 * G), _arg(dopacity, "dopacity", "f32", G),
                                   _arg(dcolor, "dcolor", "f32", 3 * G),
                                   _arg(dmean, "dmean", "f32", 3 * G, optional=True),
                                   _arg(dw2c, "dw2c", "f64", 12 * V), _stream(stream)), "splat_project_bwd")


def splat_render_fwd_stats(plan, ws, img, T_final, last_pos, stats, stream=None):
    _check(lib().splat_render_fwd_stats(C.byref(plan), _ws(plan, ws), *_render_out(plan, img, T_final, last_pos),
                                        _arg(stats, "stats", "i64", 8, at_least=True),
                                        _stream(stream)), "splat_render_fwd_stats")


def splat_render_bwd_stats(plan, ws, dL_dimg, T_final, last_pos, stats, stream=None):
    _check(lib().splat_render_bwd_stats(C.byref(plan), _ws(plan, ws),
                                        *_render_out(plan, dL_dimg, T_final, last_pos, "dL_dimg"),
                                        _arg(stats, "stats", "i64", 8, at_least=True), _stream(stream)),
           "splat_render_bwd_stats")


def _image_pair(img, target, dL_dimg):
    if img.dim() != 4 or img.shape[1] != 3:
        raise SplatError(f"img: shape {tuple(img.shape)}, expected [V, 3, H, W]")
    n = int(img.numel())
    return (_arg(img, "img", "f32", n), _arg(target, "target", "f32", n), _arg(dL_dimg, "dL_dimg", "f32", n))


def splat_l1_loss_grad(img, target, mask, dL_dimg, loss=None, roi_y0=0, weight=1.0, stream=None):
    V, _, H, W = img.shape
    pi, pt, pd = _image_pair(img, target, dL_dimg)
    _check(lib().splat_l1_loss_grad(pi, pt, _arg(mask, "mask", "u8", V * H * W, optional=True), int(V), int(W),
                                    int(H), int(roi_y0), float(weight), pd,
                                    _arg(loss, "loss", "f64", 1, at_least=True, optional=True), _stream(stream)),
           "splat_l1_loss_grad")


def splat_dssim_workspace_size(n_views, width, height, roi_y0=0) -> int:
    return int(lib().splat_dssim_workspace_size(int(n_views), int(width), int(height), int(roi_y0)))


def splat_dssim_loss_grad(img, target, ws, dL_dimg, loss=None, roi_y0=0, weight=0.2, stream=None):
    V, _, H, W = img.shape
    pi, pt, pd = _image_pair(img, target, dL_dimg)
    _check(lib().splat_dssim_loss_grad(pi, pt, int(V), int(W), int(H), int(roi_y0), float(weight),
                                       _arg(ws, "ws", "u8"), int(ws.numel() * ws.element_size()), pd,
                                       _arg(loss, "loss", "f64", 1, at_least=True, optional=True),
                                       _stream(stream)), "splat_dssim_loss_grad")


DSSIM_NOALLOC_MAX_PX = 1 << 24


def splat_dssim_loss_grad_noalloc(img, target, dL_dimg, loss=None, roi_y0=0, weight=0.2, stream=None):
    """splat_dssim_loss_grad without a workspace (the library's fixed scratch array)."""
    V, _, H, W = img.shape
    pi, pt, pd = _image_pair(img, target, dL_dimg)
    _check(lib().splat_dssim_loss_grad_noalloc(pi, pt, int(V), int(W), int(H), int(roi_y0), float(weight), pd,
                                               _arg(loss, "loss", "f64", 1, at_least=True, optional=True),
                                               _stream(stream)), "splat_dssim_loss_grad_noalloc")


def splat_adam_step(groups, step, beta1=0.9, beta2=0.999, eps=1e-15, stream=None):
    """groups: [(param, exp_avg, exp_avg_sq, grad, value or None, lr, act)] of float32 device tensors
    (lr a one-element device tensor); step: one-element float32 device tensor, advanced by one."""
    arr = (splat_adam_group * len(groups))()
    for a, (param, m, v, grad, value, lr, act) in zip(arr, groups):
        n = param.numel()
        for t in (m, v, grad) + ((value,) if value is not None else ()):
            if t.numel() != n or not t.is_contiguous() or str(t.dtype) != "torch.float32":
                raise SplatError("splat_adam_step: arrays of a group must be contiguous float32 of one size")
        a.param, a.exp_avg, a.exp_avg_sq, a.grad = _ptr(param), _ptr(m), _ptr(v), _ptr(grad)
        a.value, a.lr, a.n, a.act = _ptr(value), _ptr(lr), n, int(act)
    _check(lib().splat_adam_step(arr, len(groups), float(beta1), float(beta2), float(eps), _ptr(step),
                                 _stream(stream)), "splat_adam_step")


def splat_scale_reg(scale, lam, dscale, loss=None, stream=None):
    _check(lib().splat_scale_reg(_ptr(scale), int(scale.shape[1]), float(lam), _ptr(dscale), _ptr(loss),
                                 _stream(stream)), "splat_scale_reg")


def splat_version() -> str:
    return lib().splat_version().decode()


def ngp_struct(cfg, lo, hi, tables, w1, b1, w2, b2, w3, b3) -> splat_ngp:
    """cfg: any object with levels, feat, log2_table, n_min, n_max, hidden, scale_max."""
    return splat_ngp(int(cfg.levels), int(cfg.feat), int(cfg.log2_table), int(cfg.n_min), int(cfg.n_max),
                     int(cfg.hidden), float(cfg.scale_max), (C.c_double * 3)(*[float(v) for v in lo]),
                     (C.c_double * 3)(*[float(v) for v in hi]), _ptr(tables), _ptr(w1), _ptr(b1), _ptr(w2),
                     _ptr(b2), _ptr(w3), _ptr(b3))


def splat_ngp_fwd(model: splat_ngp, mean, quat, scale, opacity, color, stream=None):
    _check(lib().splat_ngp_fwd(C.byref(model), _ptr(mean), int(mean.shape[1]), _ptr(quat), _ptr(scale),
                               _ptr(opacity), _ptr(color), _stream(stream)), "splat_ngp_fwd")


def splat_ngp_workspace_size(n) -> int:
    return int(lib().splat_ngp_workspace_size(int(n)))


def splat_ngp_bwd(model: splat_ngp, mean, dquat, dscale, dopacity, dcolor, ws, dtables, dw1, db1, dw2, db2, dw3,
                  db3, stream=None):
    _check(lib().splat_ngp_bwd(C.byref(model), _ptr(mean), int(mean.shape[1]), _ptr(dquat), _ptr(dscale),
                               _ptr(dopacity), _ptr(dcolor), _ptr(ws), int(ws.numel() * ws.element_size()),
                               _ptr(dtables), _ptr(dw1), _ptr(db1), _ptr(dw2), _ptr(db2), _ptr(dw3), _ptr(db3),
                               _stream(stream)), "splat_ngp_bwd")


def splat_ngp_index_size(model: splat_ngp, n) -> int:
    return int(lib().splat_ngp_index_size(C.byref(model), int(n)))


def splat_ngp_index_workspace_size(model: splat_ngp, n) -> int:
    return int(lib().splat_ngp_index_workspace_size(C.byref(model), int(n)))


def splat_ngp_index_build(model: splat_ngp, mean, index, ws, stream=None):
    _check(lib().splat_ngp_index_build(C.byref(model), _ptr(mean), int(mean.shape[1]), _ptr(index),
                                       int(index.numel() * index.element_size()), _ptr(ws),
                                       int(ws.numel() * ws.element_size()), _stream(stream)), "splat_ngp_index_build")


def splat_ngp_bwd_indexed(model: splat_ngp, mean, index, dquat, dscale, dopacity, dcolor, ws, dtables, dw1, db1,
                          dw2, db2, dw3, db3, stream=None):
    _check(lib().splat_ngp_bwd_indexed(C.byref(model), _ptr(mean), int(mean.shape[1]), _ptr(index),
                                       int(index.numel() * index.element_size()), _ptr(dquat), _ptr(dscale),
                                       _ptr(dopacity), _ptr(dcolor), _ptr(ws), int(ws.numel() * ws.element_size()),
                                       _ptr(dtables), _ptr(dw1), _ptr(db1), _ptr(dw2), _ptr(db2), _ptr(dw3),
                                       _ptr(db3), _stream(stream)), "splat_ngp_bwd_indexed")


def splat_ngp_fwd_train(model: splat_ngp, mean, quat, scale, opacity, color, ws, stream=None):
    _check(lib().splat_ngp_fwd_train(C.byref(model), _ptr(mean), int(mean.shape[1]), _ptr(quat), _ptr(scale),
                                     _ptr(opacity), _ptr(color), _ptr(ws), int(ws.numel() * ws.element_size()),
                                     _stream(stream)), "splat_ngp_fwd_train")


def splat_ngp_bwd_saved(model: splat_ngp, n, index, dquat, dscale, dopacity, dcolor, ws, dtables, dw1, db1, dw2,
                        db2, dw3, db3, stream=None):
    _check(lib().splat_ngp_bwd_saved(C.byref(model), int(n), _ptr(index), int(index.numel() * index.element_size()),
                                     _ptr(dquat), _ptr(dscale), _ptr(dopacity), _ptr(dcolor), _ptr(ws),
                                     int(ws.numel() * ws.element_size()), _ptr(dtables), _ptr(dw1), _ptr(db1),
                                     _ptr(dw2), _ptr(db2), _ptr(dw3), _ptr(db3), _stream(stream)),
           "splat_ngp_bwd_saved")


def splat_voxel_workspace_size(n) -> int:
    return int(lib().splat_voxel_workspace_size(int(n)))


def splat_voxel_downsample(pts, lo, voxel, ws, keep, n_keep, status, stream=None):
    """pts [3, n] float32 device; keep int32 [>= n]; n_keep, status uint32 device scalars."""
    lo3 = (C.c_double * 3)(*[float(v) for v in lo])
    _check(lib().splat_voxel_downsample(_ptr(pts), int(pts.shape[1]), lo3, float(voxel), _ptr(ws),
                                        int(ws.numel() * ws.element_size()), _ptr(keep), _ptr(n_keep),
                                        _ptr(status), _stream(stream)), "splat_voxel_downsample")
