"""ctypes front end of the FP64 CPU oracle (``splat_oracle.c``).

TEST INFRASTRUCTURE ONLY: used by ``tests/``, the smoke check and the CPU
baseline of the benchmark; never by the product path.

Every function follows the paper's method (3DGS-Calib, arXiv 2403.11577):
  * ``pose`` / ``pose_bwd``: LiDAR trajectory by linear interpolation + SLERP
    (Sec. III-A), camera pose by Eq. (1), world->camera by Eq. (2), and their
    exact adjoint;
  * ``render`` / ``grad``: Eq. (2), Eq. (3) and the EWA splatting function Phi
    of Eq. (5), composited per pixel over all Gaussians in depth order, and the
    exact reverse-mode derivative (end of Sec. III-B);
  * ``l1_loss``: the L1 part of Eq. (4);
  * ``tile_lists``: the binning reference (which tiles every Gaussian covers and
    the per-tile depth order), derived from the projected footprints;
  * ``fd_check``: FP64 central finite differences of the loss.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import subprocess

import numpy as np

__all__ = ["Settings", "build", "lib", "pose", "pose_bwd", "project_one", "render", "grad",
           "project_all", "pixel_stack", "tile_lists", "l1_loss", "scale_reg", "render_scene",
           "loss_and_grad", "fd_loss", "view_intr", "gauss64", "num_threads", "PROJ_FIELDS"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "splat_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


@dataclasses.dataclass
class Settings:
    """Renderer constants (readings where the paper is silent)."""
    near_z: float = 0.2
    far_z: float = 256.0
    eps2d: float = 0.3
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    t_min: float = 1e-4
    guard: float = 0.15
    bg: tuple = (0.0, 0.0, 0.0)
    margin: float = 1e-4
    pad_px: float = 0.1
    pad_rel: float = 1e-4
    roi_y0: int = 0          # first image row of the region of interest (Sec. III-C, image cropping)


class _CSettings(C.Structure):
    _fields_ = [("near_z", C.c_double), ("far_z", C.c_double), ("eps2d", C.c_double),
                ("alpha_min", C.c_double), ("alpha_max", C.c_double), ("t_min", C.c_double),
                ("guard", C.c_double), ("bg", C.c_double * 3), ("margin", C.c_double),
                ("pad_px", C.c_double), ("pad_rel", C.c_double), ("roi_y0", C.c_int32), ("roi_pad_", C.c_int32)]


def _cs(s: Settings) -> _CSettings:
    return _CSettings(s.near_z, s.far_z, s.eps2d, s.alpha_min, s.alpha_max, s.t_min, s.guard,
                      (C.c_double * 3)(*s.bg), s.margin, s.pad_px, s.pad_rel, int(s.roi_y0), 0)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP contraction off so that fmaf is explicit)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        L.or_pose.argtypes = [C.c_int, P, P, P, C.c_int, P, P, P, P, C.c_int, P, P, P, P, P]
        L.or_pose_bwd.argtypes = [C.c_int, P, P, P, C.c_int, P, P, P, P, C.c_int, P, P, P, P, P]
        L.or_project_one.argtypes = [P, P, P, P, C.c_double, P, P, C.c_int, C.c_int, P]
        L.or_render.argtypes = [P, C.c_int64, P, P, P, P, P, C.c_int, P, P, C.c_int, C.c_int, C.c_int,
                                P, P, P, P, P, P, P, P, P, P, P]
        L.or_project_all.argtypes = [P, C.c_int64, P, P, P, P, C.c_int, P, P, C.c_int, C.c_int,
                                     P, P, P, P, P, P]
        L.or_grad.argtypes = [P, C.c_int64, P, P, P, P, P, C.c_int, P, P, C.c_int, C.c_int, P, P,
                              P, P, P, P, P, P]
        L.or_pixel_stack.argtypes = [P, C.c_int64, P, P, P, P, P, P, P, C.c_int, C.c_int, C.c_int,
                                     C.c_int, P, C.c_int64]
        L.or_pixel_stack.restype = C.c_int64
        L.or_num_threads.restype = C.c_int
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().or_num_threads())


def set_num_threads(n: int) -> int:
    """Threads of the OpenMP loops from now on (for timing the oracle); returns the new count."""
    f = lib().omp_set_num_threads
    f.argtypes = [C.c_int]
    f.restype = None
    f(int(n))
    return num_threads()


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def gauss64(g):
    """Gaussian SoA planes (float32 inputs) as exact float64 copies."""
    return (_f64(g.mean), _f64(g.quat), _f64(g.scale), _f64(g.opacity), _f64(g.color))


def view_intr(rig, views):
    """Per-view pinhole intrinsics [V,4] from the camera index of each view."""
    return _f64(rig.intr[np.asarray(views.cam)])


# ----------------------------------------------------------------------------
# pose
# ----------------------------------------------------------------------------
def pose(traj, rig, xi, delta, views):
    """World->camera [V,12] (row-major [W|w]) by Eq. (1)-(2) at t_v + delta_cam."""
    V = views.n
    w2c = np.zeros((V, 12))
    seg = np.zeros(V, np.int32)
    u = np.zeros(V)
    kt, kq, kp = _f64(traj.t), _f64(traj.q), _f64(traj.p)
    R0, t0, xi_, dl = _f64(rig.R0), _f64(rig.t0), _f64(xi), _f64(delta)
    vc = np.ascontiguousarray(views.cam, np.int32)
    vt = _f64(views.t)
    rc = lib().or_pose(len(kt), _p(kt), _p(kq), _p(kp), rig.n, _p(R0), _p(t0), _p(xi_), _p(dl),
                       V, _p(vc), _p(vt), _p(w2c), _p(seg), _p(u))
    assert rc == 0
    return w2c, seg, u


def pose_bwd(traj, rig, xi, delta, views, dw2c):
    """dL/dxi [C,6] and dL/ddelta [C] from dL/dW2C [V,12]."""
    Cn = rig.n
    dxi = np.zeros((Cn, 6))
    dd = np.zeros(Cn)
    kt, kq, kp = _f64(traj.t), _f64(traj.q), _f64(traj.p)
    R0, t0, xi_, dl = _f64(rig.R0), _f64(rig.t0), _f64(xi), _f64(delta)
    vc = np.ascontiguousarray(views.cam, np.int32)
    vt = _f64(views.t)
    g = _f64(dw2c)
    rc = lib().or_pose_bwd(len(kt), _p(kt), _p(kq), _p(kp), Cn, _p(R0), _p(t0), _p(xi_), _p(dl),
                           views.n, _p(vc), _p(vt), _p(g), _p(dxi), _p(dd))
    assert rc == 0
    return dxi, dd


# ----------------------------------------------------------------------------
# projection / render / gradient
# ----------------------------------------------------------------------------
PROJ_FIELDS = ["t", "depth32", "Sc", "S2", "Q", "mu", "rad", "rect", "cull", "clx", "cly", "J"]
_PROJ_SIZES = [3, 1, 9, 3, 3, 2, 2, 4, 1, 1, 1, 6]


def project_one(x, q, s, o, w2c, intr, W, H, settings=None):
    """Projection details of one Gaussian (closed-form tests)."""
    cs = _cs(settings or Settings())
    out = np.zeros(64)
    n = lib().or_project_one(C.byref(cs), _p(_f64(x)), _p(_f64(q)), _p(_f64(s)), float(o),
                             _p(_f64(w2c)), _p(_f64(intr)), int(W), int(H), _p(out))
    res, k = {}, 0
    for name, sz in zip(PROJ_FIELDS, _PROJ_SIZES):
        res[name] = out[k:k + sz].copy() if sz > 1 else float(out[k])
        k += sz
    assert k == n
    res["Sc"] = res["Sc"].reshape(3, 3)
    res["J"] = res["J"].reshape(2, 3)
    return res


def render(g, w2c, intr, W, H, settings=None, pruned=True, alternatives=False):
    """Render every view [V]: img [V,3,H,W], T [V,H,W], last Gaussian id [V,H,W]."""
    cs = _cs(settings or Settings())
    mean, quat, scale, opac, color = gauss64(g)
    w2c = _f64(w2c).reshape(-1, 12)
    intr = _f64(intr).reshape(-1, 4)
    V = w2c.shape[0]
    img = np.zeros((V, 3, H, W))
    T = np.zeros((V, H, W))
    last = np.zeros((V, H, W), np.int64)
    nflag = np.zeros((V, H, W), np.int8)
    nalt = np.zeros((V, H, W), np.int8) if alternatives else None
    alt = np.zeros((V, H, W, 4, 5)) if alternatives else None
    stats = np.zeros(4, np.int64)
    h = C.c_uint64(0)
    pixhash = np.zeros((V, H, W), np.uint64)
    ghash = np.zeros(V, np.uint64)
    kink = np.zeros((V, H, W), np.int8)
    rc = lib().or_render(C.byref(cs), g.n, _p(mean), _p(quat), _p(scale), _p(opac), _p(color), V,
                         _p(w2c), _p(intr), int(W), int(H), int(bool(pruned)), _p(img), _p(T),
                         _p(last), _p(nflag), _p(nalt), _p(alt), _p(stats), C.byref(h),
                         _p(pixhash), _p(ghash), _p(kink))
    assert rc == 0
    out = dict(img=img, T=T, last=last, nflag=nflag, stats=dict(
        evaluated=int(stats[0]), blended=int(stats[1]), visible=int(stats[2]), flagged_px=int(stats[3])),
        hash=int(h.value), pixhash=pixhash, gausshash=ghash, kink=kink)
    if alternatives:
        out["nalt"] = nalt
        out["alt"] = alt
    return out


def grad(g, w2c, intr, W, H, dimg, settings=None, mask=None):
    """Exact adjoint: per-Gaussian gradients and dL/dW2C [V,12] for a given dL/dimg."""
    cs = _cs(settings or Settings())
    mean, quat, scale, opac, color = gauss64(g)
    w2c = _f64(w2c).reshape(-1, 12)
    intr = _f64(intr).reshape(-1, 4)
    V, G = w2c.shape[0], g.n
    dimg = _f64(dimg)
    assert dimg.shape == (V, 3, H, W)
    m = None if mask is None else np.ascontiguousarray(mask, np.int8)
    out = dict(quat=np.zeros((4, G)), scale=np.zeros((3, G)), opacity=np.zeros(G),
               color=np.zeros((3, G)), mean=np.zeros((3, G)), w2c=np.zeros((V, 12)))
    rc = lib().or_grad(C.byref(cs), G, _p(mean), _p(quat), _p(scale), _p(opac), _p(color), V,
                       _p(w2c), _p(intr), int(W), int(H), _p(dimg), _p(m), _p(out["quat"]),
                       _p(out["scale"]), _p(out["opacity"]), _p(out["color"]), _p(out["mean"]),
                       _p(out["w2c"]))
    assert rc == 0
    return out


def project_all(g, w2c, intr, W, H, settings=None):
    """Per (view, Gaussian) cull code, depth32, mu, conic, pixel rect, rect margin flag."""
    cs = _cs(settings or Settings())
    mean, quat, scale, opac, _ = gauss64(g)
    w2c = _f64(w2c).reshape(-1, 12)
    intr = _f64(intr).reshape(-1, 4)
    V, G = w2c.shape[0], g.n
    cull = np.zeros((V, G), np.int8)
    depth = np.zeros((V, G), np.float32)
    mu = np.zeros((V, G, 2))
    conic = np.zeros((V, G, 3))
    rect = np.zeros((V, G, 4), np.int32)
    rm = np.zeros((V, G), np.int8)
    lib().or_project_all(C.byref(cs), G, _p(mean), _p(quat), _p(scale), _p(opac), V, _p(w2c),
                         _p(intr), int(W), int(H), _p(cull), _p(depth), _p(mu), _p(conic),
                         _p(rect), _p(rm))
    return dict(cull=cull, depth32=depth, mu=mu, conic=conic, rect=rect, rect_margin=rm)


def pixel_stack(g, w2c, intr, W, H, x, y, settings=None, cap=4096):
    """Contributors of one pixel in blend order: rows (gid, alpha, T_before, clamped)."""
    cs = _cs(settings or Settings())
    mean, quat, scale, opac, color = gauss64(g)
    out = np.zeros((cap, 4))
    n = lib().or_pixel_stack(C.byref(cs), g.n, _p(mean), _p(quat), _p(scale), _p(opac), _p(color),
                             _p(_f64(w2c)), _p(_f64(intr)), int(W), int(H), int(x), int(y),
                             _p(out), cap)
    return out[:min(n, cap)]


# ----------------------------------------------------------------------------
# binning reference
# ----------------------------------------------------------------------------
def tile_lists(proj, W, H, tile_w, tile_h, view=0):
    """Per-tile ordered Gaussian ids of one view.

    A visible Gaussian is listed in every tile its padded pixel rect touches;
    each list is in ascending (depth32, id) order.  Returns (offsets[T+1],
    ids[I], margin[I]) where tiles are row-major over (H/tile_h) x (W/tile_w)
    (partial last row/column included) and margin marks Gaussians whose rect
    boundary sits within 1e-6 px of a rounding step.
    """
    tx_n = (W + tile_w - 1) // tile_w
    ty_n = (H + tile_h - 1) // tile_h
    vis = np.nonzero(proj["cull"][view] == 0)[0]
    rect = proj["rect"][view][vis]
    depth = proj["depth32"][view][vis]
    order = np.lexsort((vis, depth))          # depth first, then id
    vis, rect = vis[order], rect[order]
    txa, txb = rect[:, 0] // tile_w, rect[:, 1] // tile_w
    tya, tyb = rect[:, 2] // tile_h, rect[:, 3] // tile_h
    tiles_of = []
    ids = []
    for k in range(vis.shape[0]):
        for ty in range(tya[k], tyb[k] + 1):
            for tx in range(txa[k], txb[k] + 1):
                tiles_of.append(ty * tx_n + tx)
                ids.append(k)
    tiles_of = np.asarray(tiles_of, np.int64)
    ids = np.asarray(ids, np.int64)
    o = np.argsort(tiles_of, kind="stable")     # keeps (depth, id) order inside a tile
    tiles_of, ids = tiles_of[o], ids[o]
    offsets = np.searchsorted(tiles_of, np.arange(tx_n * ty_n + 1))
    gid = vis[ids]
    margin = proj["rect_margin"][view][gid].astype(bool)
    return offsets, gid, margin


# ----------------------------------------------------------------------------
# loss, pipeline helpers and finite differences
# ----------------------------------------------------------------------------
def l1_loss(img, target, mask=None, roi_y0=0):
    """Mean absolute error (the L1 term of Eq. 4) and dL/dimg with sign(0) = 0.

    With roi_y0 > 0 the loss is the mean over the rows [roi_y0, H) only (Sec. III-C:
    the losses use the bottom part of the image); dL/dimg is 0 above.  A mask
    [V,H,W] leaves pixels out of the sum without changing the mean's count."""
    d = np.array(img - target, dtype=np.float64)
    d[:, :, :roi_y0, :] = 0.0
    N = d[:, :, roi_y0:, :].size
    if mask is not None:
        d = d * (1 - mask[:, None].astype(np.float64))
    return np.abs(d).sum() / N, np.sign(d) / N


def scale_reg(scale, lam=1e-3):
    """L_scale of Sec. III-C times lambda_2: lam * sum_g ||s_g - mean(s_g)||_1 over the three
    axes of every Gaussian, and its gradient with respect to the (activated) scales [3,G]."""
    s = np.asarray(scale, np.float64)
    m = s.mean(axis=0, keepdims=True)
    sg = np.sign(s - m)
    loss = lam * np.abs(s - m).sum()
    grad = lam * (sg - sg.mean(axis=0, keepdims=True))
    return loss, grad


def render_scene(scene, gauss=None, xi=None, delta=None, settings=None, pruned=True, alternatives=False):
    """Eq. (1)-(2) then the render for every view of a scene."""
    g = scene.gauss if gauss is None else gauss
    xi = scene.xi if xi is None else xi
    delta = scene.delta if delta is None else delta
    w2c, _, _ = pose(scene.traj, scene.rig, xi, delta, scene.views)
    r = render(g, w2c, view_intr(scene.rig, scene.views), scene.rig.W, scene.rig.H,
               settings, pruned=pruned, alternatives=alternatives)
    r["w2c"] = w2c
    return r


def loss_and_grad(scene, target, gauss=None, xi=None, delta=None, settings=None, mask=None):
    """L1 loss against target images and the full gradient (Gaussians + xi + delta)."""
    g = scene.gauss if gauss is None else gauss
    xi = scene.xi if xi is None else xi
    delta = scene.delta if delta is None else delta
    r = render_scene(scene, g, xi, delta, settings)
    L, dimg = l1_loss(r["img"], target, mask)
    gr = grad(g, r["w2c"], view_intr(scene.rig, scene.views), scene.rig.W, scene.rig.H, dimg,
              settings, mask)
    dxi, dd = pose_bwd(scene.traj, scene.rig, xi, delta, scene.views, gr["w2c"])
    gr["xi"] = dxi
    gr["delta"] = dd
    return L, gr, r


def fd_loss(scene, target, gauss, xi, delta, settings=None, mask=None):
    """Loss and decision signature.

    The signature covers every decision the loss is only piecewise smooth in:
    the per-view cull and guard-clamp pattern, the per-pixel blend / stop /
    alpha-clamp sequence of every unmasked pixel, and the L1 sign pattern.
    Two evaluations with equal signatures lie on the same smooth piece.
    """
    r = render_scene(scene, gauss, xi, delta, settings)
    L, dimg = l1_loss(r["img"], target, mask)
    ph = r["pixhash"]
    if mask is not None:
        ph = np.where(mask.astype(bool), np.uint64(0), ph)
    sig = (r["gausshash"].tobytes(), ph.tobytes(), np.sign(dimg).tobytes())
    return L, sig
