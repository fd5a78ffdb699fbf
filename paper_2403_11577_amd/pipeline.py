"""Device-side driver of the splatting path on top of the C ABI.

* ``DeviceScene``  -- a scene's inputs as device tensors (SoA Gaussian planes,
  trajectory knots, rig, views, calibration state).
* ``Frame``        -- one workspace plan plus the per-step output buffers.
* ``forward`` / ``backward`` -- one batched pass over all views (pose ->
  project -> bin/sort -> render, and the reverse chain), every stage a HIP
  kernel launched through ``binding``; nothing is synchronised.
* ``per_view_plain`` -- the same kernels launched one view at a time with a
  host synchronisation after every stage (the baseline the batched path is
  compared with).
* ``SplatRender``  -- a ``torch.autograd.Function`` whose backward returns
  d(loss)/d(Gaussian params), d(loss)/d(extrinsic se(3)) and d(loss)/d(delta).

PyTorch is used for device memory and streams only.
"""
from __future__ import annotations

import dataclasses
import math

import torch

from . import binding as B


# -----------------------------------------------------------------------------
# inputs on the device
# -----------------------------------------------------------------------------
@dataclasses.dataclass
class DeviceScene:
    mean: torch.Tensor
    quat: torch.Tensor
    scale: torch.Tensor
    opacity: torch.Tensor
    color: torch.Tensor
    knot_t: torch.Tensor
    knot_q: torch.Tensor
    knot_p: torch.Tensor
    R0: torch.Tensor
    t0: torch.Tensor
    view_cam: torch.Tensor
    view_t: torch.Tensor
    intr: torch.Tensor      # per view [V,4]
    W: int
    H: int

    @property
    def n_views(self) -> int:
        return int(self.view_cam.shape[0])

    @property
    def n_gauss(self) -> int:
        return int(self.opacity.shape[0])

    @property
    def n_cams(self) -> int:
        return int(self.R0.shape[0])

    @staticmethod
    def from_scene(scene, device="cuda", views=None) -> "DeviceScene":
        """Copy a synthetic scene (numpy) to the device; `views` selects a subset of views."""
        import numpy as np

        def f32(a):
            return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=device)

        def f64(a):
            return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=device)

        g = scene.gauss
        cam = np.asarray(scene.views.cam, np.int32)
        vt = np.asarray(scene.views.t, np.float64)
        if views is not None:
            cam, vt = cam[views], vt[views]
        # what the pose kernels cannot check on the device: knot times strictly increasing,
        # every view's camera index inside the rig (checked once here, on the host copy)
        kt = np.asarray(scene.traj.t, np.float64)
        if kt.ndim != 1 or kt.size < 2 or not np.all(np.diff(kt) > 0):
            raise B.SplatError("trajectory knot times must be at least two and strictly increasing")
        n_cams = int(np.asarray(scene.rig.R0).reshape(-1, 9).shape[0])
        if cam.size and (cam.min() < 0 or cam.max() >= n_cams):
            raise B.SplatError(f"view camera indices must lie in [0, {n_cams})")
        return DeviceScene(f32(g.mean), f32(g.quat), f32(g.scale), f32(g.opacity), f32(g.color),
                           f64(scene.traj.t), f64(scene.traj.q), f64(scene.traj.p),
                           f64(scene.rig.R0.reshape(-1, 9)), f64(scene.rig.t0),
                           torch.as_tensor(cam, device=device), f64(vt),
                           f64(scene.rig.intr[cam]), int(scene.rig.W), int(scene.rig.H))

    def gaussians(self, quat=None, scale=None, opacity=None, color=None) -> B.splat_gaussians:
        return B.gaussians_struct(self.mean, self.quat if quat is None else quat,
                                  self.scale if scale is None else scale,
                                  self.opacity if opacity is None else opacity,
                                  self.color if color is None else color)


# -----------------------------------------------------------------------------
# workspace + outputs
# -----------------------------------------------------------------------------
class Frame:
    """A workspace plan for (settings, V views, G Gaussians, W x H, capacities)."""

    def __init__(self, settings: B.splat_settings, n_views: int, n_gauss: int, W: int, H: int,
                 slot_cap: int, inst_cap: int, device="cuda"):
        self.settings = settings
        self.plan = B.splat_plan_make(settings, n_views, n_gauss, W, H, slot_cap, inst_cap)
        self.device = device
        self.ws = torch.empty(int(self.plan.ws_bytes), dtype=torch.uint8, device=device)
        self.V, self.G, self.W, self.H = n_views, n_gauss, W, H
        self.img = torch.empty((n_views, 3, H, W), dtype=torch.float32, device=device)
        self.T = torch.empty((n_views, H, W), dtype=torch.float32, device=device)
        self.last = torch.empty((n_views, H, W), dtype=torch.int32, device=device)
        self.w2c = torch.empty((n_views, 12), dtype=torch.float64, device=device)
        # bumped by every render into this frame: the adjoint reads the workspace state (sorted
        # lists, checkpoints, blend masks) and T / last of the most recent forward only
        self.generation = 0
        self.clear_status()

    # typed views into the workspace ----------------------------------------------------
    def buf(self, name: str, dtype, count: int) -> torch.Tensor:
        off = int(getattr(self.plan, "off_" + name))
        nbytes = count * torch.empty((), dtype=dtype).element_size()
        return self.ws[off:off + nbytes].view(dtype)

    @property
    def status_t(self) -> torch.Tensor:
        return self.buf("status", torch.int32, 1)

    def clear_status(self):
        self.status_t.zero_()

    def status(self) -> int:
        return int(self.status_t.item()) & 0xFFFFFFFF

    def counts(self):
        c = self.buf("counts", torch.int32, 2).cpu().tolist()
        return int(c[0]) & 0xFFFFFFFF, int(c[1]) & 0xFFFFFFFF

    def sorted_vals(self, n: int) -> torch.Tensor:
        base = self.buf("vals", torch.int32, 2 * int(self.plan.inst_cap))
        o = int(self.plan.inst_cap) if self.plan.sorted_buf else 0
        return base[o:o + n]

    def sorted_keys(self, n: int) -> torch.Tensor:
        """The sorted keys: int64, or int32 (key >> plan.key_shift) when the sort narrowed them."""
        base = self.buf("keys", torch.int64, 2 * int(self.plan.inst_cap))
        o = int(self.plan.inst_cap) if self.plan.sorted_buf else 0
        if int(self.plan.key_shift) >= 0:
            return base[o:o + int(self.plan.inst_cap)].view(torch.int32)[:n]
        return base[o:o + n]

    def ranges(self) -> torch.Tensor:
        n = self.V * int(self.plan.tiles_per_view)
        return self.buf("ranges", torch.int32, 2 * n).view(n, 2)

    def records(self, n: int) -> torch.Tensor:
        return self.buf("rec", torch.float32, 12 * n).view(n, 12)

    def meta(self, n: int) -> torch.Tensor:
        # (Gaussian id, view) per slot of the last projection, written on demand
        B.splat_slot_meta(self.plan, self.ws)
        return self.buf("meta", torch.int32, 2 * n).view(n, 2)

    def grad2d(self, n: int) -> torch.Tensor:
        return self.buf("grad2d", torch.float32, 9 * n).view(n, 9)


def make_settings(tile=(16, 16), batch=64, persistent=True, **kw) -> B.splat_settings:
    return B.default_settings(tile_w=int(tile[0]), tile_h=int(tile[1]), batch=int(batch),
                              persistent=int(bool(persistent)), **kw)


# -----------------------------------------------------------------------------
# one batched pass
# -----------------------------------------------------------------------------
def pose_fwd(fr: Frame, ds: DeviceScene, xi: torch.Tensor, delta: torch.Tensor):
    B.splat_pose_interp_fwd(ds.knot_t, ds.knot_q, ds.knot_p, ds.R0, ds.t0, xi, delta, ds.view_cam, ds.view_t,
                            fr.w2c, fr.status_t)
    return fr.w2c


def forward(fr: Frame, ds: DeviceScene, xi: torch.Tensor, delta: torch.Tensor, gauss=None, w2c=None, l1=None):
    """pose -> project -> bin/sort -> render; returns (img, T_final, last_pos).  With l1 = (target,
    mask, dimg, loss, weight) the render also forms the L1 term over the plan's region of
    interest in the same launch (splat_render_fwd_l1)."""
    if w2c is None:
        w2c = pose_fwd(fr, ds, xi, delta)
    else:
        fr.w2c.copy_(w2c)
    g = ds.gaussians() if gauss is None else gauss
    fr.generation += 1
    B.splat_project(fr.plan, fr.ws, g, fr.w2c, ds.intr)
    B.splat_bin_sort(fr.plan, fr.ws)
    if l1 is None:
        B.splat_render_fwd(fr.plan, fr.ws, fr.img, fr.T, fr.last)
    else:
        target, mask, dimg, loss, weight = l1
        B.splat_render_fwd_l1(fr.plan, fr.ws, fr.img, fr.T, fr.last, target, mask, dimg, loss, weight)
    return fr.img, fr.T, fr.last


@dataclasses.dataclass
class Grads:
    quat: torch.Tensor
    scale: torch.Tensor
    opacity: torch.Tensor
    color: torch.Tensor
    mean: torch.Tensor
    w2c: torch.Tensor
    xi: torch.Tensor
    delta: torch.Tensor


def alloc_grads(ds: DeviceScene, with_mean=False, n_extra64=0) -> Grads:
    """Gradient buffers as views of one float32 and one float64 allocation (each view 256-byte
    aligned), so that zero_grads clears them with two fills.  n_extra64 float64 values more
    (gr.extra64, cleared with them) hold what a step accumulates besides the gradients."""
    dev = ds.opacity.device
    G, V, Cn = ds.n_gauss, ds.n_views, ds.n_cams
    pad = lambda k, q: -(-k // q) * q
    Gp = pad(G, 64)
    rows32 = [4, 3, 1, 3] + ([3] if with_mean else [])
    f32 = torch.zeros(Gp * sum(rows32), dtype=torch.float32, device=dev)
    views, o = [], 0
    for r in rows32:
        views.append(f32[o:o + r * G].view(r, G) if r > 1 else f32[o:o + G])
        o += r * Gp
    n64 = [V * 12, Cn * 6, Cn] + ([n_extra64] if n_extra64 else [])
    f64 = torch.zeros(sum(pad(k, 32) for k in n64), dtype=torch.float64, device=dev)
    o, v64 = 0, []
    for k in n64:
        v64.append(f64[o:o + k])
        o += pad(k, 32)
    gr = Grads(views[0], views[1], views[2], views[3], views[4] if with_mean else None,
               v64[0].view(V, 12), v64[1].view(Cn, 6), v64[2])
    gr._flat = (f32, f64)
    gr.extra64 = v64[3] if n_extra64 else None
    return gr


def zero_grads(gr: Grads):
    flat = getattr(gr, "_flat", None)
    if flat is not None:
        for t in flat:
            t.zero_()
        return
    for f in dataclasses.fields(gr):
        t = getattr(gr, f.name)
        if t is not None:
            t.zero_()


def backward(fr: Frame, ds: DeviceScene, xi, delta, dimg: torch.Tensor, gr: Grads, gauss=None,
             pose=True) -> Grads:
    """render_bwd -> project_bwd -> pose_bwd, ADDING into gr (zero it first)."""
    g = ds.gaussians() if gauss is None else gauss
    B.splat_render_bwd(fr.plan, fr.ws, dimg, fr.T, fr.last)
    B.splat_project_bwd(fr.plan, fr.ws, g, fr.w2c, ds.intr, gr.quat, gr.scale, gr.opacity, gr.color,
                        gr.mean, gr.w2c)
    if pose:
        B.splat_pose_interp_bwd(ds.knot_t, ds.knot_q, ds.knot_p, ds.R0, ds.t0, xi, delta, ds.view_cam,
                                ds.view_t, gr.w2c, gr.xi, gr.delta)
    return gr


def fit_frame(ds: DeviceScene, xi, delta, settings=None, slot_cap=None, inst_cap=None, margin=1.15,
              w2c=None) -> Frame:
    """Make a Frame whose capacities fit this scene (probe run, then exact counts + margin)."""
    settings = settings or make_settings()
    V, G = ds.n_views, ds.n_gauss
    sc = slot_cap or max(1, V * G)
    ic = inst_cap or max(1024, min(4 * V * G + 1024, (1 << 31) - 1))
    while True:
        fr = Frame(settings, V, G, ds.W, ds.H, sc, ic, ds.opacity.device)
        forward(fr, ds, xi, delta, w2c=w2c)
        st = fr.status()
        if not (st & B.ST_CAPACITY):
            break
        ns, ni = fr.counts()
        if ns >= sc:
            sc = min(V * G, 2 * sc)
        ic = min((1 << 31) - 1, 2 * ic)
        del fr
    ns, ni = fr.counts()
    want_s = max(1, min(V * G, int(math.ceil(ns * margin)) + 256))
    want_i = max(1024, int(math.ceil(ni * margin)) + 4096)
    if want_s < sc or want_i < ic:
        fr = Frame(settings, V, G, ds.W, ds.H, min(sc, want_s), min(ic, want_i), ds.opacity.device)
    return fr


# -----------------------------------------------------------------------------
# loss (L1 part of Eq. 4)
# -----------------------------------------------------------------------------
def l1_loss_grad(img: torch.Tensor, target: torch.Tensor, mask=None, dimg=None, loss=None, roi_y0=0):
    """L1 mean and its gradient sign(img - target)/N (sign(0) = 0), by the library's L1 kernel.

    mask (optional) is a bool/uint8 [V,H,W] tensor of pixels to leave out; roi_y0 restricts
    the mean to the rows [roi_y0, H).  Returns (loss [1] float64 device tensor, dimg)."""
    if dimg is None:
        dimg = torch.empty_like(img)
    if loss is None:
        loss = torch.zeros(1, dtype=torch.float64, device=img.device)
    m = None if mask is None else mask.to(torch.uint8).contiguous()
    B.splat_l1_loss_grad(img, target.contiguous(), m, dimg, loss, roi_y0)
    return loss, dimg


class BatchedStep:
    """One calibration step over all views, batched: pose -> project -> bin/sort ->
    render + L1 -> render_bwd -> project_bwd -> pose_bwd, every stage one set of
    launches for all views (persistent render over the cost-ordered queue).  The
    step can be captured once in a HIP graph and replayed."""

    def __init__(self, ds: DeviceScene, xi, delta, targets, settings=None, fr: Frame = None, mask=None):
        self.ds, self.xi, self.delta = ds, xi, delta
        self.targets = targets.contiguous()
        self.mask = None if mask is None else mask.to(torch.uint8).contiguous()
        self.fr = fr or fit_frame(ds, xi, delta, settings)
        self.gr = alloc_grads(ds, n_extra64=1)
        self.dimg = torch.empty_like(self.fr.img)
        self.loss = self.gr.extra64  # cleared with the gradients
        self.graph = None
        self.events = None  # optional list of (start, end) event pairs per stage

    def run(self):
        fr, ds = self.fr, self.ds
        zero_grads(self.gr)
        pose_fwd(fr, ds, self.xi, self.delta)
        fr.generation += 1
        B.splat_project(fr.plan, fr.ws, ds.gaussians(), fr.w2c, ds.intr)
        B.splat_bin_sort(fr.plan, fr.ws)
        ev = self.events
        if ev: ev["fwd"][0].record()
        # the forward and the L1 term in one launch (the loss kernel's outputs, bit for bit)
        B.splat_render_fwd_l1(fr.plan, fr.ws, fr.img, fr.T, fr.last, self.targets, self.mask, self.dimg, self.loss)
        if ev: ev["fwd"][1].record()
        if ev: ev["bwd"][0].record()
        B.splat_render_bwd(fr.plan, fr.ws, self.dimg, fr.T, fr.last)
        if ev: ev["bwd"][1].record()
        B.splat_project_bwd(fr.plan, fr.ws, ds.gaussians(), fr.w2c, ds.intr, self.gr.quat, self.gr.scale,
                            self.gr.opacity, self.gr.color, None, self.gr.w2c)
        B.splat_pose_interp_bwd(ds.knot_t, ds.knot_q, ds.knot_p, ds.R0, ds.t0, self.xi, self.delta, ds.view_cam,
                                ds.view_t, self.gr.w2c, self.gr.xi, self.gr.delta)

    def capture(self):
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.run()  # warm-up outside the graph
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        ev, self.events = self.events, None
        with torch.cuda.graph(g):
            self.run()
        self.events = ev
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()

    def stats(self):
        """Pair counters of one instrumented fwd/bwd on the current inputs (not timed)."""
        fr, ds = self.fr, self.ds
        st = torch.zeros(8, dtype=torch.int64, device=ds.opacity.device)
        pose_fwd(fr, ds, self.xi, self.delta)
        fr.generation += 1
        B.splat_project(fr.plan, fr.ws, ds.gaussians(), fr.w2c, ds.intr)
        B.splat_bin_sort(fr.plan, fr.ws)
        B.splat_render_fwd_stats(fr.plan, fr.ws, fr.img, fr.T, fr.last, st)
        B.splat_l1_loss_grad(fr.img, self.targets, self.mask, self.dimg, None, fr.settings.roi_y0)
        B.splat_render_bwd_stats(fr.plan, fr.ws, self.dimg, fr.T, fr.last, st)
        torch.cuda.synchronize()
        v = st.cpu().tolist()
        ns, ni = fr.counts()
        return dict(fwd_eval=v[0], fwd_blend=v[1], bwd_eval=v[2], bwd_contrib=v[3], bwd_atomic_groups=v[4],
                    fwd_wave_evals=v[5], fwd_wave_blends=v[6], bwd_wave_evals=v[7], slots=ns, instances=ni)


# -----------------------------------------------------------------------------
# per-view plain launch (baseline)
# -----------------------------------------------------------------------------
class PerViewPlain:
    """The same kernels launched one view at a time: one workspace per view sized
    from the host-read counts, a host synchronisation after every stage, no
    persistence, no graph."""

    def __init__(self, ds: DeviceScene, xi, delta, settings=None):
        self.ds = ds
        base = settings or make_settings()
        s = B.default_settings()
        for name, _ in B.splat_settings._fields_:
            setattr(s, name, getattr(base, name))
        s.persistent = 0
        self.settings = s
        self.views = []
        for v in range(ds.n_views):
            dv = DeviceScene(ds.mean, ds.quat, ds.scale, ds.opacity, ds.color, ds.knot_t, ds.knot_q,
                             ds.knot_p, ds.R0, ds.t0, ds.view_cam[v:v + 1].contiguous(),
                             ds.view_t[v:v + 1].contiguous(), ds.intr[v:v + 1].contiguous(), ds.W, ds.H)
            fr = fit_frame(dv, xi, delta, s)
            self.views.append((dv, fr, alloc_grads(dv)))

    def step(self, xi, delta, targets, gr: Grads, sync=True):
        """fwd + L1 + bwd over every view, one view at a time; returns the loss (a device
        tensor when sync is False: then no stage waits for the host and no count is read)."""
        total = 0.0
        sync_fn = torch.cuda.synchronize if sync else (lambda: None)
        for v, (dv, fr, g1) in enumerate(self.views):
            fr.generation += 1
            pose_fwd(fr, dv, xi, delta); sync_fn()
            B.splat_project(fr.plan, fr.ws, dv.gaussians(), fr.w2c, dv.intr); sync_fn()
            if sync:
                fr.counts()
            B.splat_bin_sort(fr.plan, fr.ws); sync_fn()
            if sync:
                fr.counts()
            B.splat_render_fwd(fr.plan, fr.ws, fr.img, fr.T, fr.last); sync_fn()
            L, dimg = l1_loss_grad(fr.img, targets[v:v + 1], roi_y0=fr.settings.roi_y0)
            dimg.mul_(1.0 / len(self.views))  # mean over all views, as in the batched step
            total = total + (float(L) if sync else L) / len(self.views)
            zero_grads(g1)
            B.splat_render_bwd(fr.plan, fr.ws, dimg, fr.T, fr.last); sync_fn()
            B.splat_project_bwd(fr.plan, fr.ws, dv.gaussians(), fr.w2c, dv.intr, g1.quat, g1.scale,
                                g1.opacity, g1.color, None, g1.w2c); sync_fn()
            B.splat_pose_interp_bwd(dv.knot_t, dv.knot_q, dv.knot_p, dv.R0, dv.t0, xi, delta, dv.view_cam,
                                    dv.view_t, g1.w2c, g1.xi, g1.delta); sync_fn()
            gr.quat += g1.quat; gr.scale += g1.scale; gr.opacity += g1.opacity; gr.color += g1.color
            gr.xi += g1.xi; gr.delta += g1.delta
        return total


# -----------------------------------------------------------------------------
# autograd
# -----------------------------------------------------------------------------
class SplatRender(torch.autograd.Function):
    """img = Phi(X, quat, scale, opacity, color; pose(xi, delta)) for all views.

    backward returns d(loss)/d quat, scale, opacity, colour, d(loss)/d xi
    (extrinsic se(3) correction, rho then phi) and d(loss)/d delta (time offset),
    all from the hand-written adjoint kernels.

    The adjoint reads what the forward left in the Frame (sorted lists, checkpoints,
    blend masks, T and last contributor), so one Frame serves one live graph node:
    rendering into the same Frame again before this node's backward makes the
    backward raise instead of returning the gradients of the other render.
    """

    @staticmethod
    def forward(ctx, quat, scale, opacity, color, xi, delta, fr: Frame, ds: DeviceScene):
        g = ds.gaussians(quat, scale, opacity, color)
        forward(fr, ds, xi, delta, gauss=g)
        ctx.fr, ctx.ds, ctx.generation = fr, ds, fr.generation
        ctx.save_for_backward(quat, scale, opacity, color, xi, delta)
        return fr.img.clone()

    @staticmethod
    def backward(ctx, dimg):
        quat, scale, opacity, color, xi, delta = ctx.saved_tensors
        fr, ds = ctx.fr, ctx.ds
        if fr.generation != ctx.generation:
            raise B.SplatError("SplatRender.backward: the Frame was rendered into again after this forward; "
                               "give each live render its own Frame")
        gr = alloc_grads(ds)
        g = ds.gaussians(quat, scale, opacity, color)
        backward(fr, ds, xi, delta, dimg.contiguous(), gr, gauss=g)
        return gr.quat, gr.scale, gr.opacity, gr.color, gr.xi, gr.delta, None, None


def voxel_downsample(pts: torch.Tensor, voxel: float, lo=None, ws=None):
    """Indices (int64, device) of one point per voxel of pts [3, n] (the lowest index,
    in voxel order); lo defaults to the cloud's minimum.  Synchronises once to read
    the count.  Raises if a point fell outside the voxel grid."""
    n = int(pts.shape[1])
    if lo is None:
        lo = pts.min(dim=1).values.double().cpu().tolist() if n else [0.0, 0.0, 0.0]
    need = B.splat_voxel_workspace_size(n)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=pts.device)
    keep = torch.empty(max(n, 1), dtype=torch.int32, device=pts.device)
    cnt = torch.zeros(2, dtype=torch.int32, device=pts.device)   # n_keep, status
    B.splat_voxel_downsample(pts, lo, voxel, ws, keep, cnt[0:1], cnt[1:2])
    m, st = cnt.cpu().tolist()
    if st & B.ST_RANGE:
        raise B.SplatError(f"voxel_downsample: points outside the {voxel} m grid from {lo}")
    return keep[:m].long()
