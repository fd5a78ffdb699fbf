"""The calibration loop of 3DGS-Calib on top of the batched differentiable renderer.

Sec. III and IV-B of the paper: Gaussians anchored at the LiDAR points (means
fixed), view-independent colours initialised at random, scales / rotations /
opacities initialised as in 3DGS; Adam with learning rates 1e-4 (rotation),
5e-3 (translation) and 1e-3 (time offset), linearly decayed to 0.1x over the
run; a warm-up during which the calibration is frozen.  Every step renders a
batch of views forward and backward through the HIP path (pose interpolation,
projection, binning, compositing, L1, adjoints); the optimiser and the parameter
activations (sigmoid opacity, exponential scale) are plain torch.

Learning rates of the Gaussian parameters are not given in the paper; those of
the original 3DGS implementation are used.  As in Sec. III-C, only the bottom
rows of every image are rendered and enter the loss (roi_frac); the photometric
loss is Eq. (4), 0.8 L1 + 0.2 D-SSIM, and L_scale (lambda_2 = 1e-3) is added.

With the field model F(X|Theta) the Gaussians can follow the coarse-to-fine
schedule of Sec. III-C and IV-B: each stage re-anchors them at one point per
voxel of the accumulated cloud (10, 5, then 2 cm) and bounds their scales by the
voxel size; the field, its optimiser state and the calibration carry over.
"""
from __future__ import annotations

import dataclasses
import math
import time

import numpy as np
import torch

from . import binding as B
from . import pipeline as pl


# coarse-to-fine schedules of Sec. IV-B: (voxel size in metres, steps)
PAPER_STAGES = ((0.10, 4000), (0.05, 1000), (0.02, 1000))
PAPER_STAGES_LIDAR_CAMERA = ((0.10, 2000), (0.05, 500), (0.02, 500))


@dataclasses.dataclass
class CalibConfig:
    steps: int = 3000
    warmup: int = 500
    batch_views: int = 16
    lr_rot: float = 1e-4
    lr_trans: float = 5e-3
    lr_time: float = 1e-3
    lr_color: float = 2.5e-3
    lr_opacity: float = 5e-2
    lr_scale: float = 5e-3
    lr_quat: float = 1e-3
    final_lr_frac: float = 0.1
    init_opacity: float = 0.1
    seed: int = 0
    # "random": colours U[0,1), opacity init_opacity, identity rotations, the scene's scales;
    # "scene": start from the scene's own Gaussians (pure registration when frozen)
    gauss_init: str = "random"
    freeze_gaussians: bool = False
    # Sec. III-C: losses on the bottom part of the image only, and the scale regulariser
    roi_frac: float = 0.5          # fraction of the rows (from the bottom) that is rendered
    lam_scale: float = 1e-3        # lambda_2 of L_scale (0 disables it)
    lam_dssim: float = 0.2         # lambda_1 of Eq. 4: L_photo = (1 - lambda_1) L1 + lambda_1 D-SSIM
    # Gaussian parameters: "field" = F(X|Theta), hash grid + MLP with four heads (Sec. III-C);
    # "independent" = one free parameter set per Gaussian (the 3DGS model without the field)
    model: str = "independent"
    field_levels: int = 16
    field_log2_table: int = 19
    field_n_min: int = 16
    field_n_max: int = 4096
    field_scale_max: float = 0.05  # the voxel size of the point cloud (scales stay below it)
    lr_field_table: float = 1e-2
    lr_field_mlp: float = 1e-3
    field_weight_decay: float = 1e-4   # on the hash grid (Sec. IV-B)
    # coarse-to-fine voxelisation (field model): ((voxel_m, steps), ...); steps is then their sum.
    # () keeps the scene's own points for the whole run.
    stages: tuple = ()
    # replay each step's device work from a captured HIP graph (re-captured when the plan changes)
    graph: bool = True
    # every this many steps, and after every stage change, time the candidate tile shapes on a few
    # real steps and keep the fastest (the best shape moves with the Gaussians' opacities); 0 keeps
    # the given settings
    tile_tune: int = 500
    # the candidates include, for each tile shape, the forward that composites the chunks of long
    # tile lists in parallel and joins them (pays off while few pixels saturate)
    tune_split_fwd: bool = True
    # instances per chunk of a split tile list: the faint Gaussians of a calibration leave long,
    # unsaturated lists, which short chunks balance best (128 against 1,024 for saturating scenes)
    split_len: int = 128
    fused_adam: bool = True        # torch's single-kernel Adam (else its multi-tensor one)
    # independent Gaussians: the library's Adam step over the four parameter arrays in one launch,
    # fused with their activations and the clearing of their gradients (else torch's Adam)
    native_adam: bool = True


def rotation_error_deg(xi):
    """Geodesic angle of R0 Exp(phi) against the ground truth R0 (phi = 0)."""
    return np.degrees(np.linalg.norm(np.asarray(xi)[:, 3:], axis=1))


class Calibrator:
    """Optimises Gaussians, extrinsic corrections xi = (rho, phi) and time offsets delta."""

    def __init__(self, scene, cfg: CalibConfig = None, settings=None, device="cuda", cloud=None):
        """cloud: the accumulated LiDAR points [3, n] (device float32) the stages downsample;
        defaults to the scene's Gaussian means."""
        self.cfg = cfg = cfg or CalibConfig()
        if cfg.stages:
            if cfg.model != "field":
                raise ValueError("the coarse-to-fine stages need the field model (model='field')")
            cfg = self.cfg = dataclasses.replace(cfg, steps=int(sum(int(n) for _, n in cfg.stages)))
        self.scene = scene
        self.device = device
        full = pl.DeviceScene.from_scene(scene, device=device)
        self.full = full
        V, G, Bv = full.n_views, full.n_gauss, cfg.batch_views
        base = settings or pl.make_settings()
        roi = min(max(int(round(full.H * (1.0 - cfg.roi_frac))), 0), full.H - 1)
        # candidates (tile, joined forward); the first is the given settings
        cands = [((base.tile_w, base.tile_h), int(base.split_fwd))]
        if cfg.tile_tune:
            sfs = (0, 1) if cfg.tune_split_fwd else (int(base.split_fwd),)
            cands += [(t, sf) for t in ((16, 16), (8, 8)) for sf in sfs if (t, sf) != cands[0]]
        self._cands = [pl.make_settings(tile=t, batch=base.batch, roi_y0=roi,
                                        persistent=bool(base.persistent) if i == 0 else False,
                                        split_len=base.split_len or cfg.split_len, split_fwd=sf)
                       for i, (t, sf) in enumerate(cands)]
        self._cur = 0
        self.settings = self._cands[0]
        self._frames, self._graphs, self._caps = {}, {}, {}
        self._next_tune = 2 if cfg.tile_tune else None
        self._trial, self._trial_ev = [], {}
        self.tile_log = []
        # targets: every view rendered at the ground-truth calibration with the true Gaussians
        zx = torch.zeros((full.n_cams, 6), dtype=torch.float64, device=device)
        zd = torch.zeros(full.n_cams, dtype=torch.float64, device=device)
        self.targets = torch.empty((V, 3, full.H, full.W), dtype=torch.float32, device=device)
        counts = []
        for v0 in range(0, V, Bv):
            sub = self._subscene(full, torch.arange(v0, min(V, v0 + Bv), device=device))
            fr = pl.fit_frame(sub, zx, zd, self.settings)
            img, _, _ = pl.forward(fr, sub, zx, zd)
            self.targets[v0:v0 + sub.n_views] = img
            counts.append(fr.counts())
            del fr
        # capacity: the largest batch seen, with a wide margin for footprints that grow in training
        self._ns = max(c[0] for c in counts)
        self._ni = max(c[1] for c in counts)
        self.cloud = full.mean if cloud is None else cloud
        self.stage_starts = np.cumsum([0] + [int(n) for _, n in cfg.stages])[:-1].tolist()
        self.stage = -1
        self.stage_log = []
        self._set_points(full.mean)
        # the batch's targets: only the rows of the region of interest are gathered each step (the
        # losses read none above it; those rows stay zero)
        self.tgt = torch.zeros((Bv, 3, full.H, full.W), dtype=torch.float32, device=device)
        # parameters (raw) and their activations
        if cfg.gauss_init == "scene":
            o = full.opacity.clamp(1e-6, 1 - 1e-6)
            self.color = full.color.clone().requires_grad_(True)
            self.logit_o = torch.log(o / (1 - o)).requires_grad_(True)
            self.quat = full.quat.clone().requires_grad_(True)
        else:
            g = torch.Generator(device="cpu").manual_seed(cfg.seed)
            self.color = torch.rand((3, G), generator=g).to(device).requires_grad_(True)
            self.logit_o = torch.full((G,), math.log(cfg.init_opacity / (1 - cfg.init_opacity)), device=device,
                                      requires_grad=True)
            q = torch.zeros((4, G), device=device)
            q[0] = 1.0
            self.quat = q.requires_grad_(True)
        self.log_s = torch.log(full.scale.clone()).requires_grad_(True)
        self.field = None
        if cfg.model == "field":
            self._init_field(full, cfg)
        else:
            # the render reads the colour and rotation parameters in place (the optimiser updates
            # them in place too); opacity and scale are activations formed every step
            self.win.color = self.color.detach()
            self.win.quat = self.quat.detach()
        self.rho = torch.tensor(scene.xi[:, :3], dtype=torch.float64, device=device).requires_grad_(True)
        self.phi = torch.tensor(scene.xi[:, 3:], dtype=torch.float64, device=device).requires_grad_(True)
        self.delta = torch.tensor(scene.delta, dtype=torch.float64, device=device).requires_grad_(True)
        # two optimisers: the calibration one only starts stepping after the warm-up
        # in graph mode the learning rates are device tensors, updated before every replay
        lr = (lambda v: torch.tensor(v, dtype=torch.float32, device=device)) if cfg.graph else float
        self.opt_g = torch.optim.Adam([
            dict(params=[self.color], lr=lr(cfg.lr_color)),
            dict(params=[self.logit_o], lr=lr(cfg.lr_opacity)),
            dict(params=[self.log_s], lr=lr(cfg.lr_scale)),
            dict(params=[self.quat], lr=lr(cfg.lr_quat)),
        ] if self.field is None else [
            dict(params=[self.field["tables"]], lr=lr(cfg.lr_field_table), weight_decay=cfg.field_weight_decay),
            dict(params=[self.field[k] for k in ("w1", "b1", "w2", "b2", "w3", "b3")], lr=lr(cfg.lr_field_mlp)),
        ], eps=1e-15, capturable=cfg.graph, fused=cfg.fused_adam or None)
        self.opt_c = torch.optim.Adam([
            dict(params=[self.rho], lr=lr(cfg.lr_trans)),
            dict(params=[self.phi], lr=lr(cfg.lr_rot)),
            dict(params=[self.delta], lr=lr(cfg.lr_time)),
        ], eps=1e-15, capturable=cfg.graph, fused=cfg.fused_adam or None)
        self.base_lr = [[float(grp["lr"]) for grp in o.param_groups] for o in (self.opt_g, self.opt_c)]
        self._native = self.field is None and cfg.native_adam
        if self._native:
            # moments, a step counter and device learning rates of the library's Adam step, in the
            # order of opt_g's groups (colour, opacity logit, log scale, rotation); the render's
            # activations are formed once here and then rewritten by every step
            raw = (self.color, self.logit_o, self.log_s, self.quat)
            self._nat_m = [torch.zeros_like(t) for t in raw]
            self._nat_v = [torch.zeros_like(t) for t in raw]
            self._nat_lr0 = torch.tensor(self.base_lr[0], dtype=torch.float32, device=device)
            self._nat_lr_all = self._nat_lr0.clone()
            self._nat_lr = [self._nat_lr_all[i:i + 1] for i in range(len(self.base_lr[0]))]
            self._nat_step = torch.zeros(1, dtype=torch.float32, device=device)
            with torch.no_grad():
                torch.sigmoid(self.logit_o, out=self.win.opacity)
                torch.exp(self.log_s, out=self.win.scale)
        # gradient buffers the step writes in place (fixed addresses, as a captured graph needs)
        for t in (self.rho, self.phi, self.delta):
            t.grad = torch.zeros_like(t)
        if self.field is None:
            self.logit_o.grad = torch.zeros_like(self.logit_o)
            self.log_s.grad = torch.zeros_like(self.log_s)
        self._graph = None
        if self.field is not None:
            self.field_grads = {k: torch.zeros_like(v) for k, v in self.field.items()}
            for name, t in self.field.items():
                t.grad = self.field_grads[name]
        self.xi_t = torch.zeros((full.n_cams, 6), dtype=torch.float64, device=device)
        self.dl_t = torch.zeros(full.n_cams, dtype=torch.float64, device=device)
        self.loss = torch.zeros(1, dtype=torch.float64, device=device)
        self.ssim_ws = torch.empty(B.splat_dssim_workspace_size(Bv, full.W, full.H, self.settings.roi_y0),
                                   dtype=torch.uint8, device=device)
        # view order: epochs of seeded permutations, drawn on the device (no host copy per step)
        self._perm_gen = torch.Generator(device=device).manual_seed(cfg.seed)
        self.order = torch.empty(0, dtype=torch.int64, device=device)
        # status words of the last two steps, copied to pinned memory and read two steps later
        self._st_host = torch.zeros((2, 1), dtype=torch.int32).pin_memory()
        self._st_ev = [None, None]
        self.overflow_steps = []
        self.replans = 0

    def _init_field(self, full, cfg):
        """F(X|Theta): tables U(-1e-4, 1e-4), weights uniform(+-sqrt(6 / fan_in)), biases 0 (seeded)."""
        G, dev = full.n_gauss, full.mean.device
        g = torch.Generator(device="cpu").manual_seed(cfg.seed + 1)
        T, L, H = 1 << cfg.field_log2_table, cfg.field_levels, 64
        D = 2 * L

        def uni(shape, bound):
            return ((torch.rand(shape, generator=g) * 2 - 1) * bound).to(dev)

        self.field = dict(tables=uni((L, T, 2), 1e-4), w1=uni((H, D), math.sqrt(6.0 / D)), b1=torch.zeros(H, device=dev),
                          w2=uni((H, H), math.sqrt(6.0 / H)), b2=torch.zeros(H, device=dev),
                          w3=uni((11, H), math.sqrt(6.0 / H)), b3=torch.zeros(11, device=dev))
        for t in self.field.values():
            t.requires_grad_(True)
        lo = self.cloud.min(dim=1).values.double().cpu().numpy() - 1.0
        hi = self.cloud.max(dim=1).values.double().cpu().numpy() + 1.0
        self._field_box = (lo, hi)
        self._set_scale_max(cfg.field_scale_max)

    def _set_scale_max(self, scale_max):
        cfg, f = self.cfg, self.field
        conf = type("FieldCfg", (), dict(levels=cfg.field_levels, feat=2, log2_table=cfg.field_log2_table,
                                         n_min=cfg.field_n_min, n_max=cfg.field_n_max, hidden=64,
                                         scale_max=float(scale_max)))
        lo, hi = self._field_box
        self.field_struct = B.ngp_struct(conf, lo, hi, f["tables"], f["w1"], f["b1"], f["w2"], f["b2"], f["w3"],
                                         f["b3"])

    def _set_points(self, mean):
        """Anchor the Gaussians at mean [3, G] (window scene, plan, gradients, scratch)."""
        full, Bv, dev = self.full, self.cfg.batch_views, self.device
        G = int(mean.shape[1])
        z = lambda *s: torch.zeros(s, dtype=torch.float32, device=dev)
        idx = torch.arange(Bv, device=dev) % full.n_views
        self.win = pl.DeviceScene(mean, z(4, G), z(3, G), z(G), z(3, G), full.knot_t, full.knot_q, full.knot_p,
                                  full.R0, full.t0, full.view_cam[idx].contiguous(), full.view_t[idx].contiguous(),
                                  full.intr[idx].contiguous(), full.W, full.H)
        # slots scale with the number of Gaussians; instances per slot as in the targets (with the
        # first candidate's tiles; smaller tiles cut a footprint into more of them)
        r = G / max(1, full.n_gauss)
        slot_cap = int(min(Bv * G, self._ns * 2 * r + 1024))
        inst_cap = self._ni * 3 * r + 4096
        a0 = self._cands[0].tile_w * self._cands[0].tile_h
        self._caps = {i: (slot_cap, int(min((1 << 31) - 1, inst_cap * max(1.0, (a0 / (c.tile_w * c.tile_h)) ** 0.75))))
                      for i, c in enumerate(self._cands)}
        self._frames, self._graphs = {}, {}
        self._use(self._cur)
        self.gr = pl.alloc_grads(self.win)
        self.dimg = torch.empty_like(self.fr.img)
        if self.cfg.model == "field":
            self.field_ws = torch.empty(B.splat_ngp_workspace_size(G), dtype=torch.uint8, device=dev)

    def _use(self, ci):
        """Render with candidate ci from now on (its plan and graph are kept for later switches)."""
        self._cur = ci
        self.settings = self._cands[ci]
        if ci not in self._frames:
            sc, ic = self._caps[ci]
            self._frames[ci] = pl.Frame(self.settings, self.cfg.batch_views, self.win.n_gauss, self.full.W,
                                        self.full.H, sc, ic, self.device)
        self.fr = self._frames[ci]
        self.slot_cap, self.inst_cap = self._caps[ci]
        self.dimg = getattr(self, "dimg", None)
        if self.dimg is None or self.dimg.shape != self.fr.img.shape:
            self.dimg = torch.empty_like(self.fr.img)
        self._graph = self._graphs.get(ci)

    def _ensure_index(self):
        """Inverse index of the field's table lookups for the current anchors (built once per
        set of positions: the table adjoint then needs no atomics)."""
        if getattr(self, "_index_mean", None) is self.win.mean:
            return
        self.field_index = None
        G = self.win.n_gauss
        self.field_index = torch.empty(B.splat_ngp_index_size(self.field_struct, G), dtype=torch.uint8,
                                       device=self.device)
        ws = torch.empty(B.splat_ngp_index_workspace_size(self.field_struct, G), dtype=torch.uint8,
                         device=self.device)
        B.splat_ngp_index_build(self.field_struct, self.win.mean, self.field_index, ws)
        del ws
        self._index_mean = self.win.mean

    def _enter_stage(self, i):
        """Stage i of the coarse-to-fine schedule: one point per voxel of the cloud, scales below the voxel."""
        voxel, n = self.cfg.stages[i]
        self._close_stage()
        t0 = time.perf_counter()
        keep = pl.voxel_downsample(self.cloud, float(voxel))
        mean = self.cloud[:, keep].contiguous()
        self._set_points(mean)
        self._set_scale_max(voxel)
        self._ensure_index()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        self.stage = i
        if self.cfg.tile_tune:
            self._trial = []
            self._next_tune = self.stage_starts[i] + 1
        self.stage_log.append(dict(voxel_m=float(voxel), steps=int(n), gaussians=int(mean.shape[1]),
                                   setup_ms=round((t1 - t0) * 1e3, 2), done=0, _t0=t1))

    def _close_stage(self):
        """Wall time and step rate of the running stage (synchronises)."""
        if self.stage_log and "_t0" in self.stage_log[-1]:
            torch.cuda.synchronize()
            e = self.stage_log[-1]
            sec = time.perf_counter() - e.pop("_t0")
            e["seconds"] = round(sec, 3)
            e["steps_per_s"] = round(e["done"] / sec, 2) if sec > 0 else None

    @staticmethod
    def _subscene(full, idx):
        return pl.DeviceScene(full.mean, full.quat.clone(), full.scale.clone(), full.opacity.clone(),
                              full.color.clone(), full.knot_t, full.knot_q, full.knot_p, full.R0, full.t0,
                              full.view_cam[idx].contiguous(), full.view_t[idx].contiguous(),
                              full.intr[idx].contiguous(), full.W, full.H)

    def _next_views(self):
        Bv, V = self.cfg.batch_views, self.full.n_views
        if self.order.numel() < Bv:
            perm = torch.randperm(V, generator=self._perm_gen, device=self.device)
            self.order = torch.cat([self.order, perm])
        sel, self.order = self.order[:Bv], self.order[Bv:]
        return sel

    def step(self, k: int):
        cfg = self.cfg
        if cfg.stages and self.stage + 1 < len(cfg.stages) and k >= self.stage_starts[self.stage + 1]:
            self._drain_status()
            self._enter_stage(self.stage + 1)
        self._poll(k)
        if self.stage_log:
            self.stage_log[-1]["done"] += 1
        if not hasattr(self, "_idx"):
            self._idx = torch.zeros(cfg.batch_views, dtype=torch.int64, device=self.device)
        self._idx.copy_(self._next_views())
        frac = 1.0 - (1.0 - cfg.final_lr_frac) * min(1.0, k / max(1, cfg.steps - 1))
        for opt, lrs in zip((self.opt_g, self.opt_c), self.base_lr):
            if opt is self.opt_g and self._native:
                continue  # the fused step reads its own rates
            for grp, lr0 in zip(opt.param_groups, lrs):
                if cfg.graph:
                    grp["lr"].fill_(lr0 * frac)
                else:
                    grp["lr"] = lr0 * frac
        if self._native:
            torch.mul(self._nat_lr0, frac, out=self._nat_lr_all)  # all four rates in one kernel
        if self._next_tune is not None and k >= self._next_tune and not self._trial:
            # three steps per candidate; the first one of each may include a graph capture
            self._trial = [ci for ci in range(len(self._cands)) for _ in range(3)]
            self._trial_ev = {ci: [] for ci in range(len(self._cands))}
        ev = None
        if self._trial:
            ci = self._trial.pop(0)
            if ci != self._cur:
                self._use(ci)
            ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            ev[0].record()
        if cfg.graph and self._graph is not None:
            self._graph.replay()
        else:
            self._body()
            if cfg.graph:  # this step ran eagerly (lazy initialisation); record the next ones
                self._capture()
        if ev is not None:
            ev[1].record()
            self._trial_ev[self._cur].append(ev)
            if not self._trial:
                self._finish_tune(k)
        if k >= cfg.warmup:
            self.opt_c.step()
        self._queue_status(k)

    def _capture(self):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self._body()
        self._graph = g
        self._graphs[self._cur] = g

    def _finish_tune(self, k):
        torch.cuda.synchronize()
        ms = {}
        for ci, evs in self._trial_ev.items():
            t = sorted(a.elapsed_time(b) for a, b in evs[1:]) or [float("inf")]
            ms[ci] = t[len(t) // 2]
        best = min(ms, key=ms.get)
        self._use(best)
        name = lambda c: f"{c.tile_w}x{c.tile_h}" + ("+join" if c.split_fwd else "")
        self.tile_log.append(dict(step=k, ms={name(c): round(ms[i], 3) for i, c in enumerate(self._cands)},
                                  tile=name(self._cands[best])))
        self._next_tune = k + self.cfg.tile_tune

    def _body(self):
        """The device work of one step: views of the batch, Gaussian parameters, render forward,
        losses, adjoints, the Gaussian (or field) optimiser step, and the calibration gradients."""
        cfg = self.cfg
        idx = self._idx
        w, f = self.win, self.full
        torch.index_select(f.view_cam, 0, idx, out=w.view_cam)
        torch.index_select(f.view_t, 0, idx, out=w.view_t)
        torch.index_select(f.intr, 0, idx, out=w.intr)
        r0 = int(self.settings.roi_y0)
        torch.index_select(self.targets[:, :, r0:, :], 0, idx, out=self.tgt[:, :, r0:, :])
        native = self._native and not cfg.freeze_gaussians
        with torch.no_grad():
            if self.field is None:
                if not native:  # else the previous step's Adam left them in place
                    o = torch.sigmoid(self.logit_o, out=w.opacity)
                    s = torch.exp(self.log_s, out=w.scale)
            else:
                self._ensure_index()
                B.splat_ngp_fwd_train(self.field_struct, w.mean, w.quat, w.scale, w.opacity, w.color, self.field_ws)
            self.xi_t[:, :3].copy_(self.rho)
            self.xi_t[:, 3:].copy_(self.phi)
            self.dl_t.copy_(self.delta)
            fr = self.fr
            self.loss.zero_()
            if native:  # the Gaussian gradients were cleared by the previous Adam step
                for t in (self.gr.mean, self.gr.w2c, self.gr.xi, self.gr.delta):
                    if t is not None:
                        t.zero_()
            else:
                pl.zero_grads(self.gr)
            # render and the L1 term (over the plan's region of interest) in one launch
            pl.forward(fr, w, self.xi_t, self.dl_t, l1=(self.tgt, None, self.dimg, self.loss, 1.0 - cfg.lam_dssim))
            if cfg.lam_dssim > 0:
                B.splat_dssim_loss_grad(fr.img, self.tgt, self.ssim_ws, self.dimg, self.loss, self.settings.roi_y0,
                                        cfg.lam_dssim)
            pl.backward(fr, w, self.xi_t, self.dl_t, self.dimg, self.gr)
            if cfg.lam_scale > 0:
                B.splat_scale_reg(w.scale, cfg.lam_scale, self.gr.scale, self.loss)
            # gradients of the optimised tensors (written in place)
            if native:
                pass  # the fused step below chains them through the activations itself
            elif self.field is None:
                self.color.grad = self.gr.color
                self.quat.grad = self.gr.quat
                torch.mul(self.gr.opacity, o * (1 - o), out=self.logit_o.grad)
                torch.mul(self.gr.scale, s, out=self.log_s.grad)
            else:
                fg = self.field_grads
                for t in fg.values():
                    t.zero_()
                B.splat_ngp_bwd_saved(self.field_struct, w.n_gauss, self.field_index, self.gr.quat, self.gr.scale,
                                      self.gr.opacity, self.gr.color, self.field_ws, fg["tables"], fg["w1"],
                                      fg["b1"], fg["w2"], fg["b2"], fg["w3"], fg["b3"])
            self.rho.grad.copy_(self.gr.xi[:, :3])
            self.phi.grad.copy_(self.gr.xi[:, 3:])
            self.delta.grad.copy_(self.gr.delta)
        if native:
            gr = self.gr
            raw = (self.color, self.logit_o, self.log_s, self.quat)
            grads = (gr.color, gr.opacity, gr.scale, gr.quat)
            values = (None, w.opacity, w.scale, None)
            acts = (B.ACT_IDENTITY, B.ACT_SIGMOID, B.ACT_EXP, B.ACT_IDENTITY)
            B.splat_adam_step([(p.detach(), m, v, g, val, lr, a) for p, m, v, g, val, lr, a in
                               zip(raw, self._nat_m, self._nat_v, grads, values, self._nat_lr, acts)],
                              self._nat_step)
        elif not cfg.freeze_gaussians:
            self.opt_g.step()

    def _poll(self, k: int):
        """Before step k: read the status word of step k-2, which has finished by now."""
        j = k & 1
        ev, self._st_ev[j] = self._st_ev[j], None
        if ev is not None:
            ev.synchronize()
            if int(self._st_host[j, 0]) & B.ST_CAPACITY:
                self.overflow_steps.append(k - 2)
                self._grow()

    def _queue_status(self, k: int):
        """After step k: copy its status word to pinned memory and clear it."""
        j = k & 1
        st = self.fr.status_t
        self._st_host[j].copy_(st, non_blocking=True)
        st.zero_()
        e = torch.cuda.Event()
        e.record()
        self._st_ev[j] = e

    def _drain_status(self):
        """Read the pending status words (before the plan they belong to is replaced)."""
        for j in (0, 1):
            ev, self._st_ev[j] = self._st_ev[j], None
            if ev is not None:
                ev.synchronize()
                if int(self._st_host[j, 0]) & B.ST_CAPACITY:
                    self.overflow_steps.append(-1)

    def _grow(self):
        """Re-plan the current candidate with twice the capacities after a step whose instances or
        slots overflowed."""
        ns, ni = self.fr.counts()
        G, Bv = self.win.n_gauss, self.cfg.batch_views
        sc, ic = self._caps[self._cur]
        self._caps[self._cur] = (int(min(Bv * G, max(sc, 2 * ns))), int(min((1 << 31) - 1, 2 * max(ic, ni))))
        self._frames.pop(self._cur, None)
        self._graphs.pop(self._cur, None)
        self._use(self._cur)
        self.replans += 1

    def errors(self):
        xi = np.concatenate([self.rho.detach().cpu().numpy(), self.phi.detach().cpu().numpy()], axis=1)
        rot = rotation_error_deg(xi - self.scene.xi_gt)
        trans = np.linalg.norm(xi[:, :3] - self.scene.xi_gt[:, :3], axis=1) * 100.0
        dt = np.abs(self.delta.detach().cpu().numpy() - self.scene.delta_gt) * 1000.0
        return dict(rotation_deg=rot.tolist(), translation_cm=trans.tolist(), time_offset_ms=dt.tolist())

    def run(self, steps=None, log_every=0, log=print):
        steps = self.cfg.steps if steps is None else steps
        t0 = None
        for k in range(steps):
            if k == 10:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
            self.step(k)
            if log_every and (k % log_every == 0 or k == steps - 1):
                e = self.errors()
                log(f"[calib] step {k} loss {float(self.loss.item()):.5f} rot {np.round(e['rotation_deg'], 3)} "
                    f"trans_cm {np.round(e['translation_cm'], 2)} dt_ms {np.round(e['time_offset_ms'], 2)}")
        torch.cuda.synchronize()
        sps = (steps - 10) / (time.perf_counter() - t0) if steps > 10 and t0 else float("nan")
        self._close_stage()
        for k in range(max(0, steps - 2), steps):
            j = k & 1
            if self._st_ev[j] is not None and int(self._st_host[j, 0]) & B.ST_CAPACITY:
                self.overflow_steps.append(k)
            self._st_ev[j] = None
        out = dict(steps=steps, steps_per_s=sps, loss=float(self.loss.item()), replans=self.replans,
                   overflow_steps=len(self.overflow_steps), stages=self.stage_log, tiles=self.tile_log,
                   **self.errors())
        return out
