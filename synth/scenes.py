"""Seeded synthetic driving scenes standing in for KITTI-360 sequences.

The paper evaluates on KITTI-360 (front pinhole cameras, a 64-beam 360 degree
LiDAR, accumulated and voxel-downsampled clouds of 0.25-4.2 M points, 40 frames
per sensor; Sec. IV-A, Tables II and V).  That data is not available here, so
these generators draw scenes of the same shape: a ground plane plus random boxes
scanned by a simulated 64-ring LiDAR, scans accumulated along a drive, Gaussians
anchored at the returns (Sec. III-B), a smooth colour field, pinhole cameras of
KITTI-like size and a LiDAR trajectory sampled at 10 Hz.  No dataset item is
reproduced.  Everything is drawn from ``numpy.random.default_rng(seed)``.

Nothing in here renders, projects or differentiates: it only produces inputs.

Conventions shared with both implementations:
  * Gaussians are SoA planes: mean[3,G], quat[4,G] (w,x,y,z, not normalised),
    scale[3,G] (> 0), opacity[G] in (0,1), color[3,G]; float32.
  * Trajectory knots: t[K] seconds, q[K,4] (w,x,y,z) LiDAR->world rotation,
    p[K,3] LiDAR origin in world; float64.
  * Rig: per camera R0[C,3,3], t0[C,3] = camera->LiDAR prior, intr[C,4] =
    (fx, fy, cx, cy); one image size W x H for all cameras.
  * Calibration state: xi[C,6] = (rho, phi) correction of the prior, delta[C]
    time offset in seconds.
  * Views: cam[V] int32 camera index, t[V] float64 camera timestamp.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Gaussians", "Trajectory", "Rig", "Views", "Scene",
    "tiny_scene", "tiny_target", "kitti_single", "calib16", "batched64",
    "calib_full", "small_drive", "drive_scans", "random_rigid", "perturbation",
    "quat_from_euler", "anisotropic", "WORKLOADS",
]

# workload name of every generator
WORKLOADS = {
    "tiny_scene": "tiny_2k_256x64",
    "kitti_single": "kitti_single_500k_1408x376",
    "calib16": "calib_2cam_8frame_500k_1408x376",
    "batched64": "batched_uneven_64v_2M_1408x376",
    "calib_full": "calib_loop_2cam_100frame_2M_1408x376",
    "drive_scans": "lidar_accumulated_40scan",
}


# ----------------------------------------------------------------------------
# containers
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Gaussians:
    mean: np.ndarray      # [3,G] f32
    quat: np.ndarray      # [4,G] f32
    scale: np.ndarray     # [3,G] f32
    opacity: np.ndarray   # [G]   f32
    color: np.ndarray     # [3,G] f32

    @property
    def n(self) -> int:
        return int(self.opacity.shape[0])

    def copy(self) -> "Gaussians":
        return Gaussians(*(np.array(a, copy=True) for a in dataclasses.astuple(self)))

    def subset(self, idx) -> "Gaussians":
        return Gaussians(self.mean[:, idx].copy(), self.quat[:, idx].copy(),
                         self.scale[:, idx].copy(), self.opacity[idx].copy(),
                         self.color[:, idx].copy())


@dataclasses.dataclass
class Trajectory:
    t: np.ndarray   # [K] f64
    q: np.ndarray   # [K,4] f64
    p: np.ndarray   # [K,3] f64


@dataclasses.dataclass
class Rig:
    R0: np.ndarray    # [C,3,3] f64
    t0: np.ndarray    # [C,3] f64
    intr: np.ndarray  # [C,4] f64
    W: int
    H: int

    @property
    def n(self) -> int:
        return int(self.R0.shape[0])


@dataclasses.dataclass
class Views:
    cam: np.ndarray   # [V] i32
    t: np.ndarray     # [V] f64

    @property
    def n(self) -> int:
        return int(self.cam.shape[0])


@dataclasses.dataclass
class Scene:
    name: str
    gauss: Gaussians
    traj: Trajectory
    rig: Rig
    views: Views
    xi: np.ndarray       # [C,6] f64  calibration state to evaluate at
    delta: np.ndarray    # [C]   f64
    xi_gt: np.ndarray    # [C,6] f64  ground truth (zeros: the prior is exact)
    delta_gt: np.ndarray  # [C]  f64
    info: dict = dataclasses.field(default_factory=dict)


# ----------------------------------------------------------------------------
# small rotation helpers used only to *build* inputs
# ----------------------------------------------------------------------------
def _rot_z(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def _rot_y(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


def _rot_x(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[1.0, 0.0, 0.0], [0.0, c, -s], [0.0, s, c]])


def _mat_to_quat(R):
    """Rotation matrix -> unit quaternion (w,x,y,z) with w >= 0 (Shepperd)."""
    tr = R[0, 0] + R[1, 1] + R[2, 2]
    if tr > 0:
        s = math.sqrt(tr + 1.0) * 2
        q = [0.25 * s, (R[2, 1] - R[1, 2]) / s, (R[0, 2] - R[2, 0]) / s, (R[1, 0] - R[0, 1]) / s]
    elif R[0, 0] > R[1, 1] and R[0, 0] > R[2, 2]:
        s = math.sqrt(1.0 + R[0, 0] - R[1, 1] - R[2, 2]) * 2
        q = [(R[2, 1] - R[1, 2]) / s, 0.25 * s, (R[0, 1] + R[1, 0]) / s, (R[0, 2] + R[2, 0]) / s]
    elif R[1, 1] > R[2, 2]:
        s = math.sqrt(1.0 + R[1, 1] - R[0, 0] - R[2, 2]) * 2
        q = [(R[0, 2] - R[2, 0]) / s, (R[0, 1] + R[1, 0]) / s, 0.25 * s, (R[1, 2] + R[2, 1]) / s]
    else:
        s = math.sqrt(1.0 + R[2, 2] - R[0, 0] - R[1, 1]) * 2
        q = [(R[1, 0] - R[0, 1]) / s, (R[0, 2] + R[2, 0]) / s, (R[1, 2] + R[2, 1]) / s, 0.25 * s]
    q = np.array(q)
    q /= np.linalg.norm(q)
    return q if q[0] >= 0 else -q


def _quat_to_mat(q):
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def quat_from_euler(yaw, pitch=0.0, roll=0.0):
    """R = Rz(yaw) Ry(pitch) Rx(roll) as a (w,x,y,z) quaternion."""
    return _mat_to_quat(_rot_z(yaw) @ _rot_y(pitch) @ _rot_x(roll))


def perturbation(rng, deg, metres):
    """Per-axis perturbation of +-deg and +-metres with seeded signs.

    The paper perturbs "all 3 axes, either positive or negative" (Sec. IV-B);
    the rotation is applied as Rz Ry Rx.  Returns (R_pert[3,3], t_pert[3]).
    """
    sr = rng.choice([-1.0, 1.0], size=3)
    st = rng.choice([-1.0, 1.0], size=3)
    a = math.radians(deg) * sr
    return _rot_z(a[2]) @ _rot_y(a[1]) @ _rot_x(a[0]), metres * st


def random_rigid(rng, max_angle=math.pi, max_t=10.0):
    """A random rigid transform (R, t) used for invariance tests."""
    axis = rng.normal(size=3)
    axis /= np.linalg.norm(axis)
    ang = rng.uniform(-max_angle, max_angle)
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    R = np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * K @ K
    return R, rng.uniform(-max_t, max_t, size=3)


# ----------------------------------------------------------------------------
# tiny scene: 2,000 Gaussians, one 256x64 camera
# ----------------------------------------------------------------------------
def tiny_scene(seed=0, n=2000, W=256, H=64, f=200.0):
    """2,000 Gaussians in front of an identity camera (camera = LiDAR = world).

    Means x in U[-8,8], y in U[-2,2], z in U[2,20]; per-axis scale
    exp(N(ln 0.1, 0.5)); random unit quaternion; opacity sigmoid(N(0,1));
    colour U[0,1]^3.
    """
    rng = np.random.default_rng(seed)
    mean = np.stack([rng.uniform(-8, 8, n), rng.uniform(-2, 2, n), rng.uniform(2, 20, n)])
    scale = np.exp(rng.normal(math.log(0.1), 0.5, size=(3, n)))
    q = rng.normal(size=(4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    opac = 1.0 / (1.0 + np.exp(-rng.normal(size=n)))
    color = rng.uniform(0, 1, size=(3, n))
    g = Gaussians(mean.astype(np.float32), q.astype(np.float32), scale.astype(np.float32),
                  opac.astype(np.float32), color.astype(np.float32))
    traj = Trajectory(np.array([0.0, 1.0]), np.array([[1.0, 0, 0, 0], [1.0, 0, 0, 0]]),
                      np.zeros((2, 3)))
    rig = Rig(np.eye(3)[None].copy(), np.zeros((1, 3)),
              np.array([[f, f, W / 2.0, H / 2.0]]), W, H)
    views = Views(np.zeros(1, np.int32), np.array([0.5]))
    z6 = np.zeros((1, 6))
    return Scene("tiny", g, traj, rig, views, z6.copy(), np.zeros(1), z6.copy(), np.zeros(1))


def tiny_target(scene: Scene, seed=1) -> Gaussians:
    """Perturbed copy of the tiny scene's Gaussians (means stay fixed).

    colour + N(0,0.1), logit(o) + N(0,0.5), ln s + N(0,0.2), q + N(0,0.1).
    """
    rng = np.random.default_rng(seed)
    g = scene.gauss.copy()
    n = g.n
    g.color = (g.color + rng.normal(0, 0.1, size=(3, n))).astype(np.float32)
    o = g.opacity.astype(np.float64)
    lo = np.log(o / (1 - o)) + rng.normal(0, 0.5, size=n)
    g.opacity = (1 / (1 + np.exp(-lo))).astype(np.float32)
    g.scale = np.exp(np.log(g.scale.astype(np.float64)) + rng.normal(0, 0.2, size=(3, n))).astype(np.float32)
    q = g.quat.astype(np.float64) + rng.normal(0, 0.1, size=(4, n))
    g.quat = (q / np.linalg.norm(q, axis=0, keepdims=True)).astype(np.float32)
    return g


# ----------------------------------------------------------------------------
# LiDAR world simulation
# ----------------------------------------------------------------------------
LIDAR_HEIGHT = 1.73
RING_ELEV_DEG = (-25.0, 3.0)
N_RINGS = 64
AZ_STEP_DEG = 0.2
MAX_RANGE = 80.0


def _ray_dirs_lidar(n_rings=N_RINGS, az_step=AZ_STEP_DEG):
    el = np.radians(np.linspace(RING_ELEV_DEG[0], RING_ELEV_DEG[1], n_rings))
    az = np.radians(np.arange(0.0, 360.0, az_step))
    E, A = np.meshgrid(el, az, indexing="ij")
    d = np.stack([np.cos(E) * np.cos(A), np.cos(E) * np.sin(A), np.sin(E)], axis=-1)
    return d.reshape(-1, 3)


def _cast(origin, R, boxes, dirs_l, max_range=MAX_RANGE):
    """Cast one LiDAR scan against the ground plane z=0 and yawed boxes."""
    d = dirs_l @ R.T
    n = d.shape[0]
    tbest = np.full(n, np.inf)
    down = d[:, 2] < -1e-9
    tbest[down] = -origin[2] / d[down, 2]
    az = np.arctan2(d[:, 1], d[:, 0])
    order = np.argsort(az)
    az_sorted = az[order]
    for (cx, cy, yaw, hl, hw, h) in boxes:
        vx, vy = cx - origin[0], cy - origin[1]
        dist = math.hypot(vx, vy)
        rb = math.hypot(hl, hw)
        if dist - rb > max_range:
            continue
        if dist <= rb * 1.05:
            idx = np.arange(n)
        else:
            bearing = math.atan2(vy, vx)
            ha = math.asin(min(1.0, rb / dist)) + math.radians(1.0)
            lo, hi = bearing - ha, bearing + ha
            parts = []
            for a, b in ((lo, hi), (lo + 2 * math.pi, hi + 2 * math.pi), (lo - 2 * math.pi, hi - 2 * math.pi)):
                i0, i1 = np.searchsorted(az_sorted, [a, b])
                if i1 > i0:
                    parts.append(order[i0:i1])
            if not parts:
                continue
            idx = np.concatenate(parts)
        c, s = math.cos(-yaw), math.sin(-yaw)
        ox = c * vx * -1 - s * vy * -1  # origin relative to box centre, in box frame
        oy = s * vx * -1 + c * vy * -1
        oz = origin[2]
        dd = d[idx]
        dx = c * dd[:, 0] - s * dd[:, 1]
        dy = s * dd[:, 0] + c * dd[:, 1]
        dz = dd[:, 2]
        with np.errstate(divide="ignore", invalid="ignore"):
            t1x, t2x = (-hl - ox) / dx, (hl - ox) / dx
            t1y, t2y = (-hw - oy) / dy, (hw - oy) / dy
            t1z, t2z = (0.0 - oz) / dz, (h - oz) / dz
        tmin = np.maximum(np.maximum(np.minimum(t1x, t2x), np.minimum(t1y, t2y)), np.minimum(t1z, t2z))
        tmax = np.minimum(np.minimum(np.maximum(t1x, t2x), np.maximum(t1y, t2y)), np.maximum(t1z, t2z))
        hit = (tmax >= tmin) & (tmin > 0.05)
        th = np.where(hit, tmin, np.inf)
        tbest[idx] = np.minimum(tbest[idx], th)
    ok = tbest < max_range
    return origin[None, :] + tbest[ok, None] * d[ok]


def _place_boxes(rng, n, path_fn, s_lo, s_hi, weight_fn=None, corridor=4.0, lateral=28.0):
    """Boxes outside a +-corridor road around a path; density from weight_fn(s)."""
    boxes = []
    tries = 0
    while len(boxes) < n and tries < 100 * n:
        tries += 1
        s = rng.uniform(s_lo, s_hi)
        if weight_fn is not None and rng.uniform() > weight_fn(s):
            continue
        hl = rng.uniform(1.5, 5.0) / 2
        hw = rng.uniform(1.0, 2.5) / 2
        h = rng.uniform(1.0, 4.0)
        rb = math.hypot(hl, hw)
        side = rng.choice([-1.0, 1.0])
        off = side * rng.uniform(corridor + rb, lateral)
        (px, py), heading = path_fn(s)
        cx = px - math.sin(heading) * off
        cy = py + math.cos(heading) * off
        boxes.append((cx, cy, rng.uniform(0, 2 * math.pi), hl, hw, h))
    return boxes


def _color_field(rng, pts, n_waves=8):
    """Smooth random RGB: sigmoid of a sum of random 3-D sinusoids per channel."""
    out = np.zeros((3, pts.shape[0]))
    for ch in range(3):
        acc = np.zeros(pts.shape[0])
        for _ in range(n_waves):
            direc = rng.normal(size=3)
            direc /= np.linalg.norm(direc)
            k = rng.uniform(0.1, 1.0)
            acc += rng.normal(0, 1.0) * np.sin(pts @ (k * direc) + rng.uniform(0, 2 * math.pi))
        out[ch] = 1.0 / (1.0 + np.exp(-acc))
    return out


def _knn_half_spacing(pts, k=3):
    from scipy.spatial import cKDTree
    tree = cKDTree(pts)
    dist, _ = tree.query(pts, k=k + 1, workers=-1)
    return 0.5 * dist[:, 1:].mean(axis=1)


def _gaussians_from_points(rng, pts, opacity=0.8, min_scale=0.005, max_scale=0.5):
    n = pts.shape[0]
    s = np.clip(_knn_half_spacing(pts), min_scale, max_scale)
    quat = np.zeros((4, n), np.float32)
    quat[0] = 1.0
    return Gaussians(pts.T.astype(np.float32).copy(), quat,
                     np.repeat(s[None], 3, axis=0).astype(np.float32),
                     np.full(n, opacity, np.float32),
                     _color_field(rng, pts).astype(np.float32))


def _voxel_first(pts, voxel):
    keys = np.floor(pts / voxel).astype(np.int64)
    keys -= keys.min(axis=0)
    span = keys.max(axis=0) + 1
    lin = (keys[:, 0] * span[1] + keys[:, 1]) * span[2] + keys[:, 2]
    _, idx = np.unique(lin, return_index=True)
    return pts[np.sort(idx)]


def _kitti_rig(n_cams=1, W=1408, H=376, f=552.0, cx=None, cy=None):
    """Front pinhole camera(s): cam (x right, y down, z fwd) -> LiDAR (x fwd, y left, z up)."""
    cx = W / 2.0 if cx is None else cx
    cy = H / 2.0 if cy is None else cy
    Rc = np.array([[0.0, 0.0, 1.0], [-1.0, 0.0, 0.0], [0.0, -1.0, 0.0]])
    offs = [np.array([0.8, 0.3, -0.3]), np.array([0.8, 0.3 - 0.54, -0.3])]
    R0 = np.stack([Rc] * n_cams)
    t0 = np.stack(offs[:n_cams])
    intr = np.tile(np.array([[f, f, cx, cy]]), (n_cams, 1))
    return Rig(R0, t0, intr, W, H)


# ----------------------------------------------------------------------------
# straight / arc worlds for configs 1 and 2
# ----------------------------------------------------------------------------
def _kitti_world(seed, n_points, n_boxes=200, scan_step=1.0, n_rings=N_RINGS, az_step=AZ_STEP_DEG):
    rng = np.random.default_rng(seed)

    def straight(s):
        return (s, 0.0), 0.0

    boxes = _place_boxes(rng, n_boxes, straight, -30.0, 90.0)
    dirs = _ray_dirs_lidar(n_rings, az_step)
    clouds, total, k = [], 0, 0
    while total < n_points:
        origin = np.array([k * scan_step, 0.0, LIDAR_HEIGHT])
        pts = _cast(origin, np.eye(3), boxes, dirs)
        clouds.append(pts)
        total += pts.shape[0]
        k += 1
    pts = np.concatenate(clouds)
    sel = np.sort(rng.choice(pts.shape[0], size=n_points, replace=False))
    pts = pts[sel]
    return rng, pts, boxes, k


def kitti_single(seed=0, n_points=500_000, W=1408, H=376, f=552.0):
    """One KITTI-like view: 1408x376 pinhole, 500k LiDAR-anchored Gaussians.

    64 rings at elevations linspace(-25,+3) deg, 0.2 deg azimuth steps, 80 m
    range, LiDAR 1.73 m above a ground plane with 200 boxes outside a +-4 m
    road; scans every 1 m along +x until >= n_points returns, then a seeded
    subsample to exactly n_points.  Isotropic scale = half the mean distance to
    the 3 nearest neighbours, opacity 0.8, colour from a smooth random field.
    """
    rng, pts, boxes, n_scans = _kitti_world(seed, n_points)
    g = _gaussians_from_points(rng, pts)
    traj = Trajectory(np.array([0.0, 1.0]),
                      np.array([[1.0, 0, 0, 0], [1.0, 0, 0, 0]]),
                      np.array([[0.0, 0.0, LIDAR_HEIGHT], [10.0, 0.0, LIDAR_HEIGHT]]))
    rig = _kitti_rig(1, W, H, f)
    views = Views(np.zeros(1, np.int32), np.array([0.0]))
    z = np.zeros((1, 6))
    return Scene("kitti_single", g, traj, rig, views, z.copy(), np.zeros(1), z.copy(), np.zeros(1),
                 info={"n_scans": n_scans, "n_boxes": len(boxes)})


def anisotropic(scene: Scene, seed=7, jitter=0.3) -> Scene:
    """The same scene with anisotropic, randomly rotated Gaussians: every scale axis
    multiplied by exp(N(0, jitter)) and every quaternion replaced by a random unit
    quaternion (normalised N(0, I4) draw).  Means, opacities and colours are kept."""
    rng = np.random.default_rng(seed)
    g = scene.gauss.copy()
    g.scale = (g.scale.astype(np.float64) * np.exp(rng.normal(0.0, jitter, g.scale.shape))).astype(np.float32)
    q = rng.normal(size=(4, g.n))
    g.quat = (q / np.linalg.norm(q, axis=0, keepdims=True)).astype(np.float32)
    return dataclasses.replace(scene, name=scene.name + "_aniso", gauss=g)


def _arc_trajectory(n_knots, dt=0.1, speed=10.0, radius=50.0, t0=0.0, wobble_deg=1.0):
    """Ego on a circular arc at constant speed, sampled at 1/dt Hz, with a small
    pitch/roll wobble so that the interpolated rotations are not single-axis."""
    ts = t0 + dt * np.arange(n_knots)
    qs, ps = [], []
    for t in ts:
        yaw = speed * t / radius
        p = np.array([radius * math.sin(yaw), radius * (1 - math.cos(yaw)), LIDAR_HEIGHT])
        pitch = math.radians(wobble_deg) * math.sin(2.1 * t)
        roll = math.radians(wobble_deg) * math.cos(1.7 * t)
        qs.append(quat_from_euler(yaw, pitch, roll))
        ps.append(p)
    return Trajectory(ts, np.array(qs), np.array(ps))


def _perturbed_state(rng, n_cams, deg, metres, delta):
    """Calibration state xi=(rho,phi) giving an R/t error of +-deg/+-metres per axis."""
    xi = np.zeros((n_cams, 6))
    for c in range(n_cams):
        Rp, tp = perturbation(rng, deg, metres)
        # rotation vector of Rp (log map) for the phi part
        cos_a = max(-1.0, min(1.0, (np.trace(Rp) - 1) / 2))
        a = math.acos(cos_a)
        w = np.array([Rp[2, 1] - Rp[1, 2], Rp[0, 2] - Rp[2, 0], Rp[1, 0] - Rp[0, 1]])
        phi = w * (a / (2 * math.sin(a))) if a > 1e-12 else 0.5 * w
        xi[c, :3] = tp
        xi[c, 3:] = phi
    return xi, np.full(n_cams, float(delta))


def calib16(seed=0, n_points=500_000, W=1408, H=376, f=552.0, deg=5.0, metres=0.3, delta=0.05):
    """Two cameras x 8 frames on a 10 m/s, R=50 m arc with 10 Hz LiDAR poses.

    Frames sit at LiDAR knot times so that t + delta (delta = 50 ms) falls mid
    segment.  Targets are meant to be rendered at the ground truth (xi = 0,
    delta = 0); the evaluation state is perturbed by +-deg / +-metres per axis.
    """
    rng, pts, boxes, n_scans = _kitti_world(seed, n_points)
    g = _gaussians_from_points(rng, pts)
    traj = _arc_trajectory(12)
    rig = _kitti_rig(2, W, H, f)
    ft = traj.t[1:9].copy()
    views = Views(np.repeat(np.arange(2, dtype=np.int32), 8), np.tile(ft, 2))
    xi, dl = _perturbed_state(rng, 2, deg, metres, delta)
    return Scene("calib16", g, traj, rig, views, xi, dl, np.zeros((2, 6)), np.zeros(2),
                 info={"n_scans": n_scans})


def small_drive(seed=0, n_points=3000, W=96, H=40, f=40.0, n_cams=2, n_frames=2,
                deg=5.0, metres=0.3, delta=0.05, n_boxes=30, n_rings=16, az_step=1.0):
    """The two-camera calibration problem (arc drive, 10 Hz poses, perturbed extrinsic and
    time offset) at a size small enough for CPU finite differences."""
    rng = np.random.default_rng(seed)

    def arc(s):
        yaw = s / 50.0
        return (50 * math.sin(yaw), 50 * (1 - math.cos(yaw))), yaw

    boxes = _place_boxes(rng, n_boxes, arc, -5.0, 40.0, corridor=3.0, lateral=12.0)
    dirs = _ray_dirs_lidar(n_rings, az_step)
    traj = _arc_trajectory(8)
    clouds = []
    for k in range(0, 8, 2):
        R = _quat_to_mat(traj.q[k])
        clouds.append(_cast(traj.p[k], R, boxes, dirs, max_range=30.0))
    pts = np.concatenate(clouds)
    sel = np.sort(rng.choice(pts.shape[0], size=min(n_points, pts.shape[0]), replace=False))
    pts = pts[sel]
    g = _gaussians_from_points(rng, pts)
    # make the Gaussians anisotropic and varied so every parameter has a gradient
    n = g.n
    g.scale = (g.scale * np.exp(rng.normal(0, 0.3, size=(3, n)))).astype(np.float32)
    q = rng.normal(size=(4, n))
    g.quat = (q / np.linalg.norm(q, axis=0, keepdims=True)).astype(np.float32)
    g.opacity = (1 / (1 + np.exp(-rng.normal(0.5, 1.0, size=n)))).astype(np.float32)
    rig = _kitti_rig(n_cams, W, H, f)
    ft = traj.t[1:1 + n_frames].copy()
    views = Views(np.repeat(np.arange(n_cams, dtype=np.int32), n_frames), np.tile(ft, n_cams))
    xi, dl = _perturbed_state(rng, n_cams, deg, metres, delta)
    return Scene("small_drive", g, traj, rig, views, xi, dl, np.zeros((n_cams, 6)), np.zeros(n_cams))


# ----------------------------------------------------------------------------
# 300 m drive for configs 3 and 4
# ----------------------------------------------------------------------------
# City route: straight streets joined by 90 degree turns of radius 15 m,
# (kind, length or signed angle) in order; about 300 m in total.
_ROUTE = (("S", 45.0), ("A", math.pi / 2), ("S", 40.0), ("A", math.pi / 2), ("S", 45.0),
          ("A", -math.pi / 2), ("S", 40.0), ("A", -math.pi / 2), ("S", 30.0))
_TURN_R = 15.0


def _drive_path(route=_ROUTE, radius=_TURN_R):
    """Position and heading at arc length s along the route (extended straight past both ends)."""
    segs = []
    x, y, h, s0 = 0.0, 0.0, 0.0, 0.0
    for kind, val in route:
        L = val if kind == "S" else abs(val) * radius
        segs.append((kind, val, s0, L, x, y, h))
        if kind == "S":
            x, y = x + L * math.cos(h), y + L * math.sin(h)
        else:
            sg = 1.0 if val > 0 else -1.0
            cx, cy = x - sg * radius * math.sin(h), y + sg * radius * math.cos(h)
            h = h + val
            x, y = cx + sg * radius * math.sin(h), cy - sg * radius * math.cos(h)
        s0 += L
    end = (x, y, h, s0)

    def pos(s):
        if s < 0:
            _, _, _, _, x0, y0, h0 = segs[0]
            return (x0 + s * math.cos(h0), y0 + s * math.sin(h0)), h0
        for kind, val, sb, L, x0, y0, h0 in segs:
            if s <= sb + L:
                u = s - sb
                if kind == "S":
                    return (x0 + u * math.cos(h0), y0 + u * math.sin(h0)), h0
                sg = 1.0 if val > 0 else -1.0
                cx, cy = x0 - sg * radius * math.sin(h0), y0 + sg * radius * math.cos(h0)
                hh = h0 + sg * u / radius
                return (cx + sg * radius * math.sin(hh), cy - sg * radius * math.cos(hh)), hh
        xe, ye, he, se = end
        return (xe + (s - se) * math.cos(he), ye + (s - se) * math.sin(he)), he

    pos.length = s0
    return pos


def _drive_trajectory(n_knots=301, dt=0.1, speed=10.0, wobble_deg=0.8):
    pos = _drive_path()
    ts = dt * np.arange(n_knots)
    qs, ps = [], []
    for t in ts:
        (x, y), yaw = pos(speed * t)
        pitch = math.radians(wobble_deg) * math.sin(1.3 * t)
        roll = math.radians(wobble_deg) * math.cos(0.9 * t)
        qs.append(quat_from_euler(yaw, pitch, roll))
        ps.append(np.array([x, y, LIDAR_HEIGHT]))
    return Trajectory(ts, np.array(qs), np.array(ps))


def _density(s):
    """Relative box / point density along the route (uniform; the view-to-view
    spread of visible counts comes from the turns and the route ends)."""
    return 1.0


def _drive_boxes(rng, n_boxes):
    """Boxes along the route, off every street; also the road samples and their tree."""
    from scipy.spatial import cKDTree
    pos = _drive_path()
    # road centre line samples: boxes must stay off every street of the route
    s_samp = np.arange(-40.0, 341.0, 1.0)
    road = np.array([pos(s)[0] for s in s_samp])
    road_tree = cKDTree(road)
    cand = _place_boxes(rng, 3 * n_boxes, pos, -40.0, 340.0, weight_fn=_density, lateral=30.0)
    boxes = []
    for b in cand:
        rb = math.hypot(b[3], b[4])
        if road_tree.query([b[0], b[1]])[0] > 4.0 + rb:
            boxes.append(b)
        if len(boxes) == n_boxes:
            break
    return boxes, s_samp, road_tree


def drive_scans(seed=0, n_scans=40, n_boxes=700, t0=0.0, t1=None):
    """The accumulated LiDAR cloud of a drive before any downsampling: n_scans
    64-ring scans spread evenly over [t0, t1] seconds of the 30 s route (the paper
    accumulates the scans of its 40-frame sequences, Sec. IV-A), world frame,
    float32 [3, n], scans in time order.  About 0.1 M returns per scan.  The world
    (boxes) is that of the drive scenes with the same seed."""
    rng = np.random.default_rng(seed)
    traj = _drive_trajectory()
    boxes, _, _ = _drive_boxes(rng, n_boxes)
    dirs = _ray_dirs_lidar()
    t1 = traj.t[-1] if t1 is None else t1
    ks = np.unique(np.searchsorted(traj.t, np.linspace(t0, t1, n_scans) - 1e-9).clip(0, len(traj.t) - 1))
    clouds = [_cast(traj.p[k], _quat_to_mat(traj.q[k]), boxes, dirs) for k in ks]
    return np.ascontiguousarray(np.concatenate(clouds).T.astype(np.float32))


def _drive_world(seed, n_points, scan_every=5.0, voxel=0.05, n_boxes=700):
    rng = np.random.default_rng(seed)
    traj = _drive_trajectory()
    boxes, s_samp, road_tree = _drive_boxes(rng, n_boxes)
    dirs = _ray_dirs_lidar()
    clouds = []
    step = int(round(scan_every / (10.0 * 0.1)))
    for k in range(0, len(traj.t), step):
        R = _quat_to_mat(traj.q[k])
        clouds.append(_cast(traj.p[k], R, boxes, dirs))
    pts = _voxel_first(np.concatenate(clouds), voxel)
    # density weight from the arc length of the nearest road sample
    _, near = road_tree.query(pts[:, :2], workers=-1)
    w = np.array([_density(s) for s in s_samp])[near] ** 2 + 0.02
    if pts.shape[0] < n_points:
        raise RuntimeError(f"drive world has only {pts.shape[0]} points < {n_points}")
    sel = np.sort(rng.choice(pts.shape[0], size=n_points, replace=False, p=w / w.sum()))
    return rng, pts[sel], traj, len(boxes), len(clouds)


def batched64(seed=0, n_points=2_000_000, W=1408, H=376, f=552.0, n_frames=32):
    """64 views (2 cameras x 32 frames) of a 300 m drive anchored at 2 M Gaussians.

    Scans every 5 m along a zig-zag city route of four 90 degree turns (301
    LiDAR poses at 10 Hz), 5 cm voxel downsampling, then a seeded subsample to
    exactly n_points.  The turns and the route ends make the visible count vary
    strongly from view to view (about 1.1e5 to 1.4e6 at seed 0).
    """
    rng, pts, traj, nb, ns = _drive_world(seed, n_points)
    g = _gaussians_from_points(rng, pts)
    rig = _kitti_rig(2, W, H, f)
    ft = np.linspace(0.55, 28.55, n_frames)
    views = Views(np.repeat(np.arange(2, dtype=np.int32), n_frames), np.tile(ft, 2))
    z = np.zeros((2, 6))
    return Scene("batched64", g, traj, rig, views, z.copy(), np.zeros(2), z.copy(), np.zeros(2),
                 info={"n_boxes": nb, "n_scans": ns})


def calib_full(seed=0, n_points=2_000_000, W=1408, H=376, f=552.0, n_frames=100,
               deg=10.0, metres=0.5, delta=0.1, t_start=5.0):
    """Calibration loop: 2 cameras x 100 frames (10 s) in the 2 M-point drive world.

    The evaluation (initial) state is perturbed by +-10 deg / +-0.5 m per axis and
    delta = 100 ms; the ground truth is xi = 0, delta = 0.
    """
    rng, pts, traj, nb, ns = _drive_world(seed, n_points)
    g = _gaussians_from_points(rng, pts)
    rig = _kitti_rig(2, W, H, f)
    ft = t_start + 0.05 + 0.1 * np.arange(n_frames)
    views = Views(np.repeat(np.arange(2, dtype=np.int32), n_frames), np.tile(ft, 2))
    xi, dl = _perturbed_state(rng, 2, deg, metres, delta)
    return Scene("calib_full", g, traj, rig, views, xi, dl, np.zeros((2, 6)), np.zeros(2),
                 info={"n_boxes": nb, "n_scans": ns})
