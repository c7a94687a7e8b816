"""Seeded synthetic inputs for the rasterizer: Gaussian maps, cameras, targets.

This module is the only code shared by the HIP path's tests/bench and the FP64
oracle.  It draws inputs; it computes none of the renderer's arithmetic
(no projection, covariance, colour or blending).  Every generator takes an
explicit ``seed`` and uses ``numpy.random.default_rng``.

Workload shapes follow the paper's datasets, which are not available here:
640x480 keyframes (the TUM-sized images behind the 4.7 MB cost-volume figure,
Sec. III-A1) and 1200x680 (the Replica size implied by the 2.66x resolution
ratio, Sec. IV-B), indoor rooms at 0.5-6 m, and windows of 8-10 keyframes plus
4 past views (Sec. III-B2, Sec. IV-A).  Procedural rooms stand in for Replica
and TUM RGB-D.

Layouts (structure-of-arrays, component-major, float32, C-contiguous):
    means [3][N], log_scales [3][N], quats [4][N] (w, x, y, z),
    opacity_logits [N], sh [3][K][N] with K = (degree + 1)^2.
Cameras: world-to-camera rotation R (row-major 3x3), translation t, pinhole
intrinsics fx, fy, cx, cy (pixel (i, j) has its centre at (i + 0.5, j + 0.5)),
width, height.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Tuple

import numpy as np

# 80-byte camera record shared by the C ABI (gs_camera) and the oracle.
CAMERA_DTYPE = np.dtype([
    ("R", "<f4", (9,)), ("t", "<f4", (3,)),
    ("fx", "<f4"), ("fy", "<f4"), ("cx", "<f4"), ("cy", "<f4"),
    ("width", "<i4"), ("height", "<i4"), ("pad", "<i4", (2,)),
])
assert CAMERA_DTYPE.itemsize == 80


@dataclasses.dataclass
class Camera:
    R: np.ndarray          # (3, 3) world -> camera rotation
    t: np.ndarray          # (3,)   world -> camera translation
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int

    def record(self) -> np.ndarray:
        rec = np.zeros((), dtype=CAMERA_DTYPE)
        rec["R"] = np.asarray(self.R, np.float32).reshape(9)
        rec["t"] = np.asarray(self.t, np.float32).reshape(3)
        rec["fx"], rec["fy"], rec["cx"], rec["cy"] = self.fx, self.fy, self.cx, self.cy
        rec["width"], rec["height"] = self.width, self.height
        return rec

    def as_float32(self) -> "Camera":
        """The camera exactly as the float32 record stores it."""
        return Camera(np.asarray(self.R, np.float32).astype(np.float64),
                      np.asarray(self.t, np.float32).astype(np.float64),
                      float(np.float32(self.fx)), float(np.float32(self.fy)),
                      float(np.float32(self.cx)), float(np.float32(self.cy)),
                      int(self.width), int(self.height))


def camera_records(cams: List[Camera]) -> np.ndarray:
    out = np.zeros(len(cams), dtype=CAMERA_DTYPE)
    for i, c in enumerate(cams):
        out[i] = c.record()
    return out


@dataclasses.dataclass
class GaussianMap:
    means: np.ndarray           # (3, N) float32
    log_scales: np.ndarray      # (3, N) float32
    quats: np.ndarray           # (4, N) float32, (w, x, y, z), not normalised
    opacity_logits: np.ndarray  # (N,) float32
    sh: np.ndarray              # (3, K, N) float32
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means.shape[1])

    def arrays(self):
        return (self.means, self.log_scales, self.quats, self.opacity_logits, self.sh)


@dataclasses.dataclass
class Workload:
    name: str
    gmap: GaussianMap
    cams: List[Camera]
    targets: List[np.ndarray]   # per view (3, H, W) float32
    bg: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    tile_size: int = 16
    seed: int = 0


# ----------------------------------------------------------------------------
# small helpers (input drawing only)
# ----------------------------------------------------------------------------

def _rot_axis_angle(axis: np.ndarray, ang: float) -> np.ndarray:
    axis = np.asarray(axis, np.float64)
    axis = axis / np.linalg.norm(axis)
    x, y, z = axis
    K = np.array([[0, -z, y], [z, 0, -x], [-y, x, 0]], np.float64)
    return np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * (K @ K)


def _quat_from_matrix(R: np.ndarray) -> np.ndarray:
    """(w, x, y, z) of a rotation matrix (Shepperd's method); used to draw
    surface-aligned Gaussian orientations."""
    m = R
    tr = m[0, 0] + m[1, 1] + m[2, 2]
    if tr > 0:
        s = math.sqrt(tr + 1.0) * 2
        w = 0.25 * s
        x = (m[2, 1] - m[1, 2]) / s
        y = (m[0, 2] - m[2, 0]) / s
        z = (m[1, 0] - m[0, 1]) / s
    elif m[0, 0] > m[1, 1] and m[0, 0] > m[2, 2]:
        s = math.sqrt(1.0 + m[0, 0] - m[1, 1] - m[2, 2]) * 2
        w = (m[2, 1] - m[1, 2]) / s
        x = 0.25 * s
        y = (m[0, 1] + m[1, 0]) / s
        z = (m[0, 2] + m[2, 0]) / s
    elif m[1, 1] > m[2, 2]:
        s = math.sqrt(1.0 + m[1, 1] - m[0, 0] - m[2, 2]) * 2
        w = (m[0, 2] - m[2, 0]) / s
        x = (m[0, 1] + m[1, 0]) / s
        y = 0.25 * s
        z = (m[1, 2] + m[2, 1]) / s
    else:
        s = math.sqrt(1.0 + m[2, 2] - m[0, 0] - m[1, 1]) * 2
        w = (m[1, 0] - m[0, 1]) / s
        x = (m[0, 2] + m[2, 0]) / s
        y = (m[1, 2] + m[2, 1]) / s
        z = 0.25 * s
    return np.array([w, x, y, z])


def look_at(eye, target, up=(0.0, 0.0, 1.0)) -> Tuple[np.ndarray, np.ndarray]:
    """World->camera (R, t) for a camera at ``eye`` looking at ``target``;
    camera axes: x right, y down, z forward."""
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    up = np.asarray(up, np.float64)
    r = np.cross(f, up)
    if np.linalg.norm(r) < 1e-9:
        r = np.cross(f, np.array([1.0, 0.0, 0.0]))
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f])       # rows: camera axes in world coordinates
    t = -R @ eye
    return R, t


def pinhole(width: int, height: int, f: float, R=None, t=None) -> Camera:
    R = np.eye(3) if R is None else R
    t = np.zeros(3) if t is None else t
    return Camera(np.asarray(R, np.float64), np.asarray(t, np.float64),
                  float(f), float(f), width / 2.0, height / 2.0, int(width), int(height))


def perturb_pose(cam: Camera, rng, max_deg=5.0, max_m=0.1) -> Camera:
    axis = rng.normal(size=3)
    ang = math.radians(rng.uniform(0, max_deg))
    dR = _rot_axis_angle(axis, ang)
    dt = rng.normal(size=3)
    dt *= rng.uniform(0, max_m) / np.linalg.norm(dt)
    return dataclasses.replace(cam, R=dR @ cam.R, t=dR @ cam.t + dt)


# ----------------------------------------------------------------------------
# random Gaussian clouds (small configs)
# ----------------------------------------------------------------------------

def random_cloud(n: int, sh_degree: int, seed: int, *, box=((-2, 2), (-2, 2), (2, 6)),
                 log_scale_mu=-3.0, log_scale_sigma=0.5, sh_sigma=0.2) -> GaussianMap:
    """Means uniform in ``box``; log-scales N(mu, sigma)^3; quaternions from a
    normalised N(0, I4) draw; opacity logits N(0, 1); SH degree-0 colour
    uniform in [0, 1] (coefficient uniform in [-sqrt(pi), sqrt(pi)], which maps
    to colour U[0,1] through the degree-0 basis 1/(2 sqrt(pi)) and the +0.5
    offset); higher SH bands N(0, sh_sigma)."""
    rng = np.random.default_rng(seed)
    lo = np.array([b[0] for b in box], np.float64)[:, None]
    hi = np.array([b[1] for b in box], np.float64)[:, None]
    means = lo + (hi - lo) * rng.random((3, n))
    log_scales = rng.normal(log_scale_mu, log_scale_sigma, size=(3, n))
    q = rng.normal(size=(4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    ol = rng.normal(0.0, 1.0, size=n)
    K = (sh_degree + 1) ** 2
    sh = np.zeros((3, K, n))
    sh[:, 0, :] = rng.uniform(-math.sqrt(math.pi), math.sqrt(math.pi), size=(3, n))
    if K > 1:
        sh[:, 1:, :] = rng.normal(0.0, sh_sigma, size=(3, K - 1, n))
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return GaussianMap(f32(means), f32(log_scales), f32(q), f32(ol), f32(sh), sh_degree)


def uniform_target(width: int, height: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.random((3, height, width)).astype(np.float32)


# ----------------------------------------------------------------------------
# procedural room (large configs)
# ----------------------------------------------------------------------------

ROOM_X = (-2.5, 2.5)
ROOM_Y = (-2.5, 2.5)
ROOM_Z = (0.0, 3.0)


def _value_noise(points: np.ndarray, seed: int, octaves=3, base_cell=0.8) -> np.ndarray:
    """Seeded 3-octave lattice value noise in [0, 1]^3 (RGB) at world points (M, 3)."""
    rng = np.random.default_rng(seed)
    out = np.zeros((points.shape[0], 3))
    amp_total = 0.0
    for o in range(octaves):
        cell = base_cell / (2 ** o)
        lattice = rng.random((64, 64, 64, 3))
        p = (points - np.array([ROOM_X[0], ROOM_Y[0], ROOM_Z[0]]) + 1.0) / cell
        i0 = np.floor(p).astype(np.int64)
        f = p - i0
        f = f * f * (3 - 2 * f)
        acc = np.zeros((points.shape[0], 3))
        for dx in (0, 1):
            for dy in (0, 1):
                for dz in (0, 1):
                    w = ((f[:, 0] if dx else 1 - f[:, 0]) * (f[:, 1] if dy else 1 - f[:, 1])
                         * (f[:, 2] if dz else 1 - f[:, 2]))
                    idx = (i0 + np.array([dx, dy, dz])) % 64
                    acc += w[:, None] * lattice[idx[:, 0], idx[:, 1], idx[:, 2]]
        amp = 0.5 ** o
        out += amp * acc
        amp_total += amp
    return np.clip(out / amp_total, 0.0, 1.0)


@dataclasses.dataclass
class _Rect:
    origin: np.ndarray   # corner
    u: np.ndarray        # edge vector 1
    v: np.ndarray        # edge vector 2 (normal = u x v / |.|, pointing into free space)

    @property
    def area(self):
        return float(np.linalg.norm(np.cross(self.u, self.v)))

    @property
    def normal(self):
        n = np.cross(self.u, self.v)
        return n / np.linalg.norm(n)


def _room_rects(rng, n_boxes=20):
    x0, x1 = ROOM_X
    y0, y1 = ROOM_Y
    z0, z1 = ROOM_Z
    P = lambda *a: np.array(a, np.float64)
    rects = [
        _Rect(P(x0, y0, z0), P(x1 - x0, 0, 0), P(0, y1 - y0, 0)),          # floor, n=+z
        _Rect(P(x0, y0, z1), P(0, y1 - y0, 0), P(x1 - x0, 0, 0)),          # ceiling, n=-z
        _Rect(P(x0, y0, z0), P(0, y1 - y0, 0), P(0, 0, z1 - z0)),          # wall x0, n=+x
        _Rect(P(x1, y0, z0), P(0, 0, z1 - z0), P(0, y1 - y0, 0)),          # wall x1, n=-x
        _Rect(P(x0, y0, z0), P(0, 0, z1 - z0), P(x1 - x0, 0, 0)),          # wall y0, n=+y
        _Rect(P(x0, y1, z0), P(x1 - x0, 0, 0), P(0, 0, z1 - z0)),          # wall y1, n=-y
    ]
    boxes = []
    for _ in range(n_boxes):
        ex, ey, ez = rng.uniform(0.2, 1.0, size=3)
        cx = rng.uniform(x0 + 0.6, x1 - 0.6)
        cy = rng.uniform(y0 + 0.6, y1 - 0.6)
        yaw = rng.uniform(0, 2 * math.pi)
        Rz = _rot_axis_angle([0, 0, 1], yaw)
        a, b = Rz[:, 0] * ex, Rz[:, 1] * ey
        c = np.array([0, 0, ez])
        o = np.array([cx, cy, 0.0]) - 0.5 * a - 0.5 * b
        boxes.append((o, a, b, c))
        # five visible faces (bottom rests on the floor), outward normals
        rects += [
            _Rect(o + c, a, b),                 # top, n=+z
            _Rect(o, c, a),                     # side a-c at b=0, normal -b
            _Rect(o + b, a, c),                 # side at b=1, normal +b
            _Rect(o, b, c),                     # side at a=0, normal -a
            _Rect(o + a, c, b),                 # side at a=1, normal +a
        ]
    return rects, boxes


def _morton2(s: np.ndarray) -> np.ndarray:
    """Z-order code of points in [0, 1)^2 (16 bits per axis)."""
    q = np.clip((s * 65536.0).astype(np.int64), 0, 65535)

    def spread(x):
        x = (x | (x << 8)) & 0x00FF00FF
        x = (x | (x << 4)) & 0x0F0F0F0F
        x = (x | (x << 2)) & 0x33333333
        return (x | (x << 1)) & 0x55555555

    return spread(q[:, 0]) | (spread(q[:, 1]) << 1)


def procedural_room(n: int, seed: int, sh_degree: int = 3, n_boxes: int = 20):
    """A 5 x 5 x 3 m room (6 planes) plus ``n_boxes`` boxes (edges U[0.2, 1] m,
    resting on the floor, random yaw).  Gaussians are placed area-uniformly on
    the surfaces with N(0, 0.01 m) jitter along the normal, oriented with the
    third axis on the normal, scales (a, a, 0.1 a) with a = sqrt(area / n),
    opacity logits N(2, 0.5), degree-0 colour from seeded value noise and
    higher SH bands N(0, 0.05).  Index order is surface by surface and, on a
    surface, a Z-order curve over its two coordinates: a map built from
    keyframes inserts the Gaussians of one image region together, so nearby
    indices are nearby in space (drawing them in random order instead would
    make every run of indices span the whole surface).
    Returns (GaussianMap, boxes)."""
    rng = np.random.default_rng(seed)
    rects, boxes = _room_rects(rng, n_boxes)
    areas = np.array([r.area for r in rects])
    total = areas.sum()
    counts = rng.multinomial(n, areas / total)
    means = np.zeros((n, 3))
    quats = np.zeros((n, 4))
    k = 0
    for r, c in zip(rects, counts):
        if c == 0:
            continue
        s = rng.random((c, 2))
        s = s[np.argsort(_morton2(s), kind="stable")]   # insertion order: see above
        pts = r.origin + s[:, :1] * r.u + s[:, 1:] * r.v
        nrm = r.normal
        pts = pts + rng.normal(0.0, 0.01, size=(c, 1)) * nrm
        e1 = r.u / np.linalg.norm(r.u)
        e2 = np.cross(nrm, e1)
        spin = rng.uniform(0, 2 * math.pi, size=c)
        for j in range(c):
            cs, sn = math.cos(spin[j]), math.sin(spin[j])
            a1 = cs * e1 + sn * e2
            a2 = np.cross(nrm, a1)
            Rm = np.stack([a1, a2, nrm], axis=1)
            quats[k + j] = _quat_from_matrix(Rm)
        means[k:k + c] = pts
        k += c
    a = math.sqrt(total / n)
    log_scales = np.tile(np.log(np.array([a, a, 0.1 * a]))[:, None], (1, n))
    ol = rng.normal(2.0, 0.5, size=n)
    K = (sh_degree + 1) ** 2
    sh = np.zeros((3, K, n))
    rgb = _value_noise(means, seed + 7919)
    # degree-0 coefficient whose colour (through 1/(2 sqrt(pi)) and +0.5) is rgb
    sh[:, 0, :] = ((rgb - 0.5) * 2.0 * math.sqrt(math.pi)).T
    if K > 1:
        sh[:, 1:, :] = rng.normal(0.0, 0.05, size=(3, K - 1, n))
    f32 = lambda x: np.ascontiguousarray(x, dtype=np.float32)
    gmap = GaussianMap(f32(means.T), f32(log_scales), f32(quats.T), f32(ol), f32(sh), sh_degree)
    return gmap, boxes


def _clearance(p: np.ndarray, boxes) -> float:
    d = min(p[0] - ROOM_X[0], ROOM_X[1] - p[0], p[1] - ROOM_Y[0], ROOM_Y[1] - p[1],
            p[2] - ROOM_Z[0], ROOM_Z[1] - p[2])
    for (o, a, b, c) in boxes:
        # distance to an oriented box (local coordinates along a, b, c)
        M = np.stack([a / np.linalg.norm(a), b / np.linalg.norm(b), c / np.linalg.norm(c)])
        half = np.array([np.linalg.norm(a), np.linalg.norm(b), np.linalg.norm(c)]) / 2
        centre = o + (a + b + c) / 2
        q = np.abs(M @ (p - centre)) - half
        outside = np.linalg.norm(np.maximum(q, 0.0))
        inside = min(max(q[0], q[1], q[2]), 0.0)
        d = min(d, outside + inside)
    return d


def room_trajectory(n_views: int, seed: int, boxes, *, step_m=0.1, step_deg=5.0,
                    min_clear=0.5):
    """Smooth camera path: a Catmull-Rom spline through seeded waypoints with
    >= ``min_clear`` m clearance, resampled so consecutive positions differ by
    <= ``step_m``; yaw/pitch random-walk with steps <= ``step_deg``.
    Returns a list of (R, t) world->camera."""
    rng = np.random.default_rng(seed)

    def free_point():
        for _ in range(10000):
            p = np.array([rng.uniform(*ROOM_X), rng.uniform(*ROOM_Y), rng.uniform(1.0, 2.2)])
            if _clearance(p, boxes) >= min_clear + 0.05:
                return p
        raise RuntimeError("no free waypoint")

    way = [free_point() for _ in range(6)]
    pts = []
    for i in range(len(way) - 1):
        p0 = way[max(i - 1, 0)]
        p1, p2 = way[i], way[i + 1]
        p3 = way[min(i + 2, len(way) - 1)]
        for s in np.linspace(0, 1, 200, endpoint=False):
            s2, s3 = s * s, s * s * s
            p = 0.5 * ((2 * p1) + (-p0 + p2) * s + (2 * p0 - 5 * p1 + 4 * p2 - p3) * s2
                       + (-p0 + 3 * p1 - 3 * p2 + p3) * s3)
            pts.append(p)
    # arc-length resampling at step <= step_m, keeping only clear points
    poses = []
    yaw = rng.uniform(0, 2 * math.pi)
    pitch = 0.0
    last = None
    for p in pts:
        if last is not None and np.linalg.norm(p - last) < step_m * 0.9:
            continue
        if _clearance(p, boxes) < min_clear:
            continue
        yaw += math.radians(rng.uniform(-step_deg, step_deg)) * 0.7
        pitch = float(np.clip(pitch + math.radians(rng.uniform(-step_deg, step_deg)) * 0.5,
                              -0.4, 0.2))
        fwd = np.array([math.cos(yaw) * math.cos(pitch), math.sin(yaw) * math.cos(pitch),
                        math.sin(pitch)])
        poses.append(look_at(p, p + fwd))
        last = p
        if len(poses) == n_views:
            break
    if len(poses) < n_views:
        raise RuntimeError("trajectory too short")
    return poses


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------

def config_c1(seed: int = 0) -> Workload:
    """Plain fwd+bwd, 1 view 160x120: 2,000 Gaussians, fx=fy=150, cx=80, cy=60."""
    g = random_cloud(2000, 0, seed)
    cam = Camera(np.eye(3), np.zeros(3), 150.0, 150.0, 80.0, 60.0, 160, 120)
    return Workload("c1_plain_160x120_2k", g, [cam], [uniform_target(160, 120, seed + 1)], seed=seed)


def config_c2(seed: int = 0, n: int = 50000) -> Workload:
    """Gradient check, 320x240: 50,000 Gaussians, SH degree 3 coefficients
    N(0, 0.2), a seeded small camera perturbation (<= 5 deg, <= 0.1 m)."""
    g = random_cloud(n, 3, seed)
    rng = np.random.default_rng(seed + 2)
    cam = perturb_pose(Camera(np.eye(3), np.zeros(3), 300.0, 300.0, 160.0, 120.0, 320, 240), rng)
    return Workload("c2_gradcheck_320x240_50k", g, [cam], [uniform_target(320, 240, seed + 1)], seed=seed)


def room_views(n_gauss: int, sizes: List[Tuple[int, int]], seed: int, name: str) -> Workload:
    gmap, boxes = procedural_room(n_gauss, seed)
    poses = room_trajectory(len(sizes), seed + 11, boxes)
    cams = []
    targets = []
    for i, ((W, H), (R, t)) in enumerate(zip(sizes, poses)):
        f = 525.0 * W / 640.0
        cams.append(Camera(R, t, f, f, W / 2.0, H / 2.0, W, H))
        targets.append(_smooth_target(W, H, seed + 100 + i))
    return Workload(name, gmap, cams, targets, seed=seed)


def _smooth_target(W: int, H: int, seed: int) -> np.ndarray:
    """A low-frequency colour field in [0, 1] (stand-in for a keyframe)."""
    rng = np.random.default_rng(seed)
    coarse = rng.random((3, H // 32 + 2, W // 32 + 2))
    ys = np.linspace(0, coarse.shape[1] - 1.001, H)
    xs = np.linspace(0, coarse.shape[2] - 1.001, W)
    y0 = ys.astype(int)
    x0 = xs.astype(int)
    fy = (ys - y0)[None, :, None]
    fx = (xs - x0)[None, None, :]
    c00 = coarse[:, y0][:, :, x0]
    c01 = coarse[:, y0][:, :, x0 + 1]
    c10 = coarse[:, y0 + 1][:, :, x0]
    c11 = coarse[:, y0 + 1][:, :, x0 + 1]
    img = (1 - fy) * ((1 - fx) * c00 + fx * c01) + fy * ((1 - fx) * c10 + fx * c11)
    return np.ascontiguousarray(img, dtype=np.float32)


def config_c3(seed: int = 0, n: int = 200000) -> Workload:
    """Single-view mapping step, 640x480, fx=fy=525, 200,000-Gaussian room, SH 3."""
    return room_views(n, [(640, 480)], seed, "c3_mapping_640x480_200k")


def config_metric(seed: int = 0, n: int = 200000, n_views: int = 32) -> Workload:
    """Headline workload: the 200,000-Gaussian room, V views at 640x480 on a
    smooth trajectory."""
    return room_views(n, [(640, 480)] * n_views, seed, f"room_{n_views}x640x480_200k")


C4_SIZES = [(320, 240), (640, 480), (960, 540), (1200, 680)]


def config_c4(seed: int = 0, n: int = 500000, n_views: int = 32) -> Workload:
    """Batched replay: 500,000-Gaussian room, 32 keyframes cycling through
    320x240, 640x480, 960x540, 1200x680 (8 of each)."""
    sizes = [C4_SIZES[i % 4] for i in range(n_views)]
    return room_views(n, sizes, seed, f"room_{n_views}_uneven_500k")


# ----------------------------------------------------------------------------
# synthetic projected splats (stage-wise inputs for binning and compositing)
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class SplatSet:
    """2D splats for one or more views, arrays shaped [V][N] (float32/int32)."""
    xy: np.ndarray             # (V, N, 2)
    conic_opacity: np.ndarray  # (V, N, 4): Q00, Q01, Q11, opacity
    rgb_depth: np.ndarray      # (V, N, 4): r, g, b, depth
    radius: np.ndarray         # (V, N) int32, 0 = culled
    cams: List[Camera]


def random_splats(n: int, cams: List[Camera], seed: int, *, sigma_px=(0.6, 24.0),
                  cull_frac=0.05, depth_ties=0.0) -> SplatSet:
    """Random screen-space splats: centres uniform over the image plus a
    margin, inverse covariances Q drawn as R diag(1/s1^2, 1/s2^2) R^T with
    s log-uniform in ``sigma_px``, opacity U[0.02, 1], colour U[0, 1], depth
    U[0.5, 6] (a fraction ``depth_ties`` drawn from a handful of repeated
    values to exercise tie-breaking), radius drawn as ceil(3 * max(s)) and a
    fraction ``cull_frac`` marked culled (radius 0)."""
    rng = np.random.default_rng(seed)
    V = len(cams)
    xy = np.zeros((V, n, 2), np.float32)
    co = np.zeros((V, n, 4), np.float32)
    rd = np.zeros((V, n, 4), np.float32)
    rad = np.zeros((V, n), np.int32)
    for v, c in enumerate(cams):
        m = 40.0
        xy[v, :, 0] = rng.uniform(-m, c.width + m, n)
        xy[v, :, 1] = rng.uniform(-m, c.height + m, n)
        s = np.exp(rng.uniform(math.log(sigma_px[0]), math.log(sigma_px[1]), size=(n, 2)))
        th = rng.uniform(0, math.pi, n)
        cs, sn = np.cos(th), np.sin(th)
        i1, i2 = 1.0 / s[:, 0] ** 2, 1.0 / s[:, 1] ** 2
        co[v, :, 0] = cs * cs * i1 + sn * sn * i2
        co[v, :, 1] = cs * sn * (i1 - i2)
        co[v, :, 2] = sn * sn * i1 + cs * cs * i2
        co[v, :, 3] = rng.uniform(0.02, 1.0, n)
        rd[v, :, :3] = rng.random((n, 3))
        depth = rng.uniform(0.5, 6.0, n)
        if depth_ties > 0:
            k = int(depth_ties * n)
            depth[:k] = rng.choice(np.array([1.0, 2.5, 3.0, 4.25]), size=k)
            rng.shuffle(depth)
        rd[v, :, 3] = depth
        rad[v] = np.ceil(3.0 * s.max(axis=1)).astype(np.int32)
        rad[v, rng.random(n) < cull_frac] = 0
    return SplatSet(xy, co, rd, rad, cams)
