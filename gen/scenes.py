"""Seeded synthetic point clouds standing in for the paper's ICP and normal
estimation workloads (Section 4: consecutive VGA depth frames aligned with
point-to-plane ICP, and per-frame normal estimation).

The paper's recordings are not available, so each scene below reproduces the
*shape* of a workload: point count, spatial layout, density variation and
noise model.  Every function takes a ``numpy.random.Generator`` and is fully
deterministic given it.  Only geometry used to *draw* inputs lives here
(ray casting, a rotation built from axis and angle); nothing of the
registration method itself.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_SALT = 1807_00399


def rng_for(config: int, pair: int = 0) -> np.random.Generator:
    """Generator for workload ``config``, pair ``pair``."""
    return np.random.Generator(np.random.PCG64([int(config), int(pair), SEED_SALT]))


# ----------------------------------------------------------------------------
# rigid transforms used to make target clouds
# ----------------------------------------------------------------------------

def random_rigid(rng: np.random.Generator, angle_deg: float, t_norm: float) -> np.ndarray:
    """4x4 float64 rigid transform: rotation by ``angle_deg`` about a uniformly
    random axis, translation of length ``t_norm`` in a uniformly random
    direction."""
    axis = rng.standard_normal(3)
    axis /= np.linalg.norm(axis)
    th = math.radians(angle_deg)
    kx = np.array([[0.0, -axis[2], axis[1]],
                   [axis[2], 0.0, -axis[0]],
                   [-axis[1], axis[0], 0.0]])
    rot = np.eye(3) + math.sin(th) * kx + (1.0 - math.cos(th)) * (kx @ kx)
    t = rng.standard_normal(3)
    t = t_norm * t / np.linalg.norm(t)
    out = np.eye(4)
    out[:3, :3] = rot
    out[:3, 3] = t
    return out


def apply_rigid(T: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """Map float32 points through ``T`` in float64 and round once to float32."""
    p = pts.astype(np.float64)
    return (p @ T[:3, :3].T + T[:3, 3]).astype(np.float32)


# ----------------------------------------------------------------------------
# scenes
# ----------------------------------------------------------------------------

def sphere_plane(rng: np.random.Generator, n: int = 10_000, sigma: float = 0.002) -> np.ndarray:
    """Unit sphere at the origin plus the square [-1,1]^2 in the plane z=-1.

    Points are split between the two surfaces in proportion to their areas
    (4*pi and 4); each coordinate gets N(0, sigma^2) noise.  Returned in a
    random order, float32 (n, 3).
    """
    n_sph = int(n * (4.0 * math.pi) / (4.0 * math.pi + 4.0))
    n_pln = n - n_sph
    g = rng.standard_normal((n_sph, 3))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    xy = rng.uniform(-1.0, 1.0, size=(n_pln, 2))
    pl = np.column_stack([xy, np.full(n_pln, -1.0)])
    pts = np.vstack([g, pl])
    pts += rng.normal(0.0, sigma, size=pts.shape)
    pts = pts[rng.permutation(n)]
    return pts.astype(np.float32)


def _slab_hits(d: np.ndarray, lo: np.ndarray, hi: np.ndarray, origin=None) -> np.ndarray:
    """Ray parameter of the first hit of rays from ``origin`` (default the
    coordinate origin) with direction ``d`` (m, 3) on the axis-aligned box
    [lo, hi]; +inf where missed."""
    o = np.zeros(3) if origin is None else np.asarray(origin, np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        t1 = (lo[None, :] - o[None, :]) / d
        t2 = (hi[None, :] - o[None, :]) / d
    tn = np.max(np.minimum(t1, t2), axis=1)
    tf = np.min(np.maximum(t1, t2), axis=1)
    hit = (tn <= tf) & (tn > 0.0)
    return np.where(hit, tn, np.inf)


def room_scan(rng: np.random.Generator, width: int = 640, height: int = 480,
              n_boxes: int = 20, depth_noise: float = 0.003, pixels: np.ndarray | None = None) -> np.ndarray:
    """Depth-camera frame of a room with boxes, back-projected to 3-D.

    Room [-3,3]x[-1.5,1.5]x[-0.5,5.5] in camera coordinates (x right, y down,
    z forward) with ``n_boxes`` axis-aligned boxes (sides U(0.2,1) m) standing
    on the floor y=1.5, centres x~U(-2.5,2.5), z~U(1,5).  A pinhole camera at
    the origin (fx=fy=525, cx=319.5, cy=239.5 at 640x480, scaled for other
    sizes) casts one ray per pixel; depth gets N(0, (depth_noise*z^2)^2)
    noise.  Every ray hits, so the result has exactly width*height points,
    float32, pixel raster order.  With ``pixels`` (raster indices), only those
    pixels are cast, in the given order.
    """
    s = width / 640.0
    fx = fy = 525.0 * s
    cx, cy = (width - 1) / 2.0, (height - 1) / 2.0
    if pixels is None:
        pixels = np.arange(width * height)
    pixels = np.asarray(pixels, dtype=np.int64)
    u, v = (pixels % width).astype(np.float64), (pixels // width).astype(np.float64)
    d = np.column_stack([(u - cx) / fx, (v - cy) / fy, np.ones(len(pixels))])
    room_lo = np.array([-3.0, -1.5, -0.5])
    room_hi = np.array([3.0, 1.5, 5.5])
    with np.errstate(divide="ignore"):
        t_exit = np.min(np.where(d > 0, room_hi / d, np.where(d < 0, room_lo / d, np.inf)), axis=1)
    t = t_exit
    for _ in range(n_boxes):
        side = rng.uniform(0.2, 1.0, size=3)
        cxz = np.array([rng.uniform(-2.5, 2.5), rng.uniform(1.0, 5.0)])
        lo = np.array([cxz[0] - side[0] / 2, 1.5 - side[1], cxz[1] - side[2] / 2])
        hi = np.array([cxz[0] + side[0] / 2, 1.5, cxz[1] + side[2] / 2])
        t = np.minimum(t, _slab_hits(d, lo, hi))
    assert np.all(np.isfinite(t))
    z = t  # d.z == 1, so the ray parameter is the depth
    z = z + rng.standard_normal(z.shape) * (depth_noise * z * z)
    return (d * z[:, None]).astype(np.float32)


def room_views(rng: np.random.Generator, width: int = 640, height: int = 480, angle_deg: float = 3.0,
               t_norm: float = 0.03, n_boxes: int = 20, depth_noise: float = 0.003):
    """Two depth frames of one room (the room of ``room_scan``) from two
    cameras: camera 1 at the origin, camera 2 at the pose C = random_rigid
    (angle_deg, t_norm) of camera 1's frame.  Returns (source, target, C,
    intrinsics): source = frame 2 back-projected in camera 2's frame,
    target = frame 1 in camera 1's frame, both (height*width, 3) float32 in
    pixel raster order (an organized image; every ray hits); C maps source
    to target coordinates; intrinsics = (fx, fy, cx, cy) of both cameras.
    Depth noise N(0, (depth_noise z^2)^2) is drawn per frame."""
    s = width / 640.0
    fx = fy = 525.0 * s
    cx, cy = (width - 1) / 2.0, (height - 1) / 2.0
    pix = np.arange(width * height)
    u, v = (pix % width).astype(np.float64), (pix // width).astype(np.float64)
    d = np.column_stack([(u - cx) / fx, (v - cy) / fy, np.ones(len(pix))])
    room_lo = np.array([-3.0, -1.5, -0.5])
    room_hi = np.array([3.0, 1.5, 5.5])
    boxes = []
    for _ in range(n_boxes):
        side = rng.uniform(0.2, 1.0, size=3)
        cxz = np.array([rng.uniform(-2.5, 2.5), rng.uniform(1.0, 5.0)])
        boxes.append((np.array([cxz[0] - side[0] / 2, 1.5 - side[1], cxz[1] - side[2] / 2]),
                      np.array([cxz[0] + side[0] / 2, 1.5, cxz[1] + side[2] / 2])))
    C = random_rigid(rng, angle_deg, t_norm)

    def render(R, o):
        dw = d @ R.T                       # ray directions in the room frame
        with np.errstate(divide="ignore"):
            t = np.min(np.where(dw > 0, (room_hi - o) / dw, np.where(dw < 0, (room_lo - o) / dw, np.inf)), axis=1)
        for lo, hi in boxes:
            t = np.minimum(t, _slab_hits(dw, lo, hi, o))
        assert np.all(np.isfinite(t))
        z = t + rng.standard_normal(t.shape) * (depth_noise * t * t)   # d.z == 1: t is the depth
        return (d * z[:, None]).astype(np.float32)

    target = render(np.eye(3), np.zeros(3))
    source = render(C[:3, :3], C[:3, 3])
    return source, target, C, (fx, fy, cx, cy)


def street_scan(rng: np.random.Generator, n_beams: int = 64, n_az: int = 32768,
                n_boxes: int = 30, n_cyl: int = 40, range_noise: float = 0.01) -> np.ndarray:
    """Spinning-LiDAR scan of a street canyon, float32 (n_beams*n_az, 3).

    Sensor at the origin, z up, ground at z=-1.8.  Beams at elevations evenly
    spread over [-25, +3] degrees, ``n_az`` azimuths over 360 degrees.
    Facades at y=+U(8,15) and y=-U(8,15), end walls at x=+-75, all 20 m tall;
    ``n_boxes`` boxes (sides U(1,10) m) and ``n_cyl`` vertical cylinders
    (radius U(0.1,0.5), height U(3,8)) stand on the ground with their nearest
    point U(3,60) m from the sensor.  Every ray hits within [1, 80] m; range
    gets N(0, range_noise^2) noise along the ray.  Points are beam-major.
    """
    z0 = -1.8
    elev = np.deg2rad(np.linspace(-25.0, 3.0, n_beams))
    az = np.arange(n_az, dtype=np.float64) * (2.0 * math.pi / n_az)
    ce, se = np.cos(elev)[:, None], np.sin(elev)[:, None]
    d = np.stack([(ce * np.cos(az)[None, :]).ravel(),
                  (ce * np.sin(az)[None, :]).ravel(),
                  np.broadcast_to(se, (n_beams, n_az)).ravel()], axis=1)
    y_left, y_right = rng.uniform(8.0, 15.0), rng.uniform(8.0, 15.0)
    with np.errstate(divide="ignore"):
        t_ground = np.where(d[:, 2] < 0, z0 / d[:, 2], np.inf)
        t_fac = np.where(d[:, 1] > 0, y_left / d[:, 1], np.where(d[:, 1] < 0, -y_right / d[:, 1], np.inf))
        t_end = np.where(d[:, 0] > 0, 75.0 / d[:, 0], np.where(d[:, 0] < 0, -75.0 / d[:, 0], np.inf))
    t = np.minimum(t_ground, np.minimum(t_fac, t_end))
    for _ in range(n_boxes):
        side = rng.uniform(1.0, 10.0, size=3)
        phi = rng.uniform(0.0, 2.0 * math.pi)
        dist = rng.uniform(3.0, 60.0) + 0.5 * math.hypot(side[0], side[1])
        c = np.array([dist * math.cos(phi), dist * math.sin(phi)])
        lo = np.array([c[0] - side[0] / 2, c[1] - side[1] / 2, z0])
        hi = np.array([c[0] + side[0] / 2, c[1] + side[1] / 2, z0 + side[2]])
        t = np.minimum(t, _slab_hits(d, lo, hi))
    for _ in range(n_cyl):
        r = rng.uniform(0.1, 0.5)
        h = rng.uniform(3.0, 8.0)
        phi = rng.uniform(0.0, 2.0 * math.pi)
        dist = rng.uniform(3.0, 60.0) + r
        cx, cy = dist * math.cos(phi), dist * math.sin(phi)
        a = d[:, 0] ** 2 + d[:, 1] ** 2
        b = -2.0 * (d[:, 0] * cx + d[:, 1] * cy)
        c0 = cx * cx + cy * cy - r * r
        disc = b * b - 4.0 * a * c0
        ok = (disc >= 0) & (a > 0)
        with np.errstate(invalid="ignore", divide="ignore"):
            tc = (-b - np.sqrt(np.where(ok, disc, 0.0))) / (2.0 * a)
        zc = tc * d[:, 2]
        ok &= (tc > 0) & (zc >= z0) & (zc <= z0 + h)
        t = np.minimum(t, np.where(ok, tc, np.inf))
    assert np.all(np.isfinite(t)) and np.all(t * d[:, 2] <= z0 + 20.0 + 1e-9)
    t = t + rng.standard_normal(t.shape) * range_noise
    assert np.all((t >= 1.0) & (t <= 80.0))
    return (d * t[:, None]).astype(np.float32)


def lattice_cloud(n_side: int, spacing: float = 1.0, offset=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Integer lattice n_side^3 (exactly representable, full of exact ties)."""
    g = np.arange(n_side, dtype=np.float64) * spacing
    x, y, z = np.meshgrid(g, g, g, indexing="ij")
    pts = np.column_stack([x.ravel(), y.ravel(), z.ravel()]) + np.asarray(offset)
    return pts.astype(np.float32)


def uniform_cloud(rng: np.random.Generator, n: int, lo=-1.0, hi=1.0) -> np.ndarray:
    return rng.uniform(lo, hi, size=(n, 3)).astype(np.float32)


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    source: np.ndarray          # (N, 3) float32, the cloud that is moved
    target: np.ndarray          # (N, 3) float32, target = T_gt * source
    T_gt: np.ndarray            # (4, 4) float64, maps source onto target
    k: int                      # neighbours for normals
    d_max: float                # correspondence rejection distance
    iters: int                  # fixed ICP iteration count
    viewpoint: tuple = (0.0, 0.0, 0.0)

    @property
    def n(self) -> int:
        return int(self.source.shape[0])


CONFIGS = {
    0: dict(name="sphere_plane_10k", k=10, d_max=0.1, iters=20, angle=10.0, t=0.05),
    1: dict(name="room_vga_307200", k=16, d_max=0.05, iters=30, angle=15.0, t=0.1),
    2: dict(name="street_lidar_2097152", k=16, d_max=1.0, iters=40, angle=5.0, t=0.5),
}


@dataclasses.dataclass
class BatchWorkload:
    """Many independent pairs of uneven sizes, packed back to back."""
    name: str
    pairs: list                 # list of Workload

    @property
    def n_pairs(self) -> int:
        return len(self.pairs)

    def _pack(self, attr):
        return np.ascontiguousarray(np.vstack([getattr(w, attr) for w in self.pairs]).astype(np.float32))

    @property
    def source(self) -> np.ndarray:
        return self._pack("source")

    @property
    def target(self) -> np.ndarray:
        return self._pack("target")

    @property
    def offsets(self) -> np.ndarray:
        """(n_pairs + 1) int64 offsets, shared by sources and targets."""
        return np.concatenate([[0], np.cumsum([w.n for w in self.pairs])]).astype(np.int64)

    @property
    def n(self) -> int:
        return int(sum(w.n for w in self.pairs))

    def param(self, attr) -> np.ndarray:
        return np.array([getattr(w, attr) for w in self.pairs])


# parent configurations of the batched workload: sphere + plane, room
BATCH_PARENTS = {0: dict(k=10, d_max=0.1, iters=20, t=0.05), 1: dict(k=16, d_max=0.05, iters=30, t=0.1)}
BATCH_CONFIG = dict(name="uneven_pairs", n_pairs=256, n_lo=5_000, n_hi=200_000, angle=(5.0, 20.0),
                    small_n_pairs=12, small_n_lo=300, small_n_hi=3_000)


def batch_workload(config: int = 3, size: str = "full", n_pairs: int | None = None) -> BatchWorkload:
    """Workload 3: uneven pairs.  Pair j (generator rng_for(3, j)) is either a
    sphere + plane cloud or a new random room scan, each with probability
    1/2; its size is round(exp U(ln n_lo, ln n_hi)) points (rooms: that many
    of the frame's pixels, drawn without replacement, kept in raster order);
    target = T * source with a rotation angle U(5, 20) degrees and the
    parent's translation length; k, d_max and the iteration count come from
    the parent.  ``size="small"`` uses 12 pairs of 300-3000 points (rooms at
    160x120) for tests the oracle finishes quickly."""
    if config != 3:
        raise ValueError(f"unknown batched workload {config}")
    c = BATCH_CONFIG
    full = size == "full"
    m = n_pairs if n_pairs is not None else (c["n_pairs"] if full else c["small_n_pairs"])
    lo, hi = (c["n_lo"], c["n_hi"]) if full else (c["small_n_lo"], c["small_n_hi"])
    width, height = (640, 480) if full else (160, 120)
    pairs = []
    for j in range(m):
        rng = rng_for(config, j)
        kind = 0 if rng.random() < 0.5 else 1
        n = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        if kind == 0:
            src = sphere_plane(rng, n)
        else:
            n = min(n, width * height)
            pix = np.sort(rng.choice(width * height, size=n, replace=False))
            src = room_scan(rng, width, height, pixels=pix)
        par = BATCH_PARENTS[kind]
        T = random_rigid(rng, rng.uniform(*c["angle"]), par["t"])
        tgt = apply_rigid(T, src)
        pairs.append(Workload(f"{c['name']}_{j}_{'sphere' if kind == 0 else 'room'}", src, tgt, T, par["k"],
                              par["d_max"], par["iters"]))
    name = f"{c['name']}_{m}" + ("" if full else "_small")
    return BatchWorkload(name, pairs)


# learned-initialiser workload: evaluation pairs come from config 4,
# training pairs from config 40 (disjoint generator streams)
POSE_CONFIG = dict(name="pose_pairs", n_pairs=512, n_points=4096, angle=(0.0, 90.0), t=(0.0, 0.3), k=10,
                   d_max=0.3, iters=30, accept_rms=0.004, eval_config=4, train_config=40)


def pose_pairs(config: int = 4, n_pairs: int | None = None, n_points: int | None = None,
               first: int = 0) -> BatchWorkload:
    """Pairs for the learned initialiser.  Pair j (generator rng_for(config,
    first + j)) is a sphere + plane cloud or a new random room scan, each
    with probability 1/2, of n_points points (rooms: that many of a 640x480
    frame's pixels, drawn without replacement, kept in raster order); the
    target is T * source exactly (the same points), with a rotation angle
    U(0, 90) degrees about a random axis and a translation of length
    U(0, 0.3)."""
    c = POSE_CONFIG
    m = c["n_pairs"] if n_pairs is None else n_pairs
    n = c["n_points"] if n_points is None else n_points
    pairs = []
    for j in range(first, first + m):
        rng = rng_for(config, j)
        kind = 0 if rng.random() < 0.5 else 1
        if kind == 0:
            src = sphere_plane(rng, n)
        else:
            pix = np.sort(rng.choice(640 * 480, size=min(n, 640 * 480), replace=False))
            src = room_scan(rng, 640, 480, pixels=pix)
        T = random_rigid(rng, rng.uniform(*c["angle"]), rng.uniform(*c["t"]))
        pairs.append(Workload(f"{c['name']}_{j}_{'sphere' if kind == 0 else 'room'}", src, apply_rigid(T, src), T,
                              c["k"], c["d_max"], c["iters"]))
    return BatchWorkload(f"{c['name']}_{m}", pairs)


# layer shapes of the learned initialiser's flat parameter vector (W[in][out], then b)
POSE_NET_SHAPES = ((3, 64), (64,), (64, 128), (128,), (128, 256), (256,), (512, 256), (256,), (256, 4), (4,))


def pose_net_init(rng: np.random.Generator) -> np.ndarray:
    """Initial parameters: weights N(0, 2 / fan_in), biases 0 except the last
    (1, 0, 0, 0), the identity quaternion.  float32, flat."""
    out = []
    for shp in POSE_NET_SHAPES:
        if len(shp) == 2:
            out.append(rng.standard_normal(shp[0] * shp[1]) * math.sqrt(2.0 / shp[0]))
        else:
            out.append(np.zeros(shp[0]))
    out[-1][0] = 1.0
    return np.concatenate(out).astype(np.float32)


def make_workload(config: int, pair: int = 0, size: str = "full") -> Workload:
    """Build workload ``config`` (0, 1 or 2).

    ``size="small"`` shrinks the scan resolution of configs 1 and 2 (160x120
    pixels; 16 beams x 2048 azimuths) for tests the oracle finishes quickly;
    the scene geometry and parameters are unchanged.
    """
    p = CONFIGS[config]
    rng = rng_for(config, pair)
    if config == 0:
        src = sphere_plane(rng, 10_000 if size == "full" else 2_000)
    elif config == 1:
        src = room_scan(rng) if size == "full" else room_scan(rng, 160, 120)
    elif config == 2:
        src = street_scan(rng) if size == "full" else street_scan(rng, 16, 2048)
    else:
        raise ValueError(f"unknown workload {config}")
    T = random_rigid(rng, p["angle"], p["t"])
    tgt = apply_rigid(T, src)
    name = p["name"] if size == "full" else p["name"] + "_small"
    return Workload(name, src, tgt, T, p["k"], p["d_max"], p["iters"])
