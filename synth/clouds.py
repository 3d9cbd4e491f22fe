"""Seeded synthetic point clouds.

Workloads (all FP32 xyz, AoS ``[n][3]``):

* ``blobs_cloud``  -- Gaussian blobs plus planar noise, in shuffled index
  order, standing in for the paper's synthetic clusters whose point indices
  are randomised (Sec. 3.3, "Setting").
* ``lidar_frame``  -- one simulated 64-beam spinning-LiDAR scan of a seeded
  scene (ground plane, boxes, vertical cylinders), standing in for a single
  KITTI scan (Sec. 3.4, Table 4).  KITTI itself is not available here.
* ``lidar_map``    -- many such frames registered along a random-walk
  trajectory, standing in for a whole KITTI sequence accumulated into one
  unorganized cloud (Fig. 1 caption, Table 2).

Everything is computed in float64 and cast to float32 at the end.  Random
streams come from ``numpy.random.default_rng`` seeded through
``SeedSequence`` so that each map frame has its own independent stream and a
prefix of the map (its first ``k`` frames) is bit-identical to the first
``k`` frames of the full map.

Nothing here measures distances between points: this module only produces
inputs.
"""

from __future__ import annotations

import hashlib
import math
import os
import tempfile
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

_GOLDEN = (1.0 + math.sqrt(5.0)) / 2.0


# --------------------------------------------------------------------------
# sensor model and ray casting
# --------------------------------------------------------------------------

@dataclass(frozen=True)
class SensorModel:
    """Spinning multi-beam range sensor.

    Beams are evenly spaced in elevation; one revolution sweeps ``n_cols``
    azimuth columns.  Successive revolutions are offset in azimuth by the
    fractional part of ``k * golden_ratio`` of one step so that repeated
    revolutions do not retrace the same rays.
    """

    height: float = 1.8
    n_beams: int = 64
    el_min_deg: float = -25.0
    el_max_deg: float = 3.0
    az_step_deg: float = 0.2
    r_min: float = 0.5
    r_max: float = 80.0
    range_sigma: float = 0.02
    drop_prob: float = 0.05

    @property
    def n_cols(self) -> int:
        return int(round(360.0 / self.az_step_deg))


@dataclass
class Scene:
    """Axis-aligned boxes resting on z=0 and vertical cylinders on z=0.

    ``boxes``: (k, 6) float64 rows ``xmin, ymin, zmin, xmax, ymax, zmax``.
    ``cyls``:  (k, 4) float64 rows ``cx, cy, radius, height``.
    The ground is the plane z = 0.
    """

    boxes: np.ndarray = field(default_factory=lambda: np.zeros((0, 6)))
    cyls: np.ndarray = field(default_factory=lambda: np.zeros((0, 4)))


def _make_objects(rng, n_boxes, n_cyls, place):
    """Boxes (sides U[1,5] m) and cylinders (r U[0.1,0.5] m, h U[2,8] m).

    Sizes are drawn first; ``place(rb)`` then returns one (k, 2) array of
    ground-plane centres for objects whose footprint bounding radii are rb.
    """
    sides = rng.uniform(1.0, 5.0, size=(n_boxes, 3))
    rad = rng.uniform(0.1, 0.5, size=n_cyls)
    hgt = rng.uniform(2.0, 8.0, size=n_cyls)
    rb_box = 0.5 * np.hypot(sides[:, 0], sides[:, 1])
    box_xy = place(rb_box)
    cyl_xy = place(rad)
    keep_b = np.isfinite(box_xy[:, 0])
    keep_c = np.isfinite(cyl_xy[:, 0])
    sides, box_xy = sides[keep_b], box_xy[keep_b]
    rad, hgt, cyl_xy = rad[keep_c], hgt[keep_c], cyl_xy[keep_c]
    boxes = np.column_stack([
        box_xy[:, 0] - 0.5 * sides[:, 0], box_xy[:, 1] - 0.5 * sides[:, 1],
        np.zeros(box_xy.shape[0]),
        box_xy[:, 0] + 0.5 * sides[:, 0], box_xy[:, 1] + 0.5 * sides[:, 1],
        sides[:, 2]])
    cyls = np.column_stack([cyl_xy[:, 0], cyl_xy[:, 1], rad, hgt])
    return Scene(boxes=boxes, cyls=cyls)


def _az_window(dx, dy, rb, yaw, az0, step, ncol, reach):
    """Azimuth columns whose rays can meet a disc of radius rb at (dx, dy).

    Returns None when the disc is out of reach, an index array otherwise.
    """
    r = math.hypot(dx, dy)
    if r - rb > reach:
        return None
    if r <= rb * 1.001 + 1e-9:
        return np.arange(ncol)
    half = math.asin(min(1.0, rb / r)) + step
    ac = math.atan2(dy, dx) - yaw - az0
    lo = math.floor((ac - half) / step)
    hi = math.ceil((ac + half) / step)
    if hi - lo + 1 >= ncol:
        return np.arange(ncol)
    return np.arange(lo, hi + 1) % ncol


def _cast_revolution(sensor: SensorModel, origin, yaw, az0_deg, scene: Scene):
    """Nearest hit distance for every ray of one revolution.

    Returns (t, ux, uy, uz) with shape (n_cols, n_beams); t = inf for a miss.
    """
    ncol, nb = sensor.n_cols, sensor.n_beams
    step = math.radians(sensor.az_step_deg)
    az0 = math.radians(az0_deg)
    el = np.radians(np.linspace(sensor.el_min_deg, sensor.el_max_deg, nb))
    az = yaw + az0 + np.arange(ncol) * step
    ce, se = np.cos(el), np.sin(el)
    ca, sa = np.cos(az), np.sin(az)
    ux = ca[:, None] * ce[None, :]
    uy = sa[:, None] * ce[None, :]
    uz = np.broadcast_to(se[None, :], (ncol, nb))
    ox, oy, oz = (float(v) for v in origin)

    # ground plane z = 0 (only downward beams reach it)
    down = se < 0.0
    tg = np.full(nb, np.inf)
    tg[down] = -oz / se[down]
    t = np.broadcast_to(tg[None, :], (ncol, nb)).copy()

    reach = sensor.r_max + 1.0
    with np.errstate(divide="ignore", invalid="ignore"):
        for b in scene.boxes:
            cx, cy = 0.5 * (b[0] + b[3]), 0.5 * (b[1] + b[4])
            rb = 0.5 * math.hypot(b[3] - b[0], b[4] - b[1])
            cols = _az_window(cx - ox, cy - oy, rb, yaw, az0, step, ncol, reach)
            if cols is None:
                continue
            vx, vy, vz = ux[cols], uy[cols], uz[cols]
            ix, iy, iz = 1.0 / vx, 1.0 / vy, 1.0 / vz
            ax, bx_ = (b[0] - ox) * ix, (b[3] - ox) * ix
            ay, by_ = (b[1] - oy) * iy, (b[4] - oy) * iy
            az_, bz_ = (b[2] - oz) * iz, (b[5] - oz) * iz
            tmin = np.maximum(np.maximum(np.minimum(ax, bx_), np.minimum(ay, by_)),
                              np.minimum(az_, bz_))
            tmax = np.minimum(np.minimum(np.maximum(ax, bx_), np.maximum(ay, by_)),
                              np.maximum(az_, bz_))
            hit = (tmax >= tmin) & (tmin > 0.0)
            tb = np.where(hit, tmin, np.inf)
            t[cols] = np.minimum(t[cols], tb)
        for c in scene.cyls:
            cols = _az_window(c[0] - ox, c[1] - oy, c[2], yaw, az0, step, ncol, reach)
            if cols is None:
                continue
            vx, vy, vz = ux[cols], uy[cols], uz[cols]
            fx, fy = ox - c[0], oy - c[1]
            a = vx * vx + vy * vy
            bq = 2.0 * (fx * vx + fy * vy)
            cq = fx * fx + fy * fy - c[2] * c[2]
            disc = bq * bq - 4.0 * a * cq
            t1 = (-bq - np.sqrt(np.maximum(disc, 0.0))) / (2.0 * a)
            z1 = oz + t1 * vz
            hit = (disc >= 0.0) & (t1 > 0.0) & (z1 >= 0.0) & (z1 <= c[3])
            tc = np.where(hit, t1, np.inf)
            t[cols] = np.minimum(t[cols], tc)
    return t, ux, uy, uz


def _scan(sensor: SensorModel, origin, yaw, scene: Scene, n_target: int, rng):
    """Simulated returns of one sensor position, exactly ``n_target`` points.

    Revolutions are added until the pool of returns reaches ``n_target``;
    the pool is then subsampled without replacement and kept in ray order
    (revolution, azimuth column, beam).
    """
    pools = []
    total = 0
    k = 0
    while total < n_target:
        if k >= 64:
            raise RuntimeError("scene yields too few returns for n_target=%d" % n_target)
        az0 = (k * _GOLDEN % 1.0) * sensor.az_step_deg
        t, ux, uy, uz = _cast_revolution(sensor, origin, yaw, az0, scene)
        noise = rng.normal(0.0, sensor.range_sigma, size=t.shape)
        drop = rng.random(size=t.shape) < sensor.drop_prob
        keep = (t >= sensor.r_min) & (t <= sensor.r_max) & ~drop
        r = (t + noise)[keep]
        pts = np.empty((r.size, 3))
        pts[:, 0] = origin[0] + r * ux[keep]
        pts[:, 1] = origin[1] + r * uy[keep]
        pts[:, 2] = origin[2] + r * uz[keep]
        pools.append(pts)
        total += r.size
        k += 1
    pool = np.concatenate(pools, axis=0)
    pick = np.sort(rng.choice(pool.shape[0], size=n_target, replace=False))
    return pool[pick]


# --------------------------------------------------------------------------
# the three plain-path workloads
# --------------------------------------------------------------------------

def blobs_cloud(n: int = 20000, n_blobs: int = 40, sigma: float = 0.3,
                size_range=(300, 700), box=(50.0, 50.0, 5.0), seed: int = 1,
                return_truth: bool = False):
    """Gaussian blobs plus uniform noise on the z=0 plane, shuffled.

    Blob sizes are integers drawn uniformly from ``size_range``; the draw of
    all sizes is repeated until their sum does not exceed ``n`` so that the
    noise count ``n - sum`` is never negative.  The cloud is then put in a
    seeded random index order (the paper randomises indices of its synthetic
    clouds, Sec. 3.3).  With ``return_truth`` the generating blob id of each
    point is returned as well (-1 for noise).
    """
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, 1.0, size=(n_blobs, 3)) * np.asarray(box, dtype=np.float64)
    for _ in range(10000):
        sizes = rng.integers(size_range[0], size_range[1] + 1, size=n_blobs)
        if sizes.sum() <= n:
            break
    else:
        raise RuntimeError("cannot draw blob sizes summing to <= n")
    parts = [centres[b] + rng.normal(0.0, sigma, size=(int(sizes[b]), 3))
             for b in range(n_blobs)]
    n_noise = n - int(sizes.sum())
    noise = np.zeros((n_noise, 3))
    noise[:, 0] = rng.uniform(0.0, box[0], size=n_noise)
    noise[:, 1] = rng.uniform(0.0, box[1], size=n_noise)
    pts = np.concatenate(parts + [noise], axis=0)
    truth = np.concatenate([np.full(int(s), b) for b, s in enumerate(sizes)] +
                           [np.full(n_noise, -1)]).astype(np.int32)
    perm = rng.permutation(n)
    xyz = np.ascontiguousarray(pts[perm].astype(np.float32))
    if return_truth:
        return xyz, truth[perm]
    return xyz


def _ring_place(rng, r_lo=4.0, r_hi=70.0):
    """Placement around a sensor at the origin.

    Each object's centre is at angle U[0, 2*pi) and at a radius drawn so
    that its whole footprint lies in the annulus r_lo..r_hi (radius
    U[r_lo + rb, r_hi - rb]).
    """
    def place(rb):
        k = rb.shape[0]
        u = rng.uniform(0.0, 1.0, size=k)
        a = rng.uniform(0.0, 2.0 * math.pi, size=k)
        r = (r_lo + rb) + u * ((r_hi - rb) - (r_lo + rb))
        return np.column_stack([r * np.cos(a), r * np.sin(a)])
    return place


def lidar_frame(n: int = 120000, seed: int = 2, n_boxes: int = 60, n_cyls: int = 30,
                sensor: SensorModel = SensorModel()):
    """One scan of a seeded scene, sensor at (0, 0, height), exactly n points.

    Scene: 60 boxes and 30 cylinders centred at radius U[4, 70] m and angle
    U[0, 2*pi) around the sensor.  Output is in ray order.
    """
    scene_ss, scan_ss = np.random.SeedSequence(seed).spawn(2)
    srng = np.random.default_rng(scene_ss)
    scene = _make_objects(srng, n_boxes, n_cyls, _ring_place(srng))
    pts = _scan(sensor, (0.0, 0.0, sensor.height), 0.0, scene, n,
                np.random.default_rng(scan_ss))
    return np.ascontiguousarray(pts.astype(np.float32))


def map_trajectory(n_poses: int = 200, step: float = 10.0, heading_sigma_deg: float = 10.0,
                   seed: int = 3):
    """Seeded 2-D random walk: (x, y, heading) per pose, starting at the origin."""
    world_ss = np.random.SeedSequence(seed).spawn(2)[0]
    rng = np.random.default_rng(world_ss)
    turns = rng.normal(0.0, math.radians(heading_sigma_deg), size=n_poses)
    head = np.empty(n_poses)
    xy = np.zeros((n_poses, 2))
    h = 0.0
    for k in range(n_poses):
        if k > 0:
            xy[k] = xy[k - 1] + step * np.array([math.cos(h), math.sin(h)])
            h = h + turns[k]
        head[k] = h
    return xy, head, rng


def _dist_to_polyline(p, poly):
    """Distance from each point of p (k,2) to the polyline poly (m,2)."""
    best = np.full(p.shape[0], np.inf)
    for a, b in zip(poly[:-1], poly[1:]):
        ab = b - a
        den = float(ab @ ab)
        s = np.clip(((p - a) @ ab) / den, 0.0, 1.0) if den > 0 else np.zeros(p.shape[0])
        q = a + s[:, None] * ab
        best = np.minimum(best, np.hypot(p[:, 0] - q[:, 0], p[:, 1] - q[:, 1]))
    return best


def _map_world(n_poses, seed, buffer=70.0, road=4.0):
    """Trajectory plus one static scene along it.

    Object counts follow one frame-scene's density (60 boxes and 30
    cylinders per pi*(70^2-4^2) m^2) over the trajectory's bounding box
    grown by ``buffer``; an object is kept when its footprint lies between
    ``road`` and ``buffer`` metres from the trajectory polyline.
    """
    xy, head, rng = map_trajectory(n_poses=n_poses, seed=seed)
    area = math.pi * (70.0 ** 2 - 4.0 ** 2)
    lo = xy.min(axis=0) - buffer
    hi = xy.max(axis=0) + buffer
    bb_area = float(np.prod(hi - lo))

    def place(rb):
        cand = rng.uniform(0.0, 1.0, size=(rb.shape[0], 2)) * (hi - lo) + lo
        dist = _dist_to_polyline(cand, xy)
        ok = (dist - rb >= road) & (dist + rb <= buffer)
        cand[~ok] = np.nan
        return cand

    scene = _make_objects(rng, int(round(60.0 / area * bb_area)),
                          int(round(30.0 / area * bb_area)), place)
    return xy, head, scene


_CACHE_VERSION = hashlib.sha1(open(__file__, "rb").read()).hexdigest()[:12]


def _cache_path(tag: str):
    root = os.environ.get("FEC_SYNTH_CACHE", os.path.join(tempfile.gettempdir(), "fec_synth_cache"))
    if root in ("", "0", "off"):
        return None
    os.makedirs(root, exist_ok=True)
    return os.path.join(root, "%s_%s.npy" % (tag, _CACHE_VERSION))


def lidar_map(n_frames: int = 200, pts_per_frame: int = 135000, seed: int = 3,
              jitter_sigma: float = 0.05, frames=None, n_poses: int = 200,
              sensor: SensorModel = SensorModel(), workers: int | None = None,
              cache: bool = True):
    """Frames of one static world registered along a random-walk trajectory.

    The trajectory has ``n_poses`` poses 10 m apart with the heading
    perturbed by N(0, (10 deg)^2) per step.  The world is the ground plane
    plus boxes and cylinders at one frame-scene's density (60 boxes and 30
    cylinders per pi*(70^2-4^2) m^2), uniform in the corridor between 4 m and
    70 m from the trajectory.  Frame k is a scan from pose k; its points get
    one translation N(0, jitter^2 I) (registration error).  Output is
    frame-major, each frame in ray order; ``frames`` selects a subset of
    frame indices (default: the first ``n_frames``).
    """
    if frames is None:
        frames = list(range(n_frames))
    frames = [int(f) for f in frames]
    tag = "map_s%d_p%d_n%d_j%g_f%s" % (
        seed, n_poses, pts_per_frame, jitter_sigma,
        hashlib.sha1(np.asarray(frames, dtype=np.int64).tobytes()).hexdigest()[:10])
    path = _cache_path(tag) if cache else None
    if path is not None and os.path.exists(path):
        arr = np.load(path, mmap_mode=None, allow_pickle=False)
        if arr.shape == (len(frames) * pts_per_frame, 3) and arr.dtype == np.float32:
            return arr
    xy, head, scene = _map_world(n_poses, seed)
    frame_ss = np.random.SeedSequence(seed).spawn(2)[1].spawn(n_poses)
    out = np.empty((len(frames) * pts_per_frame, 3), dtype=np.float32)

    def one(slot_frame):
        slot, f = slot_frame
        rng = np.random.default_rng(frame_ss[f])
        jit = rng.normal(0.0, jitter_sigma, size=3)
        origin = (xy[f, 0], xy[f, 1], sensor.height)
        pts = _scan(sensor, origin, head[f], scene, pts_per_frame, rng)
        pts += jit[None, :]
        out[slot * pts_per_frame:(slot + 1) * pts_per_frame] = pts.astype(np.float32)

    nw = workers if workers is not None else min(8, os.cpu_count() or 1)
    if nw <= 1 or len(frames) <= 1:
        for sf in enumerate(frames):
            one(sf)
    else:
        with ThreadPoolExecutor(max_workers=nw) as ex:
            list(ex.map(one, enumerate(frames)))
    if path is not None:
        tmp = path + ".tmp%d.npy" % os.getpid()
        np.save(tmp, out)
        os.replace(tmp, path)
    return out


# --------------------------------------------------------------------------
# small structured clouds for tests
# --------------------------------------------------------------------------

def random_cloud(n: int, extent=(10.0, 10.0, 10.0), seed: int = 0, offset=(0.0, 0.0, 0.0)):
    """n points uniform in an axis-aligned box (float32)."""
    rng = np.random.default_rng(seed)
    p = rng.uniform(0.0, 1.0, size=(n, 3)) * np.asarray(extent) + np.asarray(offset)
    return np.ascontiguousarray(p.astype(np.float32))


def blob_lattice(extent=(6.0, 6.0), spacing: float = 0.22, jitter: float = 0.02,
                 pts_per_blob: int = 30, radius: float = 0.01, layers: int = 1, seed: int = 0,
                 origin=(0.0, 0.0, 0.0)):
    """Tight blobs on a jittered lattice: `layers` planes of blobs `spacing`
    apart in x, y and z, each blob `pts_per_blob` points uniform in a cube of
    half-side `radius` around its centre (float32, shuffled).  With a
    spacing near the clustering distance about half of the neighbouring
    blobs end up within reach of each other, so a dense patch holds many
    clusters of varied shapes."""
    rng = np.random.default_rng(seed)
    nx = max(1, int(extent[0] / spacing))
    ny = max(1, int(extent[1] / spacing))
    gx, gy, gz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(layers), indexing="ij")
    centres = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1) * spacing
    centres = centres + rng.uniform(-jitter, jitter, size=centres.shape) + np.asarray(origin)
    pts = np.repeat(centres, pts_per_blob, axis=0)
    pts = pts + rng.uniform(-radius, radius, size=pts.shape)
    pts = pts[rng.permutation(pts.shape[0])]
    return np.ascontiguousarray(pts.astype(np.float32))


def chain_cloud(n: int, spacing: float, axis: int = 0, origin=(0.0, 0.0, 0.0)):
    """Collinear points p_k = origin + k * spacing * e_axis (float32)."""
    p = np.zeros((n, 3))
    p[:] = origin
    p[:, axis] += np.arange(n) * spacing
    return np.ascontiguousarray(p.astype(np.float32))


def near_threshold_cloud(n_pairs: int, d: float, seed: int = 0, max_ulps: int = 3,
                         spread: float = 1000.0):
    """Point pairs whose separation straddles d by a few float32 ulps.

    Half of the pairs are axis-aligned: p and q = p + delta * e_axis with
    delta = d +/- k ulps chosen so that the float32 difference is exact.  The
    other half are in random directions at length d * (1 + eps) with
    |eps| < 4e-7, where the rounding of the squared sum decides.  Pair
    centres are spread over ``spread`` m so that pairs do not touch.
    """
    rng = np.random.default_rng(seed)
    d32 = np.float32(d)
    out = np.zeros((2 * n_pairs, 3), dtype=np.float32)
    # quantise pair anchors so that anchor + delta is exact in float32
    q = np.float32(2.0 ** math.floor(math.log2(spread) + 1 - 24 + 1))
    for k in range(n_pairs):
        base = np.floor(rng.uniform(0.0, spread, size=3) / q) * q
        p = base.astype(np.float32)
        if k % 2 == 0:
            ax = int(rng.integers(0, 3))
            ulps = int(rng.integers(-max_ulps, max_ulps + 1))
            delta = d32
            step = np.float32(np.inf) if ulps > 0 else np.float32(-np.inf)
            for _ in range(abs(ulps)):
                delta = np.nextafter(delta, step)
            qp = p.copy()
            qp[ax] = np.float32(p[ax] + delta)
        else:
            u = rng.normal(size=3)
            u /= np.linalg.norm(u)
            r = float(d) * (1.0 + rng.uniform(-4e-7, 4e-7))
            qp = (p.astype(np.float64) + r * u).astype(np.float32)
        out[2 * k] = p
        out[2 * k + 1] = qp
    return out


def lidar_batch(n_frames: int = 64, n_lo: int = 20000, n_hi: int = 200000,
                ds=(0.2, 0.35, 0.5), seed: int = 4):
    """Independent LiDAR frames for a batched call: (list of xyz, list of d).

    Frame b has round(exp(U[ln n_lo, ln n_hi])) points (log-uniform count),
    its own scene seed, and d drawn uniformly from ``ds``.
    """
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x6261]))
    counts = np.rint(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), n_frames))).astype(np.int64)
    dsel = rng.integers(0, len(ds), n_frames)
    seeds = rng.integers(0, 2**31 - 1, n_frames)
    frames = [lidar_frame(n=int(counts[b]), seed=int(seeds[b])) for b in range(n_frames)]
    return frames, [float(ds[int(k)]) for k in dsel]


def serve_trace(n_requests: int = 10000, rate: float = 400.0, pool: int = 512,
                n_lo: int = 5000, n_hi: int = 500000, ds=(0.2, 0.5), seed: int = 5):
    """A request stream for the serving engine.

    Returns (frames, arrivals, frame_of, d_of): a pool of ``pool`` seeded
    LiDAR frames with log-uniform point counts in [n_lo, n_hi]; Poisson
    arrival times (seconds, exponential gaps of mean 1/rate); for every
    request the pool frame it carries (drawn with replacement) and its d
    (uniform over ``ds``).
    """
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x7365]))
    counts = np.rint(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), pool))).astype(np.int64)
    seeds = rng.integers(0, 2**31 - 1, pool)
    frames = [lidar_frame(n=int(counts[b]), seed=int(seeds[b])) for b in range(pool)]
    arrivals = np.cumsum(rng.exponential(1.0 / rate, n_requests))
    frame_of = rng.integers(0, pool, n_requests)
    d_of = np.asarray(ds, dtype=np.float64)[rng.integers(0, len(ds), n_requests)]
    return frames, arrivals, frame_of, d_of


def voxel_clusters(n_clusters: int, density: int, subclusters: int = 0, voxel: float = 1.0,
                   seed: int = 0):
    """Synthetic clusters in the manner of the paper's synthetic experiments.

    Space is divided into cubic voxels of side ``voxel``; ``n_clusters``
    voxels are picked at random among the sites of a lattice of pitch two
    voxels (so an empty voxel separates any two clusters) and each is filled
    with ``density`` points: evenly (a random subset of a k x k x k lattice
    inside the voxel, k = ceil(density^(1/3))) when ``subclusters`` is 0,
    else around ``subclusters`` Gaussian sub-cluster centres (uniform in the
    voxel's middle 70 %, sigma = voxel / 8, clipped to the voxel).  The point
    order is shuffled.  Returns (xyz float32 [n_clusters * density, 3],
    ground-truth cluster id int32 [n]).
    """
    rng = np.random.default_rng(np.random.SeedSequence([seed, n_clusters, density,
                                                        subclusters, 0x766F]))
    L = 1
    while L ** 3 < 2 * n_clusters:
        L += 1
    sites = rng.choice(L ** 3, size=n_clusters, replace=False)
    corner = np.stack(np.unravel_index(sites, (L, L, L)), 1).astype(np.float64) * 2.0 * voxel
    m = int(density)
    if subclusters <= 0:
        k = 1
        while k ** 3 < m:
            k += 1
        g = (np.arange(k, dtype=np.float64) + 0.5) * voxel / k
        lat = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
        pick = np.argsort(rng.random((n_clusters, k ** 3)), axis=1)[:, :m]
        pts = corner[:, None, :] + lat[pick]
    else:
        centres = corner[:, None, :] + rng.uniform(0.15, 0.85, (n_clusters, subclusters, 3)) * voxel
        which = rng.integers(0, subclusters, (n_clusters, m))
        pts = np.take_along_axis(centres, which[..., None], axis=1)
        pts = pts + rng.normal(0.0, voxel / 8.0, (n_clusters, m, 3))
        lo = corner[:, None, :]
        pts = np.clip(pts, lo, lo + voxel * (1.0 - 1e-6))
    gt = np.repeat(np.arange(n_clusters, dtype=np.int32), m)
    order = rng.permutation(n_clusters * m)
    xyz = pts.reshape(-1, 3)[order].astype(np.float32)
    return np.ascontiguousarray(xyz), gt[order]


# The synthetic sweeps: (experiment, n_clusters, density, subclusters), d = 0.9 voxel.
SWEEP_D = 0.9
SWEEPS = (
    [("E1 density x clusters", c, m, 0) for c in (100, 700, 1300, 1900, 2200)
     for m in (10, 100, 200, 300, 400, 500)]
    + [("E2 clusters at density 200", c, 200, 0) for c in (100, 400, 700, 1000, 1300, 1600, 1900)]
    + [("E3 Gaussian sub-clusters", 1000, 200, s) for s in (1, 2, 4, 8, 16)]
    + [("E4 clusters and density together", c, m, 0)
       for c, m in ((100, 10), (500, 100), (1000, 200), (1600, 350), (2200, 500))]
)


# --------------------------------------------------------------------------
# named configurations
# --------------------------------------------------------------------------

CONFIGS = {
    "blobs20k": dict(kind="blobs", n=20000, d=0.5, min_size=10, max_size=20000, seed=1),
    "lidar120k": dict(kind="frame", n=120000, d=0.35, min_size=50, max_size=100000, seed=2),
    "map27m": dict(kind="map", n=27000000, d=0.2, min_size=100, max_size=5000000, seed=3,
                   n_frames=200, pts_per_frame=135000),
    # batched frames: lidar_batch(64 frames, 20k-200k points, d in {0.2, 0.35, 0.5})
    "batch64": dict(kind="batch", n_frames=64, n_lo=20000, n_hi=200000, min_size=30,
                    max_size=200000, seed=4),
}


def make_config(name: str, frames=None, **kw):
    """(xyz float32 [n,3], d, min_size, max_size) for a named workload.

    For ``map27m`` a frame subset can be requested with ``frames`` (a list of
    frame indices or an int k meaning the first k frames).
    """
    c = dict(CONFIGS[name])
    c.update(kw)
    if c["kind"] == "batch":
        raise ValueError("%s is a batch of frames: use make_batch_config" % name)
    if c["kind"] == "blobs":
        xyz = blobs_cloud(n=c["n"], seed=c["seed"])
    elif c["kind"] == "frame":
        xyz = lidar_frame(n=c["n"], seed=c["seed"])
    else:
        if isinstance(frames, int):
            frames = list(range(frames))
        xyz = lidar_map(n_frames=c["n_frames"], pts_per_frame=c["pts_per_frame"],
                        seed=c["seed"], frames=frames)
    return xyz, float(c["d"]), int(c["min_size"]), int(c["max_size"])


def make_batch_config(name: str = "batch64", **kw):
    """(list of xyz, list of d, min_size, max_size) for a named batch workload."""
    c = dict(CONFIGS[name])
    c.update(kw)
    frames, ds = lidar_batch(n_frames=c["n_frames"], n_lo=c["n_lo"], n_hi=c["n_hi"],
                             seed=c["seed"])
    return frames, ds, int(c["min_size"]), int(c["max_size"])
