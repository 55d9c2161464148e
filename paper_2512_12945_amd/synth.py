"""Seeded synthetic inputs for the integration workloads.

This module builds scenes and casts sensor rays against them analytically, in
FP64 numpy, and hands out posed point clouds with their per-point semantics.
It holds none of the mapping method's arithmetic (no voxel walk, no signed
distance of voxels, no fusion): both the HIP path and the CPU oracle take its
arrays as inputs, and neither depends on the other.

Workloads (the paper evaluates on SemanticKITTI and SceneNet with trained
segmentation networks; these synthetic scenes stand in for them):

* ``room_frame``     -- one 64x64 pinhole depth frame of a 4x4x3 m box room,
  seen from its centre, 5-class soft labels (softmax of logits).
* ``StreetScene``    -- a street of 200 boxes and 100 cylinders on a ground
  plane, swept by a 64-beam x 1024-azimuth spinning LiDAR along x, 20 classes by
  primitive id with 10 % per-frame label flicker.
* ``OpenRoomScene``  -- an 8x8x3 m room with 50 boxes seen by a 640x480 RGB-D
  camera on a circular orbit, per-pixel 512-d embeddings (per-object prototype
  plus noise, L2-normalised, bfloat16).

Point clouds are in the sensor frame (float32, N x 3); a pose is the 4x4
row-major FP64 transform map_T_sensor.  Rays that miss, or fall outside the
sensor's range, come back as NaN points.
"""
from __future__ import annotations

import numpy as np

# ----------------------------------------------------------------------------
# helpers
# ----------------------------------------------------------------------------


def _rng(*seed):
    return np.random.default_rng(list(seed))


def pose_matrix(R, t):
    P = np.eye(4)
    P[:3, :3] = R
    P[:3, 3] = t
    return P


def rot_z(yaw):
    c, s = np.cos(yaw), np.sin(yaw)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def camera_rotation(forward, up=(0.0, 0.0, 1.0)):
    """Rotation whose columns are the camera axes (x right, y down, z forward) in the world."""
    f = np.asarray(forward, float)
    f = f / np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, float))
    r = r / np.linalg.norm(r)
    d = np.cross(f, r)
    return np.stack([r, d, f], axis=1)


def softmax64(x):
    x = np.asarray(x, np.float64)
    e = np.exp(x - x.max(axis=-1, keepdims=True))
    return e / e.sum(axis=-1, keepdims=True)


def to_bf16_bits(x):
    """Round float32 values to bfloat16 (round to nearest even); returns uint16 bit patterns."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32)
    r = (u >> 16) & 1
    r += 0x7FFF
    r += u  # finite inputs cannot overflow 32 bits
    r >>= 16
    return r.astype(np.uint16)


def bf16_bits_to_float(b):
    return (np.asarray(b, np.uint16).astype(np.uint32) << 16).view(np.float32)


def _ray_box_inside(o, d, lo, hi):
    """Exit distance and face id (0..5: -x,+x,-y,+y,-z,+z) of rays from inside a box."""
    with np.errstate(divide="ignore", invalid="ignore"):
        tx = np.where(d[:, 0] > 0, (hi[0] - o[0]) / d[:, 0], (lo[0] - o[0]) / d[:, 0])
        ty = np.where(d[:, 1] > 0, (hi[1] - o[1]) / d[:, 1], (lo[1] - o[1]) / d[:, 1])
        tz = np.where(d[:, 2] > 0, (hi[2] - o[2]) / d[:, 2], (lo[2] - o[2]) / d[:, 2])
    T = np.stack([tx, ty, tz], axis=1)
    T[~np.isfinite(T)] = np.inf
    T[T < 0] = np.inf
    ax = np.argmin(T, axis=1)
    t = T[np.arange(len(d)), ax]
    face = 2 * ax + (d[np.arange(len(d)), ax] > 0)
    return t, face


def _ray_boxes(o, d, lo, hi, reach=np.inf):
    """Nearest entry distance of rays (origin o, dirs d: N x 3) into boxes (M x 3 corners).

    Boxes farther than ``reach`` from o are skipped.  Returns (t, idx), t = inf where
    nothing is hit."""
    N = d.shape[0]
    t_best = np.full(N, np.inf)
    i_best = np.full(N, -1, np.int64)
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / d
    for j in range(lo.shape[0]):
        near = np.linalg.norm(np.clip(o, lo[j], hi[j]) - o)
        if near > reach:
            continue
        tn = np.full(N, -np.inf)
        tf = np.full(N, np.inf)
        for a in range(3):
            with np.errstate(invalid="ignore"):
                t1 = (lo[j, a] - o[a]) * inv[:, a]
                t2 = (hi[j, a] - o[a]) * inv[:, a]
            par = d[:, a] == 0.0
            inside = lo[j, a] <= o[a] <= hi[j, a]
            lo_a = np.where(par, -np.inf if inside else np.inf, np.minimum(t1, t2))
            hi_a = np.where(par, np.inf if inside else -np.inf, np.maximum(t1, t2))
            np.maximum(tn, lo_a, out=tn)
            np.minimum(tf, hi_a, out=tf)
        hit = (tn <= tf) & (tn > 1e-9) & (tn < t_best)
        t_best = np.where(hit, tn, t_best)
        i_best = np.where(hit, j, i_best)
    return t_best, i_best


def _ray_cylinders(o, d, cxy, rad, h, reach=np.inf):
    """Nearest hit of rays with vertical cylinders standing on z = 0 (side and top cap)."""
    N = d.shape[0]
    t_best = np.full(N, np.inf)
    i_best = np.full(N, -1, np.int64)
    a = d[:, 0] ** 2 + d[:, 1] ** 2
    for j in range(cxy.shape[0]):
        if np.hypot(o[0] - cxy[j, 0], o[1] - cxy[j, 1]) - rad[j] > reach:
            continue
        ox, oy = o[0] - cxy[j, 0], o[1] - cxy[j, 1]
        b = 2.0 * (d[:, 0] * ox + d[:, 1] * oy)
        c = ox * ox + oy * oy - rad[j] ** 2
        disc = b * b - 4 * a * c
        with np.errstate(divide="ignore", invalid="ignore"):
            ts = (-b - np.sqrt(np.maximum(disc, 0.0))) / (2 * a)
            z = o[2] + ts * d[:, 2]
            side = (disc >= 0) & (a > 0) & (ts > 1e-9) & (z >= 0) & (z <= h[j])
            tc = (h[j] - o[2]) / d[:, 2]
            px = ox + tc * d[:, 0]
            py = oy + tc * d[:, 1]
            cap = (tc > 1e-9) & (px * px + py * py <= rad[j] ** 2)
        tt = np.minimum(np.where(side, ts, np.inf), np.where(cap, tc, np.inf))
        hit = tt < t_best
        t_best = np.where(hit, tt, t_best)
        i_best = np.where(hit, j, i_best)
    return t_best, i_best


# ----------------------------------------------------------------------------
# tiny room, one pinhole frame, closed set with soft labels
# ----------------------------------------------------------------------------

ROOM_CLASSES = 5  # floor 0, ceiling 1, x=0 wall 2, x=max wall 3, y walls 4


def room_frame(seed=1, width=64, height=64, f=50.0, cx=32.0, cy=32.0, room=(4.0, 4.0, 3.0),
               position=(2.0, 2.0, 1.5), forward=(1.0, 0.0, 0.0), noise=0.005, true_logit=3.0):
    """One pinhole frame of a box room; 5 classes given as softmax probabilities (float32).

    Returns dict(points N x 3 f32 sensor frame, pose 4x4 f64, prob N x 5 f32,
    label N i32 (true class), logits N x 5 f32)."""
    rng = _rng(seed, 0)
    R = camera_rotation(forward)
    u, v = np.meshgrid(np.arange(width), np.arange(height))
    dc = np.stack([((u + 0.5) - cx) / f, ((v + 0.5) - cy) / f, np.ones_like(u, float)], axis=-1).reshape(-1, 3)
    dc = dc / np.linalg.norm(dc, axis=1, keepdims=True)
    dw = dc @ R.T
    o = np.asarray(position, float)
    t, face = _ray_box_inside(o, dw, np.zeros(3), np.asarray(room, float))
    cls = np.array([2, 3, 4, 4, 0, 1])[face]
    r = t + rng.normal(0.0, noise, size=t.shape)
    pts = (dc * r[:, None]).astype(np.float32)
    logits = rng.normal(0.0, 1.0, size=(len(t), ROOM_CLASSES))
    logits[np.arange(len(t)), cls] = true_logit
    prob = softmax64(logits).astype(np.float32)
    return dict(points=pts, pose=pose_matrix(R, o), prob=prob, label=cls.astype(np.int32),
                logits=logits.astype(np.float32))


def room_sequence(nframes, seed=11, yaw_span=2 * np.pi, **kw):
    """Frames of the same room from near its centre, turning by ``yaw_span`` in total
    and tilting, so that corners, floor and ceiling come into view.  A small span
    makes consecutive frames overlap."""
    out = []
    for i in range(nframes):
        yaw = yaw_span * i / max(nframes, 1) + 0.3
        pitch = 0.35 * np.sin(1.7 * i + 0.2)
        fwd = (np.cos(yaw) * np.cos(pitch), np.sin(yaw) * np.cos(pitch), np.sin(pitch))
        pos = (2.0 + 0.3 * np.cos(i), 2.0 + 0.3 * np.sin(i), 1.5)
        out.append(room_frame(seed=seed * 1000 + i, forward=fwd, position=pos, **kw))
    return out


# ----------------------------------------------------------------------------
# LiDAR street, closed set with hard labels
# ----------------------------------------------------------------------------

STREET_CLASSES = 20


class StreetScene:
    """Ground plane z = 0, 200 axis-aligned boxes (sides 1-10 m) and 100 vertical
    cylinders (radius 0.2-1 m, height 2-8 m) along a street that runs in +x.

    Obstacles keep a clear corridor of 3 m either side of y = 0."""

    def __init__(self, seed=2, nboxes=200, ncyl=100, beams=64, azimuths=1024, fov=(-25.0, 3.0),
                 max_range=50.0, height=1.8, flicker=0.1, yaw_sigma=0.01):
        rng = _rng(seed, 1)
        sz = rng.uniform(1.0, 10.0, size=(nboxes, 3))
        cx = rng.uniform(-10.0, 110.0, nboxes)
        side = rng.choice([-1.0, 1.0], nboxes)
        cy = side * np.maximum(rng.uniform(5.0, 40.0, nboxes), 3.0 + sz[:, 1] / 2)
        self.box_lo = np.stack([cx - sz[:, 0] / 2, cy - sz[:, 1] / 2, np.zeros(nboxes)], axis=1)
        self.box_hi = np.stack([cx + sz[:, 0] / 2, cy + sz[:, 1] / 2, sz[:, 2]], axis=1)
        rad = rng.uniform(0.2, 1.0, ncyl)
        ccx = rng.uniform(-10.0, 110.0, ncyl)
        cside = rng.choice([-1.0, 1.0], ncyl)
        ccy = cside * np.maximum(rng.uniform(5.0, 40.0, ncyl), 3.0 + rad)
        self.cyl_xy = np.stack([ccx, ccy], axis=1)
        self.cyl_r = rad
        self.cyl_h = rng.uniform(2.0, 8.0, ncyl)
        self.box_class = 1 + (np.arange(nboxes) % 12)
        self.cyl_class = 13 + (np.arange(ncyl) % 7)
        self.seed = seed
        self.beams, self.azimuths = beams, azimuths
        self.max_range = max_range
        self.height = height
        self.flicker = flicker
        self.yaw_sigma = yaw_sigma
        el = np.deg2rad(np.linspace(fov[0], fov[1], beams))
        az = (np.arange(azimuths) + 0.5) * 2 * np.pi / azimuths
        A, E = np.meshgrid(az, el, indexing="ij")  # azimuth-major order
        self.dirs = np.stack([np.cos(E) * np.cos(A), np.cos(E) * np.sin(A), np.sin(E)], axis=-1).reshape(-1, 3)

    @property
    def n_rays(self):
        return self.dirs.shape[0]

    def pose(self, t):
        yaw = _rng(self.seed, 2, t).normal(0.0, self.yaw_sigma)
        return pose_matrix(rot_z(yaw), (float(t), 0.0, self.height))

    def cast(self, pose, dirs_s):
        """Range and primitive class of sensor-frame unit rays; inf range where nothing is hit."""
        R, o = pose[:3, :3], pose[:3, 3]
        d = dirs_s @ R.T
        with np.errstate(divide="ignore", invalid="ignore"):
            tg = np.where(d[:, 2] < 0, -o[2] / d[:, 2], np.inf)
        tb, ib = _ray_boxes(o, d, self.box_lo, self.box_hi, reach=self.max_range)
        tc, ic = _ray_cylinders(o, d, self.cyl_xy, self.cyl_r, self.cyl_h, reach=self.max_range)
        T = np.stack([tg, tb, tc], axis=1)
        which = np.argmin(T, axis=1)
        t = T[np.arange(len(T)), which]
        cls = np.zeros(len(t), np.int64)
        cls = np.where(which == 1, self.box_class[np.maximum(ib, 0)], cls)
        cls = np.where(which == 2, self.cyl_class[np.maximum(ic, 0)], cls)
        # primitive index: ground 0, boxes 1.., cylinders after the boxes
        prim = np.where(which == 1, 1 + np.maximum(ib, 0), 0)
        prim = np.where(which == 2, 1 + len(self.box_lo) + np.maximum(ic, 0), prim)
        self._last_prim = prim
        return t, cls

    def sweeps(self, ts, workers=8):
        """Several sweeps, generated in worker processes."""
        ts = list(ts)
        if workers <= 1 or len(ts) < 4:
            return [self.sweep(t) for t in ts]
        import concurrent.futures as cf
        import multiprocessing as mp

        with cf.ProcessPoolExecutor(max_workers=min(workers, len(ts)), mp_context=mp.get_context("fork")) as ex:
            return list(ex.map(self.sweep, ts))

    def sweep(self, t, nrays=None):
        """Sweep number t: points (NaN where no return within range), pose, labels (with flicker)."""
        pose = self.pose(t)
        dirs = self.dirs if nrays is None else self.dirs[:nrays]
        r, cls = self.cast(pose, dirs)
        miss = ~(r <= self.max_range)
        pts = (dirs * r[:, None]).astype(np.float32)
        pts[miss] = np.nan
        rng = _rng(self.seed, 3, t)
        flick = rng.random(len(r)) < self.flicker
        lab = np.where(flick, rng.integers(0, STREET_CLASSES, len(r)), cls).astype(np.int32)
        return dict(points=pts, pose=pose, label=lab, true_class=cls.astype(np.int32), range=r, dirs=dirs,
                    prim=self._last_prim.astype(np.int32))


    # --- differentiation workload: rays, logits, ground truth, surface samples ---

    def ray_sweep(self, t, true_logit=3.0):
        """Sweep t as (range, unit sensor-frame direction) pairs with 20-class logits:
        the observed (possibly flickered) class gets `true_logit`, the others N(0, 1).
        Misses and returns beyond max_range have range NaN."""
        sw = self.sweep(t)
        r = sw["range"].astype(np.float64)
        r = np.where(r <= self.max_range, r, np.nan).astype(np.float32)
        rng = _rng(self.seed, 5, t)
        logits = rng.normal(0.0, 1.0, size=(len(r), STREET_CLASSES))
        logits[np.arange(len(r)), sw["label"]] = true_logit
        return dict(ranges=r, dirs=sw["dirs"].astype(np.float32), pose=sw["pose"],
                    logits=logits.astype(np.float32), label=sw["label"], true_class=sw["true_class"])

    def nearest_class(self, xyz, margin=2.0):
        """Class of the primitive (ground, box or cylinder) nearest to each point.

        Primitives are tested only against points within `margin` of their
        bounding box; points left farther than `margin` from everything tested
        get a full test."""
        p_all = np.asarray(xyz, np.float64)
        order = np.argsort(p_all[:, 0], kind="stable")
        p = p_all[order]
        xs = p[:, 0]
        best = np.abs(p[:, 2])  # ground plane z = 0
        cls = np.zeros(len(p), np.int64)

        def box_dist(q, lo, hi):
            out = np.linalg.norm(np.maximum(lo - q, 0.0) + np.maximum(q - hi, 0.0), axis=1)
            inside = np.minimum(np.min(q - lo, axis=1), np.min(hi - q, axis=1))
            return np.where(out > 0, out, inside)

        def cyl_dist(q, j):
            dx = np.hypot(q[:, 0] - self.cyl_xy[j, 0], q[:, 1] - self.cyl_xy[j, 1]) - self.cyl_r[j]
            dz = np.maximum(q[:, 2] - self.cyl_h[j], 0.0) + np.maximum(-q[:, 2], 0.0)
            return np.where((dx > 0) | (dz > 0), np.hypot(np.maximum(dx, 0.0), dz),
                            np.minimum(-dx, np.minimum(q[:, 2], self.cyl_h[j] - q[:, 2])))

        def visit(lo, hi, dist, label, full):
            if full:
                sel = np.arange(len(p))
            else:
                a, b = np.searchsorted(xs, [lo[0] - margin, hi[0] + margin])
                sel = np.arange(a, b)
                q = p[sel]
                keep = np.all((q[:, 1:] >= lo[1:] - margin) & (q[:, 1:] <= hi[1:] + margin), axis=1)
                sel = sel[keep]
            if len(sel) == 0:
                return
            d = dist(p[sel])
            closer = d < best[sel]
            best[sel[closer]] = d[closer]
            cls[sel[closer]] = label

        def sweep(full):
            for j in range(len(self.box_lo)):
                lo, hi = self.box_lo[j], self.box_hi[j]
                visit(lo, hi, lambda q: box_dist(q, lo, hi), self.box_class[j], full)
            for j in range(len(self.cyl_r)):
                lo = np.array([self.cyl_xy[j, 0] - self.cyl_r[j], self.cyl_xy[j, 1] - self.cyl_r[j], 0.0])
                hi = np.array([self.cyl_xy[j, 0] + self.cyl_r[j], self.cyl_xy[j, 1] + self.cyl_r[j], self.cyl_h[j]])
                visit(lo, hi, lambda q, j=j: cyl_dist(q, j), self.cyl_class[j], full)

        sweep(False)
        far = best > margin
        if far.any():
            keep_p, keep_xs, keep_best, keep_cls = p, xs, best, cls
            p, xs = keep_p[far], keep_xs[far]
            best, cls = keep_best[far].copy(), keep_cls[far].copy()
            sweep(True)
            keep_best[far], keep_cls[far] = best, cls
            p, xs, best, cls = keep_p, keep_xs, keep_best, keep_cls
        out = np.empty(len(p_all), np.int32)
        out[order] = cls
        return out

    def surface_samples(self, frames, count=10000, seed=5):
        """`count` noiseless hit points (world frame, float32) drawn from the valid
        returns of the given ray sweeps."""
        pts = []
        for fr in frames:
            ok = np.isfinite(fr["ranges"])
            p = fr["dirs"][ok].astype(np.float64) * fr["ranges"][ok, None].astype(np.float64)
            pts.append(p @ fr["pose"][:3, :3].T + fr["pose"][:3, 3])
        pts = np.concatenate(pts)
        idx = _rng(seed, 6).choice(len(pts), size=min(count, len(pts)), replace=False)
        return pts[np.sort(idx)].astype(np.float32)


def primitive_embeddings(scene, prim, L, seed, t, noise=0.1):
    """Open-set embeddings for street points: a random unit prototype per
    primitive plus N(0, noise^2) per component, L2-normalised, bf16 bits."""
    nprim = 1 + len(scene.box_lo) + len(scene.cyl_r)
    proto = _rng(seed, 7).normal(size=(nprim, L)).astype(np.float32)
    proto /= np.linalg.norm(proto, axis=1, keepdims=True)
    z = proto[prim]
    z += _rng(seed, 8, t).standard_normal(z.shape, dtype=np.float32) * np.float32(noise)
    z /= np.linalg.norm(z, axis=1, keepdims=True)
    return to_bf16_bits(z)


def batched_draws(seed=4, nmaps=32, n_lo=10_000, n_hi=130_000):
    """(trajectory index t, ray count n) of each map of the many-map workload."""
    rng = _rng(seed, 9)
    draws = []
    for _ in range(nmaps):
        n = int(rng.integers(n_lo, n_hi + 1))
        t = int(rng.integers(0, 100))
        draws.append((t, n))
    return draws


def batched_workload(seed=4, nmaps=32, n_lo=10_000, n_hi=130_000, closed_maps=16, K=20, L=256, beams=128,
                     workers=1):
    """Many independent maps, one frame each: the first n_i rays (azimuth-major)
    of a 128-beam sweep of the street from a random trajectory pose, n_i uniform
    in [n_lo, n_hi].  Maps below `closed_maps` get int32 labels (K classes), the
    others bf16 embeddings of size L.  Returns a list of dicts (kind, frame)."""
    scene = StreetScene(seed=2, beams=beams)
    draws = batched_draws(seed, nmaps, n_lo, n_hi)
    if workers > 1 and nmaps >= 4:
        import concurrent.futures as cf
        import multiprocessing as mp

        with cf.ProcessPoolExecutor(max_workers=min(workers, nmaps), mp_context=mp.get_context("fork")) as ex:
            sweeps = list(ex.map(scene.sweep, *zip(*draws)))
    else:
        sweeps = [scene.sweep(t, nrays=n) for t, n in draws]
    out = []
    for i, ((t, n), sw) in enumerate(zip(draws, sweeps)):
        item = dict(points=sw["points"], pose=sw["pose"], n=n)
        if i < closed_maps:
            item.update(mode="closed", K=K, label=sw["label"])
        else:
            item.update(mode="open", L=L, emb=primitive_embeddings(scene, sw["prim"], L, seed, t))
        out.append(item)
    return out


# ----------------------------------------------------------------------------
# RGB-D room, open set with bf16 embeddings
# ----------------------------------------------------------------------------


class OpenRoomScene:
    """An 8x8x3 m room with 50 boxes (sides 0.2-1.5 m) standing on the floor, seen by
    a pinhole RGB-D camera on a 2.5 m circle around the room centre at 1.5 m height,
    turning by ``deg_per_frame`` each frame.  56 objects (50 boxes + 6 room faces) each
    have a random unit prototype in R^L; a pixel's embedding is its object's prototype
    plus N(0, noise^2) per component, L2-normalised and rounded to bfloat16."""

    def __init__(self, seed=3, nboxes=50, L=512, width=640, height=480, f=525.0, cx=319.5, cy=239.5,
                 depth_range=(0.3, 5.0), noise=0.1, radius=2.5, cam_height=1.5, deg_per_frame=0.5,
                 room=(8.0, 8.0, 3.0)):
        rng = _rng(seed, 1)
        self.room = np.asarray(room, float)
        centre = self.room[:2] / 2
        lo, hi = [], []
        while len(lo) < nboxes:
            s = rng.uniform(0.2, 1.5, 3)
            c = rng.uniform(s[:2] / 2, self.room[:2] - s[:2] / 2)
            # keep the camera orbit (radius +- 0.4 m) clear of boxes
            corners = np.array([[c[0] + sx * s[0] / 2, c[1] + sy * s[1] / 2] for sx in (-1, 1) for sy in (-1, 1)])
            dist = np.linalg.norm(corners - centre, axis=1)
            near = max(0.0, np.linalg.norm(np.clip(centre, c - s[:2] / 2, c + s[:2] / 2) - centre))
            if not (dist.max() < radius - 0.4 or near > radius + 0.4):
                continue
            lo.append([c[0] - s[0] / 2, c[1] - s[1] / 2, 0.0])
            hi.append([c[0] + s[0] / 2, c[1] + s[1] / 2, s[2]])
        self.box_lo, self.box_hi = np.array(lo), np.array(hi)
        self.L = L
        proto = rng.normal(size=(nboxes + 6, L))
        self.proto = proto / np.linalg.norm(proto, axis=1, keepdims=True)
        self.seed = seed
        self.width, self.height, self.f, self.cx, self.cy = width, height, f, cx, cy
        self.depth_range = depth_range
        self.noise = noise
        self.radius, self.cam_height, self.deg = radius, cam_height, deg_per_frame
        u, v = np.meshgrid(np.arange(width), np.arange(height))
        self.rays_c = np.stack([(u - cx) / f, (v - cy) / f, np.ones_like(u, float)], axis=-1).reshape(-1, 3)

    def pose(self, t):
        ang = np.deg2rad(self.deg * t)
        c = self.room[:2] / 2
        pos = np.array([c[0] + self.radius * np.cos(ang), c[1] + self.radius * np.sin(ang), self.cam_height])
        target = np.array([c[0], c[1], 1.0])
        return pose_matrix(camera_rotation(target - pos), pos)

    def frames(self, ts, workers=8):
        """Several frames with embeddings, generated in worker processes."""
        ts = list(ts)
        if workers <= 1 or len(ts) < 2:
            return [self.frame(t) for t in ts]
        import concurrent.futures as cf
        import multiprocessing as mp

        with cf.ProcessPoolExecutor(max_workers=min(workers, len(ts)), mp_context=mp.get_context("fork")) as ex:
            return list(ex.map(self.frame, ts))

    def frame(self, t, with_embeddings=True):
        pose = self.pose(t)
        R, o = pose[:3, :3], pose[:3, 3]
        dirs = self.rays_c / np.linalg.norm(self.rays_c, axis=1, keepdims=True)
        dw = dirs @ R.T
        tw, face = _ray_box_inside(o, dw, np.zeros(3), self.room)
        tb, ib = _ray_boxes(o, dw, self.box_lo, self.box_hi)
        obj = np.where(tb < tw, ib, len(self.box_lo) + face)
        tt = np.minimum(tb, tw)
        depth = tt * dirs[:, 2]
        ok = (depth >= self.depth_range[0]) & (depth <= self.depth_range[1])
        pts = (self.rays_c * depth[:, None]).astype(np.float32)
        pts[~ok] = np.nan
        # the depth image (z along the optical axis, NaN where invalid)
        dimg = np.where(ok, depth, np.nan).astype(np.float32).reshape(self.height, self.width)
        out = dict(points=pts, pose=pose, obj=obj.astype(np.int32), depth=dimg)
        if with_embeddings:
            # row blocks keep the temporaries small; the normal draws continue
            # one stream across blocks, so the result equals one whole-frame draw
            rng = _rng(self.seed, 4, t)
            proto = self.proto.astype(np.float32)
            emb = np.empty((len(obj), self.L), np.uint16)
            noise = np.float32(self.noise)
            for b in range(0, len(obj), 8192):
                z = proto[obj[b:b + 8192]]
                n = rng.standard_normal(z.shape, dtype=np.float32)
                n *= noise
                z += n
                z /= np.linalg.norm(z, axis=1, keepdims=True)
                emb[b:b + 8192] = to_bf16_bits(z)
            out["emb"] = emb
        return out
