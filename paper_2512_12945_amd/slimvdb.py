"""Python binding of libslimvdb (include/slimvdb.h): argument marshalling only.

Every step of integration, extraction and lookup runs in the library's HIP
kernels.  torch provides device memory and the current stream; nothing here
computes on the data.  If the library is not built, using this module raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libslimvdb.so")

OK, ERR_INVALID, ERR_CAPACITY, ERR_DEVICE, ERR_UNSUPPORTED = 0, -1, -2, -3, -4
SEM_NONE, SEM_CLOSED, SEM_OPEN, SEM_CLOSED_LAST, SEM_OPEN_LAST = 0, 1, 2, 3, 4
IN_NONE, IN_LABEL_I32, IN_PROB_F32, IN_LOGIT_F32, IN_EMB_BF16, IN_EMB_F32 = range(6)
KERNELS = ("ray_walk_emit", "leaf_plan", "pair_bucket", "leaf_fuse", "voxel_combine", "frame_commit")

EXPORTS = ("slim_map_create", "slim_map_destroy", "slim_map_reset", "slim_integrate", "slim_integrate_rays",
           "slim_integrate_depth",
           "slim_map_stats", "slim_extract", "slim_extract_noalloc", "slim_query", "slim_predict", "slim_render", "slim_map_loss",
           "slim_backward_rays",
           "slim_integrate_batched", "slim_integrate_sequence", "slim_set_launch_shape", "slim_profile_enable",
           "slim_profile_read", "slim_profile_sets",
           "slim_last_error")


class PredictParams(ctypes.Structure):
    _fields_ = [("alpha0", ctypes.c_float), ("temperature", ctypes.c_float), ("threshold", ctypes.c_float),
                ("num_prototypes", ctypes.c_int32), ("prototypes_dev", ctypes.c_void_p)]


class MapConfig(ctypes.Structure):
    _fields_ = [("voxel_size", ctypes.c_float), ("sdf_trunc", ctypes.c_float), ("min_range", ctypes.c_float),
                ("max_range", ctypes.c_float), ("sem_mode", ctypes.c_int32), ("num_classes", ctypes.c_int32),
                ("embed_dim", ctypes.c_int32), ("device", ctypes.c_int32), ("max_leaves", ctypes.c_int64),
                ("max_voxels", ctypes.c_int64)]


class Stats(ctypes.Structure):
    _fields_ = [("leaves", ctypes.c_int64), ("voxels", ctypes.c_int64), ("points_last", ctypes.c_int64),
                ("rejected_last", ctypes.c_int64), ("pairs_last", ctypes.c_int64),
                ("touched_leaves_last", ctypes.c_int64), ("new_leaves_last", ctypes.c_int64),
                ("voxels_old_last", ctypes.c_int64), ("voxels_new_last", ctypes.c_int64),
                ("status_last", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class Frame(ctypes.Structure):
    _fields_ = [("points", ctypes.c_void_p), ("ranges", ctypes.c_void_p), ("dirs", ctypes.c_void_p),
                ("n", ctypes.c_int64), ("pose", ctypes.c_double * 16), ("sem", ctypes.c_void_p),
                ("sem_kind", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class LaunchShape(ctypes.Structure):
    _fields_ = [("plan_blocks", ctypes.c_int32), ("bucket_blocks", ctypes.c_int32),
                ("leaf_blocks_per_cu", ctypes.c_int32), ("pass_frames", ctypes.c_int32),
                ("batch_mode", ctypes.c_int32), ("walk_chunk", ctypes.c_int32),
                ("wave_pairs", ctypes.c_int32), ("slab_pairs", ctypes.c_int32)]


class SlimError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"slimvdb error {code}: {msg}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Loads libslimvdb.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with `python -m paper_2512_12945_amd.build`")
        L = ctypes.CDLL(path)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        L.slim_map_create.argtypes = [ctypes.POINTER(MapConfig), ctypes.POINTER(vp)]
        L.slim_map_destroy.argtypes = [vp]
        L.slim_map_reset.argtypes = [vp, vp]
        L.slim_integrate.argtypes = [vp, vp, i64, vp, vp, i32, vp]
        L.slim_integrate_rays.argtypes = [vp, vp, vp, i64, vp, vp, i32, vp]
        L.slim_integrate_depth.argtypes = [vp, vp, i32, i32, vp, vp, vp, i32, vp]
        L.slim_map_loss.argtypes = [vp, vp, vp, i64, vp, i64, ctypes.c_float, vp, vp]
        L.slim_backward_rays.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp, vp, vp]
        L.slim_map_stats.argtypes = [vp, ctypes.POINTER(Stats), vp]
        L.slim_extract.argtypes = [vp, i64, vp, vp, vp, vp, ctypes.POINTER(i64), vp]
        L.slim_extract_noalloc.argtypes = [vp, i64, vp, vp, vp, vp, ctypes.POINTER(i64), vp]
        L.slim_query.argtypes = [vp, vp, i64, vp, vp, vp, vp]
        L.slim_predict.argtypes = [vp, vp, i64, ctypes.POINTER(PredictParams), vp, vp, vp, vp]
        L.slim_render.argtypes = [vp, vp, vp, i32, i32, ctypes.c_float, ctypes.c_float, vp, vp, vp, vp]
        L.slim_integrate_batched.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(Frame), i32, vp]
        L.slim_integrate_sequence.argtypes = [vp, ctypes.POINTER(Frame), i32, vp]
        L.slim_set_launch_shape.argtypes = [vp, ctypes.POINTER(LaunchShape)]
        L.slim_profile_enable.argtypes = [vp, i32]
        L.slim_profile_read.argtypes = [vp, vp, vp, i32, vp]
        L.slim_profile_sets.argtypes = [vp, i32, vp, vp, vp, ctypes.POINTER(i32), vp]
        L.slim_last_error.restype = ctypes.c_char_p
        for f in EXPORTS[:-1]:
            getattr(L, f).restype = i32
        _lib = L
    return _lib


def _check(code):
    if code != OK:
        raise SlimError(code, _lib.slim_last_error().decode())


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else None


class Map:
    """A sparse semantic TSDF map living on one GPU (see include/slimvdb.h)."""

    def __init__(self, voxel_size, sdf_trunc, min_range=0.0, max_range=100.0, sem_mode=SEM_NONE, num_classes=0,
                 embed_dim=0, device=0, max_leaves=1 << 18, max_voxels=1 << 24):
        self._L = load()
        self.device = torch.device("cuda", device)
        self.cfg = MapConfig(voxel_size, sdf_trunc, min_range, max_range, sem_mode, num_classes, embed_dim, device,
                             max_leaves, max_voxels)
        self.sem_mode = sem_mode
        self.nsem = {SEM_CLOSED: num_classes, SEM_OPEN: 2 * embed_dim, SEM_CLOSED_LAST: 1,
                     SEM_OPEN_LAST: embed_dim}.get(sem_mode, 0)
        h = ctypes.c_void_p()
        _check(self._L.slim_map_create(ctypes.byref(self.cfg), ctypes.byref(h)))
        self.h = h
        self._pose = np.zeros(16, np.float64)

    def close(self):
        if getattr(self, "h", None):
            self._L.slim_map_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def reset(self):
        _check(self._L.slim_map_reset(self.h, _stream(self.device)))

    def integrate(self, points, pose, sem=None, kind=IN_NONE):
        """points: (N, 3) float32 cuda tensor; pose: 4x4 map_T_sensor; sem: cuda tensor in `kind` layout."""
        self._pose[:] = np.asarray(pose, np.float64).reshape(16)
        n = points.shape[0] if points is not None else 0
        _check(self._L.slim_integrate(self.h, _ptr(points), n, self._pose.ctypes.data_as(ctypes.c_void_p),
                                      _ptr(sem), kind, _stream(self.device)))

    def integrate_rays(self, ranges, dirs, pose, sem=None, kind=IN_NONE):
        """ranges: (N,) float32; dirs: (N, 3) float32 unit sensor-frame directions (cuda tensors)."""
        self._pose[:] = np.asarray(pose, np.float64).reshape(16)
        n = ranges.shape[0]
        _check(self._L.slim_integrate_rays(self.h, _ptr(ranges), _ptr(dirs), n,
                                           self._pose.ctypes.data_as(ctypes.c_void_p), _ptr(sem), kind,
                                           _stream(self.device)))

    def integrate_depth(self, depth, intrinsics, pose, sem=None, kind=IN_NONE):
        """depth: (H, W) float32 cuda tensor (metres along the optical axis); intrinsics: (fx, fy, cx, cy)."""
        self._pose[:] = np.asarray(pose, np.float64).reshape(16)
        H, W = depth.shape
        k = (ctypes.c_float * 4)(*[float(v) for v in intrinsics])
        _check(self._L.slim_integrate_depth(self.h, _ptr(depth), W, H, k, self._pose.ctypes.data_as(ctypes.c_void_p),
                                            _ptr(sem), kind, _stream(self.device)))

    def loss(self, keys, labels, samples, alpha0=1.0, out=None):
        """Map loss (see include/slimvdb.h); returns a (3,) cuda tensor (total, ce, l1)."""
        out = torch.empty(3, dtype=torch.float32, device=self.device) if out is None else out
        _check(self._L.slim_map_loss(self.h, _ptr(keys), _ptr(labels), keys.shape[0], _ptr(samples),
                                     samples.shape[0], float(alpha0), _ptr(out), _stream(self.device)))
        return out

    def predict(self, xyz, alpha0=1.0, temperature=1.0, threshold=0.0, prototypes=None, prob=True, var=False):
        """Semantic read-out at world points xyz (m, 3) (see slim_predict in include/slimvdb.h): returns
        dict(prob=(m, C) or None, label=(m,) int32, var=(m, L) or None) as cuda tensors."""
        m = xyz.shape[0]
        open_set = self.cfg.sem_mode in (SEM_OPEN, SEM_OPEN_LAST)
        C = prototypes.shape[0] if open_set else self.cfg.num_classes
        pp = PredictParams(alpha0, temperature, threshold, C if open_set else 0,
                           _ptr(prototypes) if open_set else None)
        out_p = torch.empty((max(m, 1), C), dtype=torch.float32, device=self.device) if prob else None
        out_l = torch.empty(max(m, 1), dtype=torch.int32, device=self.device)
        out_v = torch.empty((max(m, 1), max(self.cfg.embed_dim, 1)), dtype=torch.float32,
                            device=self.device) if var else None
        _check(self._L.slim_predict(self.h, _ptr(xyz), m, ctypes.byref(pp), _ptr(out_p), _ptr(out_l), _ptr(out_v),
                                    _stream(self.device)))
        return dict(prob=None if out_p is None else out_p[:m], label=out_l[:m],
                    var=None if out_v is None else out_v[:m])

    def render(self, pose, intrinsics, width, height, near, far, keys=True, labels=True):
        """First surface per pixel (see slim_render in include/slimvdb.h): dict(depth (H, W), key (H, W, 3)
        or None, label (H, W) or None) as cuda tensors."""
        pose = np.ascontiguousarray(pose, np.float64).reshape(16)
        k = (ctypes.c_float * 4)(*[float(v) for v in intrinsics])
        depth = torch.empty((height, width), dtype=torch.float32, device=self.device)
        key = torch.empty((height, width, 3), dtype=torch.int32, device=self.device) if keys else None
        lab = torch.empty((height, width), dtype=torch.int32, device=self.device) if labels else None
        _check(self._L.slim_render(self.h, pose.ctypes.data_as(ctypes.c_void_p), k, width, height, float(near),
                                   float(far), _ptr(depth), _ptr(key), _ptr(lab), _stream(self.device)))
        return dict(depth=depth, key=key, label=lab)

    def backward_rays(self, ranges, dirs, pose, logits, grad_logits, grad_ranges, grad_scale=None):
        self._pose[:] = np.asarray(pose, np.float64).reshape(16)
        _check(self._L.slim_backward_rays(self.h, _ptr(ranges), _ptr(dirs), ranges.shape[0],
                                          self._pose.ctypes.data_as(ctypes.c_void_p), _ptr(logits),
                                          _ptr(grad_scale), _ptr(grad_logits), _ptr(grad_ranges),
                                          _stream(self.device)))

    def stats(self):
        st = Stats()
        _check(self._L.slim_map_stats(self.h, ctypes.byref(st), _stream(self.device)))
        return st.as_dict()

    def extract(self, noalloc=False):
        """All voxels with W > 0 as cuda tensors: keys (M, 3) int32, D, W (M,), sem (M, S).
        noalloc: through slim_extract_noalloc (the library allocates nothing;
        the output tensors are still allocated here, by torch)."""
        fn = self._L.slim_extract_noalloc if noalloc else self._L.slim_extract
        cnt = ctypes.c_int64()
        s = _stream(self.device)
        _check(fn(self.h, 0, None, None, None, None, ctypes.byref(cnt), s))
        M = cnt.value
        keys = torch.empty((max(M, 1), 3), dtype=torch.int32, device=self.device)
        d = torch.empty(max(M, 1), dtype=torch.float32, device=self.device)
        w = torch.empty(max(M, 1), dtype=torch.float32, device=self.device)
        sem = torch.empty((max(M, 1), max(self.nsem, 1)), dtype=torch.float32, device=self.device)
        _check(fn(self.h, max(M, 1), _ptr(keys), _ptr(d), _ptr(w), _ptr(sem) if self.nsem else None,
                  ctypes.byref(cnt), s))
        M = cnt.value
        return dict(keys=keys[:M], D=d[:M], W=w[:M], sem=sem[:M, : self.nsem])

    def query(self, xyz):
        m = xyz.shape[0]
        d = torch.empty(max(m, 1), dtype=torch.float32, device=self.device)
        w = torch.empty(max(m, 1), dtype=torch.float32, device=self.device)
        sem = torch.empty((max(m, 1), max(self.nsem, 1)), dtype=torch.float32, device=self.device)
        _check(self._L.slim_query(self.h, _ptr(xyz), m, _ptr(d), _ptr(w), _ptr(sem) if self.nsem else None,
                                  _stream(self.device)))
        return dict(D=d[:m], W=w[:m], sem=sem[:m, : self.nsem])

    def set_launch_shape(self, plan_blocks=None, bucket_blocks=None, leaf_blocks_per_cu=None, pass_frames=0,
                         batch_mode=0, walk_chunk=0, wave_pairs=0, slab_pairs=0):
        """Grid sizes of the grid-stride kernels (in a persistent batched launch:
        items of each stage), the frames integrate_sequence takes in one pass
        (0: the default, 1: one at a time), the batched form (0 default, 1
        persistent, 2 one launch per stage), the ray-chunk size in 256-ray
        blocks and the leaf-tile thresholds (see slim_launch_shape); all None /
        0 restores the defaults, grid sizes left None take their defaults."""
        if (plan_blocks is None and bucket_blocks is None and leaf_blocks_per_cu is None and not pass_frames
                and not batch_mode and not walk_chunk and not wave_pairs and not slab_pairs):
            _check(self._L.slim_set_launch_shape(self.h, None))
        else:
            cus = torch.cuda.get_device_properties(self.device).multi_processor_count
            sh = LaunchShape(cus if plan_blocks is None else plan_blocks,
                             16 * cus if bucket_blocks is None else bucket_blocks,
                             16 if leaf_blocks_per_cu is None else leaf_blocks_per_cu, int(pass_frames),
                             int(batch_mode), int(walk_chunk), int(wave_pairs), int(slab_pairs))
            _check(self._L.slim_set_launch_shape(self.h, ctypes.byref(sh)))

    def profile(self, enable=True):
        _check(self._L.slim_profile_enable(self.h, 1 if enable else 0))

    def profile_sets(self, capacity=1 << 16):
        """Per launch set since the last call: list of (frames, {kernel: ms}, span_ms)."""
        fr = np.zeros(capacity, np.int32)
        ms = np.zeros((capacity, len(KERNELS)), np.float64)
        sp = np.zeros(capacity, np.float64)
        cnt = ctypes.c_int32()
        _check(self._L.slim_profile_sets(self.h, capacity, fr.ctypes.data_as(ctypes.c_void_p),
                                         ms.ctypes.data_as(ctypes.c_void_p), sp.ctypes.data_as(ctypes.c_void_p),
                                         ctypes.byref(cnt), _stream(self.device)))
        n = min(cnt.value, capacity)
        return [(int(fr[i]), dict(zip(KERNELS, ms[i].tolist())), float(sp[i])) for i in range(n)]

    def profile_read(self):
        ms = np.zeros(len(KERNELS), np.float64)
        n = np.zeros(len(KERNELS), np.int64)
        _check(self._L.slim_profile_read(self.h, ms.ctypes.data_as(ctypes.c_void_p),
                                         n.ctypes.data_as(ctypes.c_void_p), len(KERNELS), _stream(self.device)))
        return {k: (float(a), int(b)) for k, a, b in zip(KERNELS, ms, n)}


def _frames(frames):
    arr = (Frame * len(frames))()
    for i, f in enumerate(frames):
        pts = f.get("points")
        arr[i].points = pts.data_ptr() if pts is not None else None
        arr[i].ranges = f["ranges"].data_ptr() if f.get("ranges") is not None else None
        arr[i].dirs = f["dirs"].data_ptr() if f.get("dirs") is not None else None
        arr[i].n = (pts if pts is not None else f["ranges"]).shape[0]
        arr[i].pose[:] = [float(v) for v in np.asarray(f["pose"], np.float64).reshape(16)]
        arr[i].sem = f["sem"].data_ptr() if f.get("sem") is not None else None
        arr[i].sem_kind = f.get("kind", IN_NONE)
    return arr


def integrate_sequence(m, frames):
    """Integrates frames (dicts as for integrate_batched) into map m in order, the ray walk of each next
    frame overlapping the rest of the current one (see include/slimvdb.h)."""
    arr = _frames(frames)
    _check(m._L.slim_integrate_sequence(m.h, arr, len(frames), _stream(m.device)))


def integrate_batched(maps, frames, use_graph=False):
    """frames[i] = dict(points=cuda (n,3) | ranges=..., dirs=..., pose=4x4, sem=cuda tensor, kind=IN_*)
    integrated into maps[i], all in one batched launch sequence (see include/slimvdb.h)."""
    L = load()
    n = len(maps)
    arr = _frames(frames)
    handles = (ctypes.c_void_p * n)(*[m.h.value for m in maps])
    _check(L.slim_integrate_batched(handles, n, arr, 1 if use_graph else 0, _stream(maps[0].device)))
