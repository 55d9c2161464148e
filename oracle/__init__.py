"""Plain FP64 CPU oracle for SLIM-VDB's per-frame integration (arXiv 2512.12945).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product library
(``paper_2512_12945_amd``) never imports, links or calls it, and it shares no
code with the HIP path.

The arithmetic lives in ``slim_oracle.c`` (plain C11, gcc, ``-ffp-contract=off``);
this module is a ctypes wrapper plus the FP64 map loss of the differentiation
workload (``loss.py``).  What each function computes, and the paper passage it
follows, is stated in the C source.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "slim_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

SEM_NONE, SEM_CLOSED, SEM_OPEN, SEM_CLOSED_LAST, SEM_OPEN_LAST = 0, 1, 2, 3, 4
IN_NONE, IN_LABEL_I32, IN_PROB_F32, IN_LOGIT_F32, IN_EMB_BF16, IN_EMB_F32 = range(6)

GCC_FLAGS = ["-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-Wall"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/liboracle.so``."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *GCC_FLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        vp, i64, f32, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_float, ctypes.c_int
        L.om_create.restype = vp
        L.om_create.argtypes = [f32, f32, f32, f32, i32, i32, i32]
        L.om_destroy.argtypes = [vp]
        L.om_maxsteps.argtypes = [vp]
        L.om_maxsteps.restype = i32
        L.om_ray_visits.argtypes = [f32, f32, vp, vp, vp, i32]
        L.om_ray_visits.restype = i32
        L.om_frame_pairs.argtypes = [vp, vp, i64, vp, vp, i32, vp, vp, vp, vp, i64, vp]
        L.om_frame_pairs.restype = i64
        L.om_apply.argtypes = [vp, i64, vp, vp, vp, vp, i32, i32]
        L.om_depth_points.argtypes = [vp, i32, i32, f32, f32, f32, f32, vp]
        L.om_render.argtypes = [vp, vp, f32, f32, f32, f32, i32, i32, f32, f32, vp, vp, vp, vp]
        L.om_render.restype = None
        L.om_depth_points.restype = None
        L.om_apply.restype = i32
        L.om_integrate.argtypes = [vp, vp, i64, vp, vp, i32, i32]
        L.om_integrate.restype = i32
        L.om_count.argtypes = [vp]
        L.om_count.restype = i64
        L.om_leaf_count.argtypes = [vp]
        L.om_leaf_count.restype = i64
        L.om_stats.argtypes = [vp, vp]
        L.om_extract.argtypes = [vp, vp, vp, vp, vp, i64]
        L.om_extract.restype = i64
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _sem_array(sem, kind):
    if kind == IN_NONE or sem is None:
        return None
    if kind == IN_LABEL_I32:
        return np.ascontiguousarray(sem, dtype=np.int32)
    if kind == IN_EMB_BF16:
        return np.ascontiguousarray(sem, dtype=np.uint16)
    return np.ascontiguousarray(sem, dtype=np.float32)


class OracleMap:
    """A sparse voxel map in FP64, keyed by integer voxel coordinates."""

    def __init__(self, voxel_size, sdf_trunc, min_range=0.0, max_range=1e30, sem_mode=SEM_NONE,
                 num_classes=0, embed_dim=0):
        self._L = lib()
        self.h = self._L.om_create(voxel_size, sdf_trunc, min_range, max_range, sem_mode, num_classes, embed_dim)
        if not self.h:
            raise ValueError("invalid oracle map configuration")
        self.voxel_size = float(np.float32(voxel_size))
        self.sdf_trunc = float(np.float32(sdf_trunc))
        self.sem_mode = sem_mode
        self.K = num_classes
        self.L = embed_dim
        self.nsem = {SEM_CLOSED: num_classes, SEM_OPEN: 2 * embed_dim, SEM_CLOSED_LAST: 1,
                     SEM_OPEN_LAST: embed_dim}.get(sem_mode, 0)
        self.maxsteps = self._L.om_maxsteps(self.h)

    def __del__(self):
        if getattr(self, "h", None):
            self._L.om_destroy(self.h)
            self.h = None

    def frame_pairs(self, pts, pose, sem=None, kind=IN_NONE):
        """All kept (voxel, point) observations of one frame, in point order."""
        pts = np.ascontiguousarray(pts, dtype=np.float32).reshape(-1, 3)
        pose = np.ascontiguousarray(pose, dtype=np.float64).reshape(16)
        s = _sem_array(sem, kind)
        n = pts.shape[0]
        rej = np.zeros(1, np.int64)
        P = self._L.om_frame_pairs(self.h, _ptr(pts), n, _ptr(pose), _ptr(s), kind, None, None, None, None, 0,
                                   _ptr(rej))
        keys = np.zeros((max(P, 1), 3), np.int32)
        pid = np.zeros(max(P, 1), np.uint32)
        tsdf = np.zeros(max(P, 1), np.float64)
        s32 = np.zeros(max(P, 1), np.float32)
        self._L.om_frame_pairs(self.h, _ptr(pts), n, _ptr(pose), _ptr(s), kind, _ptr(keys), _ptr(pid), _ptr(tsdf),
                               _ptr(s32), P, _ptr(rej))
        return dict(keys=keys[:P], pid=pid[:P], tsdf=tsdf[:P], sdf32=s32[:P], rejected=int(rej[0]))

    def apply(self, keys, pid, tsdf, sem=None, kind=IN_NONE, mode=0):
        keys = np.ascontiguousarray(keys, dtype=np.int32).reshape(-1, 3)
        pid = np.ascontiguousarray(pid, dtype=np.uint32)
        tsdf = np.ascontiguousarray(tsdf, dtype=np.float64)
        s = _sem_array(sem, kind)
        rc = self._L.om_apply(self.h, keys.shape[0], _ptr(keys), _ptr(pid), _ptr(tsdf), _ptr(s), kind, mode)
        if rc:
            raise MemoryError("oracle apply failed")

    def integrate(self, pts, pose, sem=None, kind=IN_NONE, mode=0):
        pts = np.ascontiguousarray(pts, dtype=np.float32).reshape(-1, 3)
        pose = np.ascontiguousarray(pose, dtype=np.float64).reshape(16)
        s = _sem_array(sem, kind)
        rc = self._L.om_integrate(self.h, _ptr(pts), pts.shape[0], _ptr(pose), _ptr(s), kind, mode)
        if rc:
            raise MemoryError("oracle integrate failed")
        return self.stats()

    def stats(self):
        out = np.zeros(8, np.int64)
        self._L.om_stats(self.h, _ptr(out))
        names = ["points", "rejected", "pairs", "u_old", "u_new", "new_leaves", "voxels", "leaves"]
        return {k: int(v) for k, v in zip(names, out)}

    def count(self):
        return int(self._L.om_count(self.h))

    def leaf_count(self):
        return int(self._L.om_leaf_count(self.h))

    def extract(self):
        """Every voxel with W > 0, ordered by leaf coordinate then in-leaf offset."""
        M = self.count()
        keys = np.zeros((max(M, 1), 3), np.int32)
        D = np.zeros(max(M, 1), np.float64)
        W = np.zeros(max(M, 1), np.float64)
        sem = np.zeros((max(M, 1), max(self.nsem, 1)), np.float64)
        self._L.om_extract(self.h, _ptr(keys), _ptr(D), _ptr(W), _ptr(sem) if self.nsem else None, M)
        return dict(keys=keys[:M], D=D[:M], W=W[:M], sem=sem[:M, : self.nsem])


def render(omap, pose, fx, fy, cx, cy, width, height, near, far):
    """First surface per pixel (see om_render in slim_oracle.c): depth (H, W) FP64 (NaN: none),
    key (H, W, 3) of the cell behind the surface, label (H, W), margin (H, W)."""
    pose = np.ascontiguousarray(pose, dtype=np.float64).reshape(16)
    n = width * height
    depth = np.zeros(n, np.float64)
    key = np.zeros((n, 3), np.int32)
    label = np.zeros(n, np.int32)
    margin = np.zeros(n, np.float64)
    lib().om_render(omap.h, _ptr(pose), fx, fy, cx, cy, width, height, near, far, _ptr(depth), _ptr(key),
                    _ptr(label), _ptr(margin))
    return dict(depth=depth.reshape(height, width), key=key.reshape(height, width, 3),
                label=label.reshape(height, width), margin=margin.reshape(height, width))


def depth_points(depth, fx, fy, cx, cy):
    """Sensor-frame points (H*W, 3) of a depth image (H, W), binary32 back-projection."""
    d = np.ascontiguousarray(depth, dtype=np.float32)
    H, W = d.shape
    pts = np.zeros((H * W, 3), np.float32)
    lib().om_depth_points(_ptr(d), W, H, ctypes.c_float(fx), ctypes.c_float(fy), ctypes.c_float(cx),
                          ctypes.c_float(cy), _ptr(pts))
    return pts


def ray_visits(voxel_size, sdf_trunc, origin, point, cap=4096):
    """Cells of the band walk of one ray (coordinates relative to the anchor), pre-gate."""
    o = np.ascontiguousarray(origin, dtype=np.float32)
    p = np.ascontiguousarray(point, dtype=np.float32)
    cells = np.zeros((cap, 3), np.int32)
    n = lib().om_ray_visits(voxel_size, sdf_trunc, _ptr(o), _ptr(p), _ptr(cells), cap)
    return cells[:n]
