"""The C ABI library loads, exports every function include/slimvdb.h declares,
and rejects bad arguments on the host before touching a GPU."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2512_12945_amd import slimvdb as sv

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "slimvdb.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(slim_[a-z_]+)\s*\(", src)))


def test_header_declares_binding_exports():
    assert set(_declared()) == set(sv.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = sv.load()
    for name in _declared():
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", sv.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (slim_[a-z_]+)", out))
    assert set(_declared()) <= exported


def _cfg(**kw):
    base = dict(voxel_size=0.1, sdf_trunc=0.3, min_range=0.0, max_range=50.0, sem_mode=sv.SEM_CLOSED,
                num_classes=20, embed_dim=0, device=0, max_leaves=1000, max_voxels=100000)
    base.update(kw)
    return sv.MapConfig(*[base[f] for f, _ in sv.MapConfig._fields_])


@pytest.mark.parametrize("bad,code", [
    (dict(voxel_size=0.0), sv.ERR_INVALID),
    (dict(voxel_size=float("nan")), sv.ERR_INVALID),
    (dict(sdf_trunc=0.05), sv.ERR_INVALID),
    (dict(sdf_trunc=0.7), sv.ERR_UNSUPPORTED),
    (dict(min_range=-1.0), sv.ERR_INVALID),
    (dict(max_range=0.0), sv.ERR_INVALID),
    (dict(max_range=float("inf")), sv.ERR_INVALID),
    (dict(sem_mode=7), sv.ERR_INVALID),
    (dict(sem_mode=5), sv.ERR_INVALID),
    (dict(sem_mode=sv.SEM_CLOSED_LAST, num_classes=0), sv.ERR_INVALID),
    (dict(sem_mode=sv.SEM_OPEN_LAST, embed_dim=0), sv.ERR_INVALID),
    (dict(num_classes=0), sv.ERR_INVALID),
    (dict(num_classes=257), sv.ERR_INVALID),
    (dict(sem_mode=sv.SEM_OPEN, embed_dim=0), sv.ERR_INVALID),
    (dict(sem_mode=sv.SEM_OPEN, embed_dim=2000), sv.ERR_INVALID),
    (dict(max_leaves=0), sv.ERR_INVALID),
    (dict(max_voxels=1 << 31), sv.ERR_INVALID),
    (dict(device=-1), sv.ERR_INVALID),
])
def test_create_rejects_bad_config(bad, code):
    L = sv.load()
    h = ctypes.c_void_p()
    cfg = _cfg(**bad)
    assert L.slim_map_create(ctypes.byref(cfg), ctypes.byref(h)) == code
    assert h.value is None
    assert L.slim_last_error()


def test_null_arguments():
    L = sv.load()
    assert L.slim_map_create(None, None) == sv.ERR_INVALID
    assert L.slim_integrate(None, None, 0, None, None, 0, None) == sv.ERR_INVALID
    assert L.slim_map_stats(None, None, None) == sv.ERR_INVALID
    cnt = ctypes.c_int64()
    assert L.slim_extract(None, 0, None, None, None, None, ctypes.byref(cnt), None) == sv.ERR_INVALID
    assert L.slim_extract_noalloc(None, 0, None, None, None, None, ctypes.byref(cnt), None) == sv.ERR_INVALID
    assert L.slim_query(None, None, 0, None, None, None, None) == sv.ERR_INVALID
    assert L.slim_profile_enable(None, 1) == sv.ERR_INVALID
    cnt32 = ctypes.c_int32()
    assert L.slim_profile_sets(None, 0, None, None, None, ctypes.byref(cnt32), None) == sv.ERR_INVALID
    assert L.slim_map_destroy(None) == sv.OK


def test_read_out_and_depth_entry_points_reject_null_map():
    L = sv.load()
    pp = sv.PredictParams(1.0, 1.0, 0.0, 0, None)
    assert L.slim_predict(None, None, 0, ctypes.byref(pp), None, None, None, None) == sv.ERR_INVALID
    k = (ctypes.c_float * 4)(1.0, 1.0, 0.0, 0.0)
    assert L.slim_integrate_depth(None, None, 0, 0, k, None, None, 0, None) == sv.ERR_INVALID
    assert L.slim_render(None, None, k, 0, 0, 0.0, 1.0, None, None, None, None) == sv.ERR_INVALID
    assert L.slim_integrate_sequence(None, None, 0, None) == sv.ERR_INVALID


def test_differentiation_entry_points_reject_bad_arguments():
    L = sv.load()
    assert L.slim_integrate_rays(None, None, None, 0, None, None, 0, None) == sv.ERR_INVALID
    assert L.slim_map_loss(None, None, None, 0, None, 0, 1.0, None, None) == sv.ERR_INVALID
    assert L.slim_backward_rays(None, None, None, 0, None, None, None, None, None, None) == sv.ERR_INVALID
