"""GPU test of slim_extract_noalloc (the allocation-free variant of
slim_extract), called through the C ABI: its output equals slim_extract's bit
for bit on two calls in a row, the second on a map with fewer leaves, so stale
scratch contents of the first call cannot leak into the second."""
import ctypes
import sys

import numpy as np
import pytest
import torch

from paper_2512_12945_amd import slimvdb as sv
from paper_2512_12945_amd import synth

from _gpu_util import cuda

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sv.load()


def _np(ex):
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in ex.items()}


def _same(a, b):
    for k in ("keys", "D", "W", "sem"):
        assert a[k].shape == b[k].shape, k
        assert np.array_equal(a[k].view(np.uint32) if a[k].dtype == np.float32 else a[k],
                              b[k].view(np.uint32) if b[k].dtype == np.float32 else b[k]), k


def _lidar_map():
    sc = synth.StreetScene(seed=2)
    g = sv.Map(0.1, 0.3, 0.0, 50.0, sv.SEM_CLOSED, 20, 0, 0, 1 << 18, 1 << 24)
    for t in (0, 1, 2):
        sw = sc.sweep(t)
        g.integrate(cuda(sw["points"]), sw["pose"], cuda(sw["label"]), sv.IN_LABEL_I32)
    return g


def _room_map():
    fr = synth.room_frame(seed=1)
    g = sv.Map(0.05, 0.15, 0.0, 100.0, sv.SEM_CLOSED, 5, 0, 0, 1 << 12, 1 << 18)
    g.integrate(cuda(fr["points"]), fr["pose"], cuda(fr["prob"]), sv.IN_PROB_F32)
    return g


def test_noalloc_extract_equals_extract_twice_shrinking():
    big = _lidar_map()
    small = _room_map()
    sb, ss = big.stats(), small.stats()
    _say(f"lidar map {sb['leaves']} leaves / {sb['voxels']} voxels; room map {ss['leaves']} / {ss['voxels']}")
    assert ss["leaves"] < sb["leaves"] and ss["voxels"] < sb["voxels"]
    # the allocation-free call first on the larger map, then on the smaller one
    nb = _np(big.extract(noalloc=True))
    ns = _np(small.extract(noalloc=True))
    _same(nb, _np(big.extract()))
    _same(ns, _np(small.extract()))
    assert nb["keys"].shape[0] == sb["voxels"] and ns["keys"].shape[0] == ss["voxels"]
    # and again on the larger map after the smaller one
    _same(_np(big.extract(noalloc=True)), nb)


def test_noalloc_extract_count_capacity_and_empty_map():
    L = sv.load()
    g = _room_map()
    cnt = ctypes.c_int64(-1)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.slim_extract_noalloc(g.h, 0, None, None, None, None, ctypes.byref(cnt), s) == sv.OK
    M = cnt.value
    assert M == g.stats()["voxels"] > 0
    keys = torch.empty((M, 3), dtype=torch.int32, device="cuda")
    d = torch.empty(M, dtype=torch.float32, device="cuda")
    w = torch.empty(M, dtype=torch.float32, device="cuda")
    # capacity below the voxel count is refused before anything is written
    assert L.slim_extract_noalloc(g.h, M - 1, keys.data_ptr(), d.data_ptr(), w.data_ptr(), None,
                                  ctypes.byref(cnt), s) == sv.ERR_INVALID
    assert b"capacity" in L.slim_last_error()
    # an empty map exports nothing
    e = sv.Map(0.05, 0.15, 0.0, 100.0, sv.SEM_CLOSED, 5, 0, 0, 1 << 12, 1 << 18)
    ex = _np(e.extract(noalloc=True))
    assert ex["keys"].shape == (0, 3) and ex["D"].shape == (0,)
