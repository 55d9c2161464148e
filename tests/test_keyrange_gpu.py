"""The voxel key range |k| < 2^20 on the GPU against the oracle: points whose
band walk leaves the range are rejected one by one (and counted), a sensor
origin 2^20 or more voxels out is anchored at +2^20 exactly as the oracle
anchors it, and a map's max_range is not bounded by the key range."""
import sys

import numpy as np
import pytest
import torch

from paper_2512_12945_amd import slimvdb as sv

from _gpu_util import assert_stats_equal, compare_maps, extract_np, integrate_both, make_pair

pytestmark = pytest.mark.gpu

VS, TAU, LIM = 0.1, 0.3, 1 << 20


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sv.load()


def _fan(rng, n, reach):
    """n sensor-frame points spread over +-reach metres along x, a little in y, z."""
    pts = np.stack([rng.uniform(-reach, reach, n), rng.uniform(-1.0, 1.0, n), rng.uniform(-0.5, 0.5, n)], 1)
    return pts.astype(np.float32)


@pytest.mark.parametrize("origin_voxels", [LIM - 12.5, -(LIM - 12.5), LIM + 30.5, -(LIM + 40.5), 3e9])
def test_bands_crossing_the_key_range(origin_voxels):
    """Origins near +-2^20 voxels: the rays towards the boundary leave the
    range and are rejected; origins beyond it are anchored at +2^20, where only
    points that walk back into range are kept."""
    rng = np.random.default_rng(int(abs(origin_voxels)) % 1000)
    g, o = make_pair(VS, TAU, 0.0, 1000.0, sv.SEM_CLOSED, K=4)
    pose = np.eye(4)
    pose[:3, 3] = (origin_voxels * np.float64(np.float32(VS)), 0.25, -0.15)
    pts = _fan(rng, 4096, 12.0)
    lab = rng.integers(0, 4, len(pts)).astype(np.int32)
    gst, ost = integrate_both(g, o, pts, pose, lab, sv.IN_LABEL_I32)
    _say(f"origin {origin_voxels} voxels: {ost['rejected']} of {len(pts)} rejected, {ost['pairs']} pairs")
    assert_stats_equal(gst, ost)
    if abs(origin_voxels) < 2 * LIM:
        assert 0 < ost["rejected"] < len(pts)
    else:
        assert ost["rejected"] == len(pts)
    compare_maps(extract_np(g), o.extract(), TAU, sv.SEM_CLOSED, K=4, exact_counts=True)


def test_max_range_beyond_the_key_range():
    """max_range is a range gate only: a map may set it beyond 2^19 voxel
    sizes; points within it integrate as usual."""
    rng = np.random.default_rng(5)
    g, o = make_pair(VS, TAU, 0.0, 1.0e6, sv.SEM_NONE)
    pts = _fan(rng, 2000, 30.0)
    gst, ost = integrate_both(g, o, pts, np.eye(4))
    assert_stats_equal(gst, ost)
    assert ost["rejected"] == 0
    compare_maps(extract_np(g), o.extract(), TAU, sv.SEM_NONE)
