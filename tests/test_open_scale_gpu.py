"""Open-set parity at the sizes the open-set workloads run (Thm. 2 / Eqs.
(11)-(14) with lambda = 2 nu = W, Sec. III-D): the HIP path through the C ABI
against the FP64 oracle, element by element.

Each test first counts, with the oracle, the largest number of observations in
one voxel, of pairs in one leaf and of pairs in one x-slab of a leaf, and
asserts that they pass the sizes at which the kernels change path: more than
64 observations in a voxel (the wave combines load point indices 64 at a
time), more than 2048 pairs in a leaf (a leaf then splits into x-slab items)
and in one x-slab or one voxel (ordered in memory instead of LDS)."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2512_12945_amd import slimvdb as sv
from paper_2512_12945_amd import synth

from _gpu_util import assert_stats_equal, compare_maps, cuda, extract_np

pytestmark = pytest.mark.gpu

LDS_PAIRS = 2048  # pairs a leaf-kernel workgroup orders in LDS
WINDOW = 64       # observations whose point indices a wave combine holds at once


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sv.load()


def _sizes(o, pts, pose):
    """Largest observation count of a voxel, of a leaf and of an x-slab (8 x 8
    voxels of a leaf with one x offset) in one frame, from the oracle's pairs."""
    pr = o.frame_pairs(pts, pose)
    k = pr["keys"].astype(np.int64)
    _, per_vox = np.unique(k, axis=0, return_counts=True)
    leaf = np.floor_divide(k, 8)
    _, per_leaf = np.unique(leaf, axis=0, return_counts=True)
    slab = np.concatenate([leaf, np.mod(k[:, :1], 8)], axis=1)
    _, per_slab = np.unique(slab, axis=0, return_counts=True)
    return int(per_vox.max()), int(per_leaf.max()), int(per_slab.max())


def test_rgbd_room_full_frames_depth_ingest():
    """Two 640 x 480 depth frames of the open-set room (voxel 0.02 m, tau
    0.06 m, 512-d bf16 embeddings), through the depth-image ingest."""
    L, vs, tau = 512, 0.02, 0.06
    sc = synth.OpenRoomScene(L=L)
    intr = (sc.f, sc.f, sc.cx, sc.cy)
    g = sv.Map(vs, tau, 0.0, 10.0, sv.SEM_OPEN, 0, L, 0, 1 << 14, 1 << 21)
    o = oracle.OracleMap(vs, tau, 0.0, 10.0, oracle.SEM_OPEN, 0, L)
    for t in range(2):
        fr = sc.frame(t)
        pts = oracle.depth_points(fr["depth"], *intr)
        mv, ml, ms = _sizes(o, pts, fr["pose"])
        _say(f"room frame {t}: 640x480, L={L}; max obs/voxel {mv}, pairs/leaf {ml}, pairs/x-slab {ms}")
        assert mv > WINDOW and ml > LDS_PAIRS and ms > LDS_PAIRS
        g.integrate_depth(cuda(fr["depth"]), intr, fr["pose"], cuda(fr["emb"]), sv.IN_EMB_BF16)
        ost = o.integrate(pts, fr["pose"], fr["emb"], oracle.IN_EMB_BF16)
        assert_stats_equal(g.stats(), ost)
    err = compare_maps(extract_np(g), o.extract(), tau, sv.SEM_OPEN, L=L)
    _say(f"  errors {err}")


def test_densest_open_map_of_many_map_workload():
    """The open map with the most rays of the many-map workload (128-beam
    street, voxel 0.1 m, 256-d bf16 embeddings), integrated twice (the second
    time every voxel exists), alone and inside a batched launch."""
    L, vs, tau = 256, 0.1, 0.3
    draws = synth.batched_draws()
    i = max(range(16, 32), key=lambda j: draws[j][1])
    t, n = draws[i]
    scene = synth.StreetScene(seed=2, beams=128)
    sw = scene.sweep(t, nrays=n)
    emb = synth.primitive_embeddings(scene, sw["prim"], L, 4, t)
    g = sv.Map(vs, tau, 0.0, 50.0, sv.SEM_OPEN, 0, L, 0, 1 << 15, 1 << 21)
    gb = sv.Map(vs, tau, 0.0, 50.0, sv.SEM_OPEN, 0, L, 0, 1 << 15, 1 << 21)
    side = sv.Map(vs, tau, 0.0, 50.0, sv.SEM_CLOSED, 20, 0, 0, 1 << 15, 1 << 21)
    o = oracle.OracleMap(vs, tau, 0.0, 50.0, oracle.SEM_OPEN, 0, L)
    mv, ml, ms = _sizes(o, sw["points"], sw["pose"])
    _say(f"many-map workload, map {i}: {n} rays, L={L}; max obs/voxel {mv}, pairs/leaf {ml}, pairs/x-slab {ms}")
    assert mv > WINDOW and ml > LDS_PAIRS
    pts, e = cuda(sw["points"]), cuda(emb)
    side_pts = cuda(sw["points"][:5000])
    side_lab = cuda(sw["label"][:5000])
    frames = [dict(points=pts, pose=sw["pose"], sem=e, kind=sv.IN_EMB_BF16),
              dict(points=side_pts, pose=sw["pose"], sem=side_lab, kind=sv.IN_LABEL_I32)]
    for rep in range(2):
        g.integrate(pts, sw["pose"], e, sv.IN_EMB_BF16)
        sv.integrate_batched([gb, side], frames, use_graph=False)
        ost = o.integrate(sw["points"], sw["pose"], emb, oracle.IN_EMB_BF16)
        assert_stats_equal(g.stats(), ost)
        assert_stats_equal(gb.stats(), ost)
    ox = o.extract()
    gx = extract_np(g)
    err = compare_maps(gx, ox, tau, sv.SEM_OPEN, L=L)
    bx = extract_np(gb)
    for k in gx:
        assert np.array_equal(gx[k], bx[k]), k
    _say(f"  errors {err}")


@pytest.mark.parametrize("kind,L", [(sv.IN_EMB_BF16, 256), (sv.IN_EMB_F32, 256), (sv.IN_EMB_BF16, 512),
                                    (sv.IN_EMB_BF16, 100)])
def test_duplicated_points_huge_voxel_open(kind, L):
    """Thousands of copies of one point put more than 2048 observations in the
    voxels of its band (beyond one voxel in LDS and many 64-observation
    windows) and more than 2048 pairs in one x-slab; L = 100 takes the generic
    wave combine, the multiples of 64 the vectorised one."""
    rng = np.random.default_rng(23)
    vs, tau = 0.1, 0.3
    pose = np.eye(4)
    pose[:3, 3] = (0.05, 0.05, 0.05)
    base = np.array([3.037, 0.412, 0.227], np.float32)
    pts = np.concatenate([np.repeat(base[None], 3000, 0),
                          base + rng.normal(0, 0.12, (4000, 3)).astype(np.float32),
                          rng.uniform(-4, 4, (500, 3)).astype(np.float32)]).astype(np.float32)
    z = rng.normal(size=(len(pts), L)).astype(np.float32)
    z /= np.linalg.norm(z, axis=1, keepdims=True)
    emb = synth.to_bf16_bits(z)
    sem = emb if kind == sv.IN_EMB_BF16 else synth.bf16_bits_to_float(emb) * np.float32(0.999)
    g = sv.Map(vs, tau, 0.0, 50.0, sv.SEM_OPEN, 0, L, 0, 1 << 14, 1 << 20)
    o = oracle.OracleMap(vs, tau, 0.0, 50.0, oracle.SEM_OPEN, 0, L)
    mv, ml, ms = _sizes(o, pts, pose)
    _say(f"duplicated points, L={L} kind {kind}: max obs/voxel {mv}, pairs/leaf {ml}, pairs/x-slab {ms}")
    assert mv > LDS_PAIRS and ms > LDS_PAIRS
    for rep in range(2):
        g.integrate(cuda(pts), pose, cuda(sem), kind)
        ost = o.integrate(pts, pose, sem, kind)
        assert_stats_equal(g.stats(), ost)
    err = compare_maps(extract_np(g), o.extract(), tau, sv.SEM_OPEN, L=L)
    _say(f"  errors {err}")
