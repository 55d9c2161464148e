"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.  Voxel keys, leaf and voxel counts, W, pair and reject
counts and one-hot class counts are compared bit for bit; D, class posteriors
and open-set statistics within the stated tolerances."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2512_12945_amd import slimvdb as sv
from paper_2512_12945_amd import synth

from _gpu_util import assert_stats_equal, compare_maps, cuda, extract_np, integrate_both, make_pair

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sv.load()


# ---------------------------------------------------------------------------
# tiny room (one 64x64 frame, 5 classes, softmax probabilities)
# ---------------------------------------------------------------------------


def test_room_single_frame_prob():
    _say("room 64x64, PROB_F32 K=5, vs 0.05 tau 0.15")
    fr = synth.room_frame(seed=1)
    g, o = make_pair(0.05, 0.15, 0.0, 100.0, sv.SEM_CLOSED, K=5)
    gst, ost = integrate_both(g, o, fr["points"], fr["pose"], fr["prob"], sv.IN_PROB_F32)
    assert_stats_equal(gst, ost)
    err = compare_maps(extract_np(g), o.extract(), 0.15, sv.SEM_CLOSED, K=5)
    _say(f"  errors {err}")


@pytest.mark.parametrize("kind", [sv.IN_LABEL_I32, sv.IN_PROB_F32, sv.IN_LOGIT_F32])
def test_room_sequence(kind):
    _say(f"room sequence 6 frames 96x72, kind {kind}")
    frames = synth.room_sequence(6, seed=3, yaw_span=1.2, width=96, height=72, f=60.0, cx=48.0, cy=36.0)
    g, o = make_pair(0.05, 0.15, 0.0, 100.0, sv.SEM_CLOSED, K=5)
    for fr in frames:
        sem = {sv.IN_LABEL_I32: fr["label"], sv.IN_PROB_F32: fr["prob"], sv.IN_LOGIT_F32: fr["logits"]}[kind]
        gst, ost = integrate_both(g, o, fr["points"], fr["pose"], sem, kind)
        assert_stats_equal(gst, ost)
    err = compare_maps(extract_np(g), o.extract(), 0.15, sv.SEM_CLOSED, K=5,
                       exact_counts=kind == sv.IN_LABEL_I32)
    _say(f"  errors {err}")


def test_geometry_only():
    _say("room sequence, geometry only")
    frames = synth.room_sequence(3, seed=4, yaw_span=0.8, width=80, height=60, f=50.0, cx=40.0, cy=30.0)
    g, o = make_pair(0.05, 0.15)
    for fr in frames:
        gst, ost = integrate_both(g, o, fr["points"], fr["pose"])
        assert_stats_equal(gst, ost)
    compare_maps(extract_np(g), o.extract(), 0.15, sv.SEM_NONE)


# ---------------------------------------------------------------------------
# LiDAR street (64 x 1024 sweeps, 20 classes, labels with flicker)
# ---------------------------------------------------------------------------


def test_lidar_sweeps():
    sc = synth.StreetScene(seed=2)
    g, o = make_pair(0.1, 0.3, 0.0, 50.0, sv.SEM_CLOSED, K=20, max_leaves=1 << 18, max_voxels=1 << 24)
    for t in range(4):
        _say(f"lidar sweep {t} (65536 rays)")
        sw = sc.sweep(t)
        gst, ost = integrate_both(g, o, sw["points"], sw["pose"], sw["label"], sv.IN_LABEL_I32)
        assert_stats_equal(gst, ost)
    err = compare_maps(extract_np(g), o.extract(), 0.3, sv.SEM_CLOSED, K=20, exact_counts=True)
    _say(f"  errors {err}")


# ---------------------------------------------------------------------------
# open set (small embedding, bf16 and fp32)
# ---------------------------------------------------------------------------


@pytest.mark.parametrize("kind,L", [(sv.IN_EMB_BF16, 16), (sv.IN_EMB_F32, 16), (sv.IN_EMB_BF16, 100)])
def test_open_set(kind, L):
    _say(f"open set L={L} kind {kind}")
    sc = synth.OpenRoomScene(seed=9, L=L, width=80, height=60, f=65.6, cx=39.5, cy=29.5, nboxes=12,
                             deg_per_frame=8.0)
    g, o = make_pair(0.05, 0.15, 0.0, 100.0, sv.SEM_OPEN, L=L)
    for t in range(3):
        fr = sc.frame(t)
        z = fr["emb"] if kind == sv.IN_EMB_BF16 else synth.bf16_bits_to_float(fr["emb"]) * np.float32(0.999)
        gst, ost = integrate_both(g, o, fr["points"], fr["pose"], z, kind)
        assert_stats_equal(gst, ost)
    err = compare_maps(extract_np(g), o.extract(), 0.15, sv.SEM_OPEN, L=L)
    _say(f"  errors {err}")


@pytest.mark.parametrize("kind,L", [(sv.IN_EMB_BF16, 128), (sv.IN_EMB_F32, 64), (sv.IN_EMB_BF16, 256),
                                    (sv.IN_EMB_F32, 256), (sv.IN_EMB_BF16, 512), (sv.IN_EMB_BF16, 1024)])
def test_open_set_wide(kind, L):
    """Embedding sizes that are multiples of 64 (rows read as whole words per lane)."""
    _say(f"open set wide L={L} kind {kind}")
    sc = synth.OpenRoomScene(seed=9, L=L, width=64, height=48, f=52.5, cx=31.5, cy=23.5, nboxes=12,
                             deg_per_frame=8.0)
    g, o = make_pair(0.05, 0.15, 0.0, 100.0, sv.SEM_OPEN, L=L)
    for t in range(3):
        fr = sc.frame(t)
        z = fr["emb"] if kind == sv.IN_EMB_BF16 else synth.bf16_bits_to_float(fr["emb"]) * np.float32(0.999)
        gst, ost = integrate_both(g, o, fr["points"], fr["pose"], z, kind)
        assert_stats_equal(gst, ost)
    err = compare_maps(extract_np(g), o.extract(), 0.15, sv.SEM_OPEN, L=L)
    _say(f"  errors {err}")


# ---------------------------------------------------------------------------
# edge cases
# ---------------------------------------------------------------------------


def test_empty_and_rejected_frames():
    _say("empty frame, all-rejected frame, ragged sizes")
    g, o = make_pair(0.05, 0.15, 0.2, 10.0, sv.SEM_CLOSED, K=5)
    pose = np.eye(4)
    gst, ost = integrate_both(g, o, np.zeros((0, 3), np.float32), pose, np.zeros(0, np.int32), sv.IN_LABEL_I32)
    assert_stats_equal(gst, ost)
    bad = np.array([[np.nan, 0, 0], [0.0, 0.0, 0.0], [0.1, 0, 0], [20.0, 0, 0], [np.inf, 0, 0]], np.float32)
    gst, ost = integrate_both(g, o, bad, pose, np.array([0, 1, 2, 3, 4], np.int32), sv.IN_LABEL_I32)
    assert_stats_equal(gst, ost)
    assert gst["rejected_last"] == 5 and gst["voxels"] == 0
    rng = np.random.default_rng(5)
    for n in (1, 63, 65, 257, 1000):
        pts = rng.uniform(-3, 3, size=(n, 3)).astype(np.float32)
        lab = rng.integers(-1, 6, size=n).astype(np.int32)  # -1 and 5 are invalid labels
        gst, ost = integrate_both(g, o, pts, pose, lab, sv.IN_LABEL_I32)
        assert_stats_equal(gst, ost)
    compare_maps(extract_np(g), o.extract(), 0.15, sv.SEM_CLOSED, K=5, exact_counts=True)


def test_exact_boundaries_and_duplicates():
    _say("dyadic geometry: points on voxel faces, duplicated points")
    g, o = make_pair(0.125, 0.375, 0.0, 100.0, sv.SEM_CLOSED, K=3)
    pose = np.eye(4)
    pose[:3, 3] = (0.0, 0.0625, 0.0625)
    xs = np.arange(-24, 25) * 0.125
    pts = np.stack(np.meshgrid(xs, xs, [2.0, 2.5, -1.75]), -1).reshape(-1, 3).astype(np.float32)
    pts = np.concatenate([pts, pts[::7]])
    lab = (np.arange(len(pts)) % 3).astype(np.int32)
    gst, ost = integrate_both(g, o, pts, pose, lab, sv.IN_LABEL_I32)
    assert_stats_equal(gst, ost)
    compare_maps(extract_np(g), o.extract(), 0.375, sv.SEM_CLOSED, K=3, exact_counts=True)


def test_large_leaf_bucket():
    """A dense camera close to a wall puts more pairs in one leaf than the LDS
    sort holds, exercising the in-memory sort path."""
    _say("large bucket: dense pinhole at 0.6 m, vs 0.02")
    fr = synth.room_frame(seed=8, width=200, height=200, f=500.0, cx=100.0, cy=100.0, room=(4.0, 4.0, 3.0),
                          position=(3.4, 2.0, 1.5))
    g, o = make_pair(0.02, 0.06, 0.0, 10.0, sv.SEM_CLOSED, K=5)
    pr = o.frame_pairs(fr["points"], fr["pose"])
    _, per_leaf = np.unique(np.floor_divide(pr["keys"], 8), axis=0, return_counts=True)
    assert per_leaf.max() > 4096  # more than the LDS path holds
    gst, ost = integrate_both(g, o, fr["points"], fr["pose"], fr["prob"], sv.IN_PROB_F32)
    assert_stats_equal(gst, ost)
    compare_maps(extract_np(g), o.extract(), 0.06, sv.SEM_CLOSED, K=5)


@pytest.mark.parametrize("mode", [sv.SEM_CLOSED, sv.SEM_CLOSED_LAST])
def test_huge_voxel_and_slab(mode):
    """Thousands of duplicated points put more pairs in one voxel, and in one
    x-slab of a leaf, than the leaf kernel holds in LDS (the split of a large
    leaf by slab, the chunked slab and the in-memory order of one bin)."""
    _say(f"huge voxel bin and slab, mode {mode}")
    rng = np.random.default_rng(17)
    g, o = make_pair(0.1, 0.3, 0.0, 50.0, mode, K=6)
    pose = np.eye(4)
    pose[:3, 3] = (0.05, 0.05, 0.05)
    base = np.array([3.037, 0.412, 0.227], np.float32)
    pts = np.concatenate([np.repeat(base[None], 3000, 0),
                          base + rng.normal(0, 0.12, (4000, 3)).astype(np.float32),
                          rng.uniform(-4, 4, (500, 3)).astype(np.float32)]).astype(np.float32)
    lab = rng.integers(0, 6, len(pts)).astype(np.int32)
    pr = o.frame_pairs(pts, pose, lab, oracle.IN_LABEL_I32)
    _, per_vox = np.unique(pr["keys"], axis=0, return_counts=True)
    assert per_vox.max() > 2048
    for rep in range(2):
        gst, ost = integrate_both(g, o, pts, pose, lab, sv.IN_LABEL_I32)
        assert_stats_equal(gst, ost)
    gx, ox = extract_np(g), o.extract()
    compare_maps(gx, ox, 0.3, mode, K=6, exact_counts=mode == sv.SEM_CLOSED)
    if mode == sv.SEM_CLOSED_LAST:
        assert np.array_equal(gx["sem"].astype(np.float64), ox["sem"])


def test_capacity_all_or_nothing():
    _say("capacity: a frame that does not fit leaves the map unchanged")
    frames = synth.room_sequence(2, seed=6, yaw_span=2.0, width=64, height=48, f=40.0, cx=32.0, cy=24.0)
    o = oracle.OracleMap(0.05, 0.15, 0.0, 100.0, oracle.SEM_CLOSED, 5)
    o.integrate(frames[0]["points"], frames[0]["pose"], frames[0]["label"], oracle.IN_LABEL_I32)
    cap = o.leaf_count() + 1
    st = o.integrate(frames[1]["points"], frames[1]["pose"], frames[1]["label"], oracle.IN_LABEL_I32)
    assert st["new_leaves"] > 1  # the second frame does not fit
    g = sv.Map(0.05, 0.15, 0.0, 100.0, sv.SEM_CLOSED, 5, 0, 0, cap, 1 << 20)
    g.integrate(cuda(frames[0]["points"]), frames[0]["pose"], cuda(frames[0]["label"]), sv.IN_LABEL_I32)
    st0 = g.stats()
    assert st0["leaves"] == cap - 1
    before = extract_np(g)
    g.integrate(cuda(frames[1]["points"]), frames[1]["pose"], cuda(frames[1]["label"]), sv.IN_LABEL_I32)
    with pytest.raises(sv.SlimError) as ei:
        g.stats()
    assert ei.value.code == sv.ERR_CAPACITY
    st1 = g.stats()  # error reported once
    assert st1["status_last"] == sv.ERR_CAPACITY and st1["leaves"] == st0["leaves"]
    after = extract_np(g)
    for k in before:
        assert np.array_equal(before[k], after[k])
    # the map keeps working after a rejected frame
    g.integrate(cuda(frames[0]["points"]), frames[0]["pose"], cuda(frames[0]["label"]), sv.IN_LABEL_I32)
    assert g.stats()["status_last"] == 0


def test_voxel_capacity_all_or_nothing():
    _say("voxel capacity")
    fr = synth.room_frame(seed=2)
    g = sv.Map(0.05, 0.15, 0.0, 100.0, sv.SEM_CLOSED, 5, 0, 0, 1 << 12, 1000)
    g.integrate(cuda(fr["points"]), fr["pose"], cuda(fr["label"]), sv.IN_LABEL_I32)
    with pytest.raises(sv.SlimError):
        g.stats()
    assert g.stats()["voxels"] == 0


def test_determinism_and_reset():
    _say("determinism: two maps, same frames -> bitwise equal; reset")
    sc = synth.StreetScene(seed=2)
    sw = [sc.sweep(t) for t in (10, 11)]
    outs = []
    for _ in range(2):
        g = sv.Map(0.1, 0.3, 0.0, 50.0, sv.SEM_CLOSED, 20, 0, 0, 1 << 16, 1 << 22)
        for s in sw:
            g.integrate(cuda(s["points"]), s["pose"], cuda(s["label"]), sv.IN_LABEL_I32)
        outs.append(extract_np(g))
        g.reset()
        assert g.stats()["voxels"] == 0
        g.integrate(cuda(sw[0]["points"]), sw[0]["pose"], cuda(sw[0]["label"]), sv.IN_LABEL_I32)
        assert g.stats()["voxels"] > 0
    for k in outs[0]:
        assert np.array_equal(outs[0][k], outs[1][k])


def test_query_matches_extract():
    _say("query vs extract")
    frames = synth.room_sequence(2, seed=7, yaw_span=0.5, width=64, height=48, f=40.0, cx=32.0, cy=24.0)
    g = sv.Map(0.05, 0.15, 0.0, 100.0, sv.SEM_CLOSED, 5, 0, 0)
    for fr in frames:
        g.integrate(cuda(fr["points"]), fr["pose"], cuda(fr["prob"]), sv.IN_PROB_F32)
    ex = extract_np(g)
    centres = ((ex["keys"].astype(np.float64) + 0.5) * np.float64(np.float32(0.05))).astype(np.float32)
    q = g.query(cuda(centres))
    torch.cuda.synchronize()
    assert np.array_equal(q["W"].cpu().numpy(), ex["W"])
    assert np.array_equal(q["D"].cpu().numpy(), ex["D"])
    assert np.array_equal(q["sem"].cpu().numpy(), ex["sem"])
    far = cuda(np.array([[100.0, 100.0, 100.0], [np.nan, 0, 0]], np.float32))
    q = g.query(far)
    assert float(q["W"].abs().sum()) == 0.0


def test_oracle_not_loaded_by_product():
    import paper_2512_12945_amd.slimvdb as mod

    assert "oracle" not in open(mod.__file__).read()
