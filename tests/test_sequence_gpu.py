"""slim_integrate_sequence gives bitwise the map (and last-frame statistics)
of one slim_integrate call per frame, interleaved with single frames and
resets: label and geometry maps through multi-frame passes of every size, with
empty frames and a pass that exceeds the leaf capacity; open-set maps with the
walk of each next frame overlapping the rest of the current one."""
import numpy as np
import pytest
import torch

import oracle
from paper_2512_12945_amd import slimvdb as sv
from paper_2512_12945_amd import synth

from _gpu_util import compare_maps, cuda, extract_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sweeps():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sv.load()
    sc = synth.StreetScene(seed=2)
    out = []
    for t in range(9):
        sw = sc.sweep(t, nrays=12_000 + 2_000 * t)  # ragged sizes
        out.append(dict(points=cuda(sw["points"]), pose=sw["pose"], sem=cuda(sw["label"]), kind=sv.IN_LABEL_I32,
                        np_points=sw["points"], np_label=sw["label"]))
    return out


def _map():
    return sv.Map(0.1, 0.3, 0.0, 50.0, sv.SEM_CLOSED, 20, 0, 0, 1 << 16, 1 << 22)


def _same(a, b):
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_sequence_equals_single_frames(sweeps):
    ref, seq = _map(), _map()
    for f in sweeps:
        ref.integrate(f["points"], f["pose"], f["sem"], f["kind"])
    sv.integrate_sequence(seq, sweeps)
    assert ref.stats() == seq.stats()
    _same(extract_np(ref), extract_np(seq))


def test_sequence_interleaved_with_single_frames_and_reset(sweeps):
    ref, seq = _map(), _map()
    plan = [("seq", 0, 3), ("one", 3, 4), ("seq", 4, 7), ("one", 7, 8), ("seq", 8, 9)]
    for rep in range(2):
        for what, a, b in plan:
            for f in sweeps[a:b]:
                ref.integrate(f["points"], f["pose"], f["sem"], f["kind"])
            if what == "seq":
                sv.integrate_sequence(seq, sweeps[a:b])
            else:
                for f in sweeps[a:b]:
                    seq.integrate(f["points"], f["pose"], f["sem"], f["kind"])
            assert ref.stats() == seq.stats(), (rep, what, a)
        _same(extract_np(ref), extract_np(seq))
        ref.reset()
        seq.reset()


def test_sequence_matches_oracle(sweeps):
    g = _map()
    o = oracle.OracleMap(0.1, 0.3, 0.0, 50.0, oracle.SEM_CLOSED, 20)
    sv.integrate_sequence(g, sweeps[:5])
    for f in sweeps[:5]:
        o.integrate(f["np_points"], f["pose"], f["np_label"], oracle.IN_LABEL_I32)
    compare_maps(extract_np(g), o.extract(), 0.3, sv.SEM_CLOSED, K=20, exact_counts=True)


def test_sequence_open_set():
    L = 64
    sc = synth.OpenRoomScene(seed=9, L=L, width=64, height=48, f=52.5, cx=31.5, cy=23.5, nboxes=12,
                             deg_per_frame=8.0)
    frames = []
    for t in range(5):
        fr = sc.frame(t)
        frames.append(dict(points=cuda(fr["points"]), pose=fr["pose"], sem=cuda(fr["emb"]), kind=sv.IN_EMB_BF16))
    ref = sv.Map(0.05, 0.15, 0.0, 100.0, sv.SEM_OPEN, 0, L, 0, 1 << 14, 1 << 21)
    seq = sv.Map(0.05, 0.15, 0.0, 100.0, sv.SEM_OPEN, 0, L, 0, 1 << 14, 1 << 21)
    for f in frames:
        ref.integrate(f["points"], f["pose"], f["sem"], f["kind"])
    sv.integrate_sequence(seq, frames)
    _same(extract_np(ref), extract_np(seq))


def _stats_status(m):
    """Statistics and the asynchronous error they report (0 if none)."""
    try:
        return m.stats(), 0
    except sv.SlimError as e:
        return m.stats(), e.code


@pytest.mark.parametrize("pass_frames", [1, 2, 3, 5, 8])
def test_sequence_pass_sizes(sweeps, pass_frames):
    # geometry and label maps take consecutive frames in multi-frame passes:
    # every pass size gives the per-frame map and the last frame's statistics
    ref, seq = _map(), _map()
    seq.set_launch_shape(pass_frames=pass_frames)
    for f in sweeps:
        ref.integrate(f["points"], f["pose"], f["sem"], f["kind"])
    sv.integrate_sequence(seq, sweeps)
    assert ref.stats() == seq.stats()
    _same(extract_np(ref), extract_np(seq))


def test_sequence_geometry_only(sweeps):
    ref = sv.Map(0.1, 0.3, 0.0, 50.0, sv.SEM_NONE, 0, 0, 0, 1 << 16, 1 << 22)
    seq = sv.Map(0.1, 0.3, 0.0, 50.0, sv.SEM_NONE, 0, 0, 0, 1 << 16, 1 << 22)
    frames = [dict(points=f["points"], pose=f["pose"]) for f in sweeps]
    for f in frames:
        ref.integrate(f["points"], f["pose"])
    sv.integrate_sequence(seq, frames)
    assert ref.stats() == seq.stats()
    _same(extract_np(ref), extract_np(seq))


def test_sequence_empty_frames_inside_passes(sweeps):
    empty = dict(points=torch.zeros((0, 3), dtype=torch.float32, device="cuda"), pose=sweeps[0]["pose"],
                 sem=torch.zeros(0, dtype=torch.int32, device="cuda"), kind=sv.IN_LABEL_I32)
    frames = [sweeps[0], empty, sweeps[1], sweeps[2], empty, empty, sweeps[3], sweeps[4]]
    ref, seq = _map(), _map()
    for f in frames:
        ref.integrate(f["points"], f["pose"], f["sem"], f["kind"])
    sv.integrate_sequence(seq, frames)
    assert ref.stats() == seq.stats()
    _same(extract_np(ref), extract_np(seq))


def test_sequence_capacity_fallback(sweeps):
    # a leaf capacity that frame 4 exceeds: the pass holding it is not applied,
    # and its frames and the later ones are integrated again one at a time,
    # ending exactly where per-frame calls end (rejected frames, error status)
    big = _map()
    leaves = []
    for f in sweeps:
        big.integrate(f["points"], f["pose"], f["sem"], f["kind"])
        leaves.append(big.stats()["leaves"])
    assert leaves[4] > leaves[3] + 1
    cap = (leaves[3] + leaves[4]) // 2
    ref = sv.Map(0.1, 0.3, 0.0, 50.0, sv.SEM_CLOSED, 20, 0, 0, cap, 1 << 22)
    seq = sv.Map(0.1, 0.3, 0.0, 50.0, sv.SEM_CLOSED, 20, 0, 0, cap, 1 << 22)
    for f in sweeps:
        ref.integrate(f["points"], f["pose"], f["sem"], f["kind"])
    sv.integrate_sequence(seq, sweeps)
    st_ref, err_ref = _stats_status(ref)
    st_seq, err_seq = _stats_status(seq)
    assert err_ref == sv.ERR_CAPACITY and err_seq == err_ref
    assert st_ref == st_seq and st_ref["leaves"] <= cap
    _same(extract_np(ref), extract_np(seq))
    # the map keeps taking passes afterwards
    ref.reset()
    seq.reset()
    for f in sweeps[:3]:
        ref.integrate(f["points"], f["pose"], f["sem"], f["kind"])
    sv.integrate_sequence(seq, sweeps[:3])
    assert ref.stats() == seq.stats()
    _same(extract_np(ref), extract_np(seq))


def test_sequence_passes_with_kernel_timing(sweeps):
    # with kernel timing on, passes run on one staging buffer with events around
    # each kernel: one launch set per pass or single frame, same map
    ref, seq = _map(), _map()
    for f in sweeps:
        ref.integrate(f["points"], f["pose"], f["sem"], f["kind"])
    seq.set_launch_shape(pass_frames=2)
    seq.profile(True)
    seq.profile_read()
    seq.profile_sets()
    sv.integrate_sequence(seq, sweeps)
    kern = seq.profile_read()
    sets = seq.profile_sets()
    seq.profile(False)
    assert ref.stats() == seq.stats()
    _same(extract_np(ref), extract_np(seq))
    # 9 frames in passes of 2 with the last alone: 4 passes + 1 single frame
    assert all(n == 5 for _, n in kern.values()), kern
    # label frames combine inside the leaf kernel: the voxel-combine stage is empty
    assert all(ms > 0 for k, (ms, _) in kern.items() if k != "voxel_combine"), kern
    assert [f for f, _, _ in sets] == [2, 2, 2, 2, 1], sets
    for f, ms, span in sets:
        assert span >= max(ms.values()) > 0
    assert abs(sum(ms["leaf_fuse"] for _, ms, _ in sets) - kern["leaf_fuse"][0]) <= 1e-6 * kern["leaf_fuse"][0] + 1e-9


def test_sequence_probability_rows_and_mixed_kinds(sweeps):
    # probability rows are not taken in passes (overlapped form); a call that
    # mixes rows and labels is overlapped as a whole; both equal per-frame calls
    rng = np.random.default_rng(5)
    frames = []
    for t, f in enumerate(sweeps[:6]):
        n = f["points"].shape[0]
        if t % 2:
            p = rng.random((n, 20)).astype(np.float32)
            p /= p.sum(axis=1, keepdims=True)
            frames.append(dict(points=f["points"], pose=f["pose"], sem=cuda(p), kind=sv.IN_PROB_F32))
        else:
            frames.append(f)
    for subset in (frames[1::2], frames):
        ref, seq = _map(), _map()
        for f in subset:
            ref.integrate(f["points"], f["pose"], f["sem"], f["kind"])
        sv.integrate_sequence(seq, subset)
        assert ref.stats() == seq.stats()
        _same(extract_np(ref), extract_np(seq))


def test_sequence_passes_of_ray_frames(sweeps):
    # frames given as ranges and unit directions go through passes too
    frames = []
    for f in sweeps[:5]:
        p = f["np_points"].astype(np.float64)
        r = np.linalg.norm(p, axis=1)
        keep = r > 0
        d = np.zeros_like(p)
        d[keep] = p[keep] / r[keep, None]
        frames.append(dict(ranges=cuda(r.astype(np.float32)), dirs=cuda(d.astype(np.float32)), pose=f["pose"],
                           sem=f["sem"], kind=sv.IN_LABEL_I32))
    ref, seq = _map(), _map()
    for f in frames:
        ref.integrate_rays(f["ranges"], f["dirs"], f["pose"], f["sem"], f["kind"])
    sv.integrate_sequence(seq, frames)
    assert ref.stats() == seq.stats()
    _same(extract_np(ref), extract_np(seq))
