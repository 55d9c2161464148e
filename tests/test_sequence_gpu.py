"""slim_integrate_sequence (the walk of each next frame overlapping the rest
of the current one on a second staging buffer) gives bitwise the map of one
slim_integrate call per frame, interleaved with single frames and resets."""
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
