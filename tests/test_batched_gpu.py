"""Batched integration of many maps (one launch per kernel stage for all maps,
optionally replayed from a captured HIP graph) against one slim_integrate per
map, and launch-shape invariance.  Results must be bitwise identical."""
import sys

import numpy as np
import pytest
import torch

from paper_2512_12945_amd import slimvdb as sv
from paper_2512_12945_amd import synth

from _gpu_util import compare_maps, cuda, extract_np
import oracle

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def workload():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sv.load()
    # small version of the 32-map workload: 6 maps, 3 closed (K = 20), 3 open (L = 32)
    w = synth.batched_workload(seed=4, nmaps=6, n_lo=2_000, n_hi=20_000, closed_maps=3, L=32)
    frames = []
    for item in w:
        if item["mode"] == "closed":
            frames.append(dict(points=cuda(item["points"]), pose=item["pose"], sem=cuda(item["label"]),
                               kind=sv.IN_LABEL_I32))
        else:
            frames.append(dict(points=cuda(item["points"]), pose=item["pose"], sem=cuda(item["emb"]),
                               kind=sv.IN_EMB_BF16))
    return w, frames


def _maps(w):
    out = []
    for item in w:
        if item["mode"] == "closed":
            out.append(sv.Map(0.1, 0.3, 0.0, 50.0, sv.SEM_CLOSED, item["K"], 0, 0, 1 << 14, 1 << 21))
        else:
            out.append(sv.Map(0.1, 0.3, 0.0, 50.0, sv.SEM_OPEN, 0, item["L"], 0, 1 << 14, 1 << 21))
    return out


def _same(a, b):
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_batched_equals_sequential_and_graph_replays(workload):
    w, frames = workload
    seq, bat, gra = _maps(w), _maps(w), _maps(w)
    for rep in range(3):
        _say(f"replay {rep}")
        for m, f in zip(seq, frames):
            m.integrate(f["points"], f["pose"], f["sem"], f["kind"])
        sv.integrate_batched(bat, frames, use_graph=False)
        sv.integrate_batched(gra, frames, use_graph=True)
        torch.cuda.synchronize()
        for i in range(len(w)):
            a, b, c = seq[i].stats(), bat[i].stats(), gra[i].stats()
            assert a == b == c, (i, a, b, c)
            ea = extract_np(seq[i])
            _same(ea, extract_np(bat[i]))
            _same(ea, extract_np(gra[i]))


def test_batched_matches_oracle(workload):
    w, frames = workload
    maps = _maps(w)
    sv.integrate_batched(maps, frames, use_graph=True)
    for i, item in enumerate(w):
        if item["mode"] == "closed":
            o = oracle.OracleMap(0.1, 0.3, 0.0, 50.0, oracle.SEM_CLOSED, item["K"])
            o.integrate(item["points"], item["pose"], item["label"], oracle.IN_LABEL_I32)
            compare_maps(extract_np(maps[i]), o.extract(), 0.3, sv.SEM_CLOSED, K=item["K"], exact_counts=True)
        else:
            o = oracle.OracleMap(0.1, 0.3, 0.0, 50.0, oracle.SEM_OPEN, 0, item["L"])
            o.integrate(item["points"], item["pose"], item["emb"], oracle.IN_EMB_BF16)
            compare_maps(extract_np(maps[i]), o.extract(), 0.3, sv.SEM_OPEN, L=item["L"])


@pytest.mark.parametrize("shape", [(1, 1, 1), (7, 13, 3), (1024, 8192, 32)])
def test_launch_shape_does_not_change_results(workload, shape):
    w, frames = workload
    ref, alt = _maps(w), _maps(w)
    for m in alt:
        m.set_launch_shape(*shape)
    for _ in range(2):
        for m, f in zip(ref, frames):
            m.integrate(f["points"], f["pose"], f["sem"], f["kind"])
        for m, f in zip(alt, frames):
            m.integrate(f["points"], f["pose"], f["sem"], f["kind"])
    sv.integrate_batched(alt, frames, use_graph=False)
    for m, f in zip(ref, frames):
        m.integrate(f["points"], f["pose"], f["sem"], f["kind"])
    for i in range(len(w)):
        _same(extract_np(ref[i]), extract_np(alt[i]))


@pytest.mark.parametrize("L", [256, 512])
def test_joint_combine_list_over_maps_of_one_kind(L):
    """Several maps of one vectorised wave-combine kind in one batched call:
    the combine takes their voxel lists as one.  A map whose frame has no
    valid point (no voxel) sits between the others.  Bitwise equal to one
    call per map, on first frames and on frames into existing voxels, eager
    and from a graph."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sv.load()
    sc = synth.StreetScene(seed=2, beams=128)
    rng = np.random.default_rng(L)
    frames = []
    for j in range(4):
        t = int(rng.integers(0, 100))
        sw = sc.sweep(t, nrays=int(rng.integers(3_000, 12_000)))
        pts = sw["points"].copy()
        if j == 1:
            pts[:] = np.nan  # every point rejected: the map lists no voxel
        emb = synth.primitive_embeddings(sc, sw["prim"], L, 7 + j, t)
        frames.append(dict(points=cuda(pts), pose=sw["pose"], sem=cuda(emb), kind=sv.IN_EMB_BF16))

    def maps():
        return [sv.Map(0.1, 0.3, 0.0, 50.0, sv.SEM_OPEN, 0, L, 0, 1 << 14, 1 << 21) for _ in frames]

    seq, bat, gra = maps(), maps(), maps()
    for rep in range(2):
        for m, f in zip(seq, frames):
            m.integrate(f["points"], f["pose"], f["sem"], f["kind"])
        sv.integrate_batched(bat, frames, use_graph=False)
        sv.integrate_batched(gra, frames, use_graph=True)
        torch.cuda.synchronize()
        for i in range(len(frames)):
            a, b, c = seq[i].stats(), bat[i].stats(), gra[i].stats()
            assert a == b == c, (rep, i, a, b, c)
            ea = extract_np(seq[i])
            _same(ea, extract_np(bat[i]))
            _same(ea, extract_np(gra[i]))
        _say(f"L={L} rep {rep}: voxels per map {[s.stats()['voxels'] for s in seq]}")
    assert seq[1].stats()["voxels"] == 0 and min(seq[i].stats()["voxels"] for i in (0, 2, 3)) > 0
