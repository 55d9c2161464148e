"""The persistent batched launch: one launch whose workgroups take the
ray-chunk, planning, bucketing, leaf-tile, voxel-combine and commit items of
every map from an integer queue.  Checked against one slim_integrate per map
and against the per-stage batched launches, over maps of every leaf-kernel
variant, for several work splits and leaf-tile thresholds, on first frames and
on frames into existing maps, with and without a captured graph.  Every
comparison is bitwise; the L = 256 open-set and K = 20 label maps are also
checked against the oracle."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2512_12945_amd import slimvdb as sv
from paper_2512_12945_amd import synth

from _gpu_util import compare_maps, cuda, extract_np

pytestmark = pytest.mark.gpu

# (name, sem_mode, K, L, input kind): one map of each leaf-kernel variant
SPECS = [
    ("geometry", sv.SEM_NONE, 0, 0, sv.IN_NONE),
    ("labels5", sv.SEM_CLOSED, 5, 0, sv.IN_LABEL_I32),
    ("labels20", sv.SEM_CLOSED, 20, 0, sv.IN_LABEL_I32),
    ("logits20", sv.SEM_CLOSED, 20, 0, sv.IN_LOGIT_F32),
    ("probs8", sv.SEM_CLOSED, 8, 0, sv.IN_PROB_F32),
    ("last20", sv.SEM_CLOSED_LAST, 20, 0, sv.IN_LABEL_I32),
    ("open32", sv.SEM_OPEN, 0, 32, sv.IN_EMB_BF16),
    ("open256", sv.SEM_OPEN, 0, 256, sv.IN_EMB_BF16),
    ("open64f32", sv.SEM_OPEN, 0, 64, sv.IN_EMB_F32),
    ("openlast32", sv.SEM_OPEN_LAST, 0, 32, sv.IN_EMB_BF16),
]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _frames(sc, rep, seed=21):
    """One street frame per map; ray counts and trajectory points differ per map and rep."""
    rng = np.random.default_rng([seed, rep])
    out = []
    for j, (name, mode, K, L, kind) in enumerate(SPECS):
        n = int(rng.integers(3_000, 24_000))
        t = int(rng.integers(0, 100))
        sw = sc.sweep(t, nrays=n)
        sem = None
        if kind == sv.IN_LABEL_I32:
            sem = (sw["label"] % K).astype(np.int32)
        elif kind in (sv.IN_LOGIT_F32, sv.IN_PROB_F32):
            x = rng.normal(0.0, 1.0, size=(n, K))
            x[np.arange(n), sw["label"] % K] = 3.0
            sem = (synth.softmax64(x) if kind == sv.IN_PROB_F32 else x).astype(np.float32)
        elif kind in (sv.IN_EMB_BF16, sv.IN_EMB_F32):
            b = synth.primitive_embeddings(sc, sw["prim"], L, seed + j, t)
            sem = b if kind == sv.IN_EMB_BF16 else synth.bf16_bits_to_float(b).astype(np.float32)
        out.append(dict(points=sw["points"], pose=sw["pose"], sem=sem, kind=kind, name=name))
    return out


def _dev(frames):
    return [dict(points=cuda(f["points"]), pose=f["pose"], sem=None if f["sem"] is None else cuda(f["sem"]),
                 kind=f["kind"]) for f in frames]


def _maps():
    return [sv.Map(0.1, 0.3, 0.0, 50.0, mode, K, L, 0, 1 << 14, 1 << 20) for _, mode, K, L, _ in SPECS]


def _same(a, b, what):
    for k in a:
        assert np.array_equal(a[k], b[k]), (what, k)


@pytest.fixture(scope="module")
def street():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sv.load()
    sc = synth.StreetScene(seed=2, beams=128)
    reps = [_frames(sc, r) for r in range(3)]
    return reps


def test_persistent_equals_per_map_and_per_stage(street):
    seq, per_stage, pers, graph = _maps(), _maps(), _maps(), _maps()
    per_stage[0].set_launch_shape(batch_mode=2)
    pers[0].set_launch_shape(batch_mode=1)
    graph[0].set_launch_shape(batch_mode=1)
    for rep, host in enumerate(street):
        _say(f"persistent rep {rep}: {len(host)} maps, {sum(f['points'].shape[0] for f in host)} rays")
        dev = _dev(host)
        for m, f in zip(seq, dev):
            m.integrate(f["points"], f["pose"], f["sem"], f["kind"])
        sv.integrate_batched(per_stage, dev, use_graph=False)
        sv.integrate_batched(pers, dev, use_graph=False)
        sv.integrate_batched(graph, dev, use_graph=True)
        torch.cuda.synchronize()
        for i, f in enumerate(host):
            a = seq[i].stats()
            assert a["status_last"] == 0, f["name"]
            assert a == per_stage[i].stats() == pers[i].stats() == graph[i].stats(), f["name"]
            ea = extract_np(seq[i])
            _same(ea, extract_np(per_stage[i]), (rep, f["name"], "per-stage"))
            _same(ea, extract_np(pers[i]), (rep, f["name"], "persistent"))
            _same(ea, extract_np(graph[i]), (rep, f["name"], "graph"))


def test_persistent_graph_replays(street):
    """Replays of one captured persistent launch (new frames each time, same walk grid)."""
    ref, gra = _maps(), _maps()
    gra[0].set_launch_shape(batch_mode=1, walk_chunk=2)
    host = street[0]
    dev = _dev(host)
    for rep in range(4):
        _say(f"graph replay {rep}")
        for m, f in zip(ref, dev):
            m.integrate(f["points"], f["pose"], f["sem"], f["kind"])
        sv.integrate_batched(gra, dev, use_graph=True)
        torch.cuda.synchronize()
        for i, f in enumerate(host):
            assert ref[i].stats() == gra[i].stats(), f["name"]
            _same(extract_np(ref[i]), extract_np(gra[i]), (rep, f["name"]))


SHAPES = [
    dict(plan_blocks=1, bucket_blocks=1, leaf_blocks_per_cu=1, batch_mode=1, walk_chunk=1),
    dict(plan_blocks=7, bucket_blocks=13, leaf_blocks_per_cu=3, batch_mode=1, walk_chunk=64),
    dict(plan_blocks=1024, bucket_blocks=8192, leaf_blocks_per_cu=32, batch_mode=1, walk_chunk=3),
    dict(batch_mode=1, walk_chunk=16, wave_pairs=16, slab_pairs=512),
    dict(batch_mode=1, wave_pairs=64, slab_pairs=1024),
    dict(batch_mode=2, wave_pairs=32, slab_pairs=600),
]


@pytest.mark.parametrize("shape", SHAPES, ids=[str(i) for i in range(len(SHAPES))])
def test_work_split_and_tiles_do_not_change_results(street, shape):
    ref, alt = _maps(), _maps()
    alt[0].set_launch_shape(**shape)
    for rep, host in enumerate(street[:2]):
        _say(f"shape {shape} rep {rep}")
        dev = _dev(host)
        for m, f in zip(ref, dev):
            m.integrate(f["points"], f["pose"], f["sem"], f["kind"])
        sv.integrate_batched(alt, dev, use_graph=rep == 1)
        torch.cuda.synchronize()
        for i, f in enumerate(host):
            assert ref[i].stats() == alt[i].stats(), f["name"]
            _same(extract_np(ref[i]), extract_np(alt[i]), (rep, f["name"]))


def test_tiles_on_single_map_calls(street):
    """The leaf-tile thresholds also apply to slim_integrate: same maps."""
    host = street[0]
    dev = _dev(host)
    ref, alt = _maps(), _maps()
    for m in alt:
        m.set_launch_shape(wave_pairs=16, slab_pairs=512)
    for m, a, f in zip(ref, alt, dev):
        m.integrate(f["points"], f["pose"], f["sem"], f["kind"])
        a.integrate(f["points"], f["pose"], f["sem"], f["kind"])
    for i, f in enumerate(host):
        _same(extract_np(ref[i]), extract_np(alt[i]), f["name"])


def test_persistent_matches_oracle(street):
    host = street[0]
    maps = _maps()
    maps[0].set_launch_shape(batch_mode=1)
    sv.integrate_batched(maps, _dev(host), use_graph=True)
    for i, f in enumerate(host):
        name, mode, K, L, kind = SPECS[i]
        if name not in ("labels20", "open256"):
            continue
        _say(f"oracle {name}")
        o = oracle.OracleMap(0.1, 0.3, 0.0, 50.0, mode, K, L)
        o.integrate(f["points"], f["pose"], f["sem"], kind)
        if mode == sv.SEM_CLOSED:
            compare_maps(extract_np(maps[i]), o.extract(), 0.3, mode, K=K, exact_counts=True)
        else:
            compare_maps(extract_np(maps[i]), o.extract(), 0.3, mode, L=L)


def test_shape_validation():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    m = sv.Map(0.1, 0.3, 0.0, 50.0, sv.SEM_NONE, 0, 0, 0, 1 << 10, 1 << 16)
    for bad in (dict(batch_mode=3), dict(walk_chunk=65), dict(wave_pairs=8), dict(wave_pairs=257),
                dict(slab_pairs=511), dict(slab_pairs=2049)):
        with pytest.raises(sv.SlimError):
            m.set_launch_shape(**bad)
    m.set_launch_shape(batch_mode=2, walk_chunk=64, wave_pairs=256, slab_pairs=2048)
    m.set_launch_shape()
