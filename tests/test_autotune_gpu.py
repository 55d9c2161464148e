"""The launch-shape autotuner picks a shape from its knob values (batched form,
ray-chunk size, work split, leaf tiles), caches it by device, map mix and
point-count bucket, and the chosen shape gives the same maps."""
import json

import numpy as np
import pytest
import torch

from paper_2512_12945_amd import autotune
from paper_2512_12945_amd import slimvdb as sv
from paper_2512_12945_amd import synth

from _gpu_util import cuda, extract_np

pytestmark = pytest.mark.gpu


def test_tune_caches_and_keeps_results(tmp_path):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sv.load()
    w = synth.batched_workload(seed=4, nmaps=4, n_lo=2_000, n_hi=8_000, closed_maps=2, L=64)
    frames, cfgs = [], []
    for item in w:
        closed = item["mode"] == "closed"
        frames.append(dict(points=cuda(item["points"]), pose=item["pose"],
                           sem=cuda(item["label"] if closed else item["emb"]),
                           kind=sv.IN_LABEL_I32 if closed else sv.IN_EMB_BF16))
        cfgs.append(dict(voxel_size=0.1, sdf_trunc=0.3, min_range=0.0, max_range=50.0,
                         sem_mode=sv.SEM_CLOSED if closed else sv.SEM_OPEN, num_classes=item.get("K", 0),
                         embed_dim=item.get("L", 0), device=0, max_leaves=1 << 13, max_voxels=1 << 20))
    cache = str(tmp_path / "tune.json")
    shape = autotune.tune(cfgs, frames, reps=2, cache_path=cache)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    ax = autotune.axes(cus)
    assert set(shape) == set(ax)
    for k, v in shape.items():
        assert v in ax[k], (k, v)
    rec = json.load(open(cache))
    assert list(rec.values())[0]["shape"] == shape
    assert list(rec.values())[0]["shapes_timed"] >= sum(len(v) - 1 for v in ax.values()) + 1
    assert autotune.tune(cfgs, frames, cache_path=cache) == shape  # served from the cache
    ref = [sv.Map(**c) for c in cfgs]
    alt = [sv.Map(**c) for c in cfgs]
    alt[0].set_launch_shape(**shape)
    sv.integrate_batched(ref, frames, use_graph=True)
    sv.integrate_batched(alt, frames, use_graph=True)
    for a, b in zip(ref, alt):
        ea, eb = extract_np(a), extract_np(b)
        for k in ea:
            assert np.array_equal(ea[k], eb[k]), k
