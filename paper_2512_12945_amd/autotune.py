"""Launch-shape autotuner for batched integration.

The grid sizes of the grid-stride kernels (leaf planning, pair bucketing, and
the per-leaf sort-and-combine kernel, see ``slim_set_launch_shape``) only move
time: every voxel is reduced in point order, so results are bitwise identical
for every shape.  The tuner times each candidate shape on scratch maps that
have the configurations of the real ones, integrating the real batch of frames
in steady state (every voxel already present), and caches the winner in a JSON
file keyed by device, map mix and point-count bucket.  Timing goes through the
library's own batched call; nothing here computes on the data.
"""
from __future__ import annotations

import json
import math
import os
import time

import torch

from . import slimvdb as sv

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "slimvdb_mi", "autotune.json")


def candidates(cus):
    out = []
    for plan in (cus // 2, cus, 2 * cus):
        for bucket in (4 * cus, 16 * cus):
            for leaf in (2, 4, 8, 16):
                out.append((max(plan, 1), max(bucket, 1), leaf))
    return out


def key_of(cfgs, frames):
    props = torch.cuda.get_device_properties(0)
    mix = sorted((c["sem_mode"], c.get("num_classes", 0), c.get("embed_dim", 0)) for c in cfgs)
    n = [int((f.get("points") if f.get("points") is not None else f["ranges"]).shape[0]) for f in frames]
    bucket = int(round(math.log2(max(sum(n) / max(len(n), 1), 1))))
    return f"{getattr(props, 'gcnArchName', props.name)}|{len(cfgs)}|{mix}|{bucket}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tune(cfgs, frames, reps=5, cache_path=DEFAULT_CACHE, use_graph=True, log=None):
    """Returns the fastest (plan_blocks, bucket_blocks, leaf_blocks_per_cu) for this batch.

    cfgs: list of dicts with Map constructor arguments, one per map; frames: the
    frames of integrate_batched.  Cached results are reused."""
    key = key_of(cfgs, frames)
    cache = _load(cache_path)
    if key in cache:
        return tuple(cache[key]["shape"])
    maps = [sv.Map(**c) for c in cfgs]
    sv.integrate_batched(maps, frames, use_graph=False)  # allocation-heavy first pass
    torch.cuda.synchronize()
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    best, best_t, table = None, float("inf"), []
    for shape in candidates(cus):
        maps[0].set_launch_shape(*shape)
        sv.integrate_batched(maps, frames, use_graph=use_graph)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            sv.integrate_batched(maps, frames, use_graph=use_graph)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        t = sorted(ts)[len(ts) // 2]
        table.append((shape, t))
        if t < best_t:
            best, best_t = shape, t
    for m in maps:
        m.close()
    if log:
        log(f"autotune {key}: best {best} {best_t * 1e3:.3f} ms of {len(table)} shapes")
    cache[key] = {"shape": list(best), "ms": best_t * 1e3}
    os.makedirs(os.path.dirname(cache_path), exist_ok=True)
    tmp = cache_path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1)
    os.replace(tmp, cache_path)
    return best
