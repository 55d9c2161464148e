"""Launch-shape autotuner for batched integration.

A shape (``slim_set_launch_shape``) has three kinds of knobs:

* the form of the batched call: one persistent launch whose workgroups take
  work items of every map from a queue (batch_mode 1), or one launch per stage
  for all maps (batch_mode 2);
* the work split: the ray-chunk size of the walk items (walk_chunk, in blocks
  of 256 rays) and the numbers of planning, bucketing and leaf-tile items
  (grid sizes of the per-stage form);
* the leaf tiles: the most pairs of a leaf done by one wave (wave_pairs) and
  the pairs above which a sorted leaf is split into x-slab items (slab_pairs).

None of them changes a result: every voxel's sums are exact integers or formed
in point order, so the maps are bitwise identical for every shape.  The tuner
times shapes on scratch maps that have the configurations of the real ones,
integrating the real batch of frames in steady state (every voxel already
present), by coordinate descent from the library's defaults: one knob at a time
over its values, keeping the best, until a sweep over all knobs gains nothing.
The winner is cached in a JSON file keyed by device, map mix and point-count
bucket.  Timing goes through the library's own batched call; nothing here
computes on the data.
"""
from __future__ import annotations

import json
import math
import os
import time

import torch

from . import slimvdb as sv

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "slimvdb_mi", "autotune.json")


def axes(cus):
    """Values each knob may take; the first value of each is the library default."""
    return {
        "batch_mode": [1, 2],
        "walk_chunk": [4, 1, 2, 8, 16],
        "leaf_blocks_per_cu": [16, 2, 4, 8, 32],
        "bucket_blocks": [16 * cus, 2 * cus, 4 * cus, 32 * cus],
        "plan_blocks": [cus, max(cus // 2, 1), 2 * cus],
        "wave_pairs": [0, 32, 64, 128],
        "slab_pairs": [0, 1024, 512],
    }


def default_shape(cus):
    return {k: v[0] for k, v in axes(cus).items()}


def key_of(cfgs, frames):
    props = torch.cuda.get_device_properties(0)
    mix = sorted((c["sem_mode"], c.get("num_classes", 0), c.get("embed_dim", 0)) for c in cfgs)
    n = [int((f.get("points") if f.get("points") is not None else f["ranges"]).shape[0]) for f in frames]
    bucket = int(round(math.log2(max(sum(n) / max(len(n), 1), 1))))
    return f"v3|{getattr(props, 'gcnArchName', props.name)}|{len(cfgs)}|{mix}|{bucket}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tune(cfgs, frames, reps=5, cache_path=DEFAULT_CACHE, use_graph=True, log=None, max_sweeps=3):
    """Returns the fastest shape found for this batch, as keyword arguments of
    Map.set_launch_shape.

    cfgs: list of dicts with Map constructor arguments, one per map; frames: the
    frames of integrate_batched.  Cached results are reused."""
    key = key_of(cfgs, frames)
    cache = _load(cache_path)
    if key in cache:
        return dict(cache[key]["shape"])
    maps = [sv.Map(**c) for c in cfgs]
    sv.integrate_batched(maps, frames, use_graph=False)  # allocation-heavy first pass
    torch.cuda.synchronize()
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    ax = axes(cus)
    seen = {}

    def cost(shape):
        k = tuple(sorted(shape.items()))
        if k not in seen:
            maps[0].set_launch_shape(**shape)
            sv.integrate_batched(maps, frames, use_graph=use_graph)
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                t0 = time.perf_counter()
                sv.integrate_batched(maps, frames, use_graph=use_graph)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            seen[k] = sorted(ts)[len(ts) // 2]
        return seen[k]

    best = default_shape(cus)
    best_t = cost(best)
    for _ in range(max_sweeps):
        improved = False
        for name, values in ax.items():
            for v in values:
                if v == best[name]:
                    continue
                cand = dict(best, **{name: v})
                t = cost(cand)
                if t < best_t:
                    best, best_t, improved = cand, t, True
        if not improved:
            break
    for m in maps:
        m.close()
    if log:
        log(f"autotune {key}: best {best} {best_t * 1e3:.3f} ms after {len(seen)} shapes")
    cache[key] = {"shape": best, "ms": best_t * 1e3, "shapes_timed": len(seen)}
    os.makedirs(os.path.dirname(cache_path), exist_ok=True)
    tmp = cache_path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1)
    os.replace(tmp, cache_path)
    return best
