"""Throughput of fused TSDF + Bayesian semantic integration on one MI355X.

Default workload: the LiDAR street -- sweeps of a 64-beam x 1024-azimuth
spinning sensor (65,536 points per sweep) driving along a synthetic street of
boxes and cylinders, voxel 0.1 m, truncation 0.3 m, 20 closed-set classes
given as per-point labels with 10 % flicker.  One step integrates one sweep
into the growing map (ray walk, leaf allocation, TSDF fusion, Dirichlet
update).  All sweeps are generated and copied to the GPU before timing.

Prints one JSON line.  Besides points/s it reports voxel updates/s, the
fraction of the HBM roofline of the dominant kernel (algorithmic bytes over
its average duration, HIP events on the stream it runs on) and of the whole
step, and the CPU oracle timed on a bounded sample of the same sweeps.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak, GB/s

METRIC = "points/s & voxel-updates/s, fused TSDF+semantic; fwd+bwd vs plain, same GPU"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=90)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the CPU oracle sample")
    ap.add_argument("--no-diff", action="store_true", help="skip the forward+backward measurement")
    ap.add_argument("--diff-reps", type=int, default=5)
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def diff_bench(sv, synth, torch, scene, frames=16, reps=5, vs=0.1, tau=0.3, ncls=20):
    """Differentiation workload: 16 ray sweeps (ranges, directions, 20-class
    logits) integrated into a fresh map, the map loss, and its backward w.r.t.
    logits and ranges; times the plain forward and forward + backward."""
    t0 = time.time()
    sw = [scene.ray_sweep(t) for t in range(frames)]
    dev = torch.device("cuda", 0)
    ranges = torch.from_numpy(np.stack([s["ranges"] for s in sw])).to(dev)
    dirs = torch.from_numpy(np.stack([s["dirs"] for s in sw])).to(dev)
    logits = torch.from_numpy(np.stack([s["logits"] for s in sw])).to(dev)
    poses = [s["pose"] for s in sw]
    gmap = sv.Map(vs, tau, 0.0, 50.0, sv.SEM_CLOSED, ncls, 0, 0, max_leaves=1 << 18, max_voxels=1 << 24)

    def forward():
        gmap.reset()
        for f in range(frames):
            gmap.integrate_rays(ranges[f], dirs[f], poses[f], logits[f], sv.IN_LOGIT_F32)

    forward()
    ex = gmap.extract()
    keys = ex["keys"]
    labels = torch.from_numpy(scene.nearest_class((keys.cpu().numpy() + 0.5) * np.float64(np.float32(vs)))).to(dev)
    samples = torch.from_numpy(scene.surface_samples(sw, count=10000)).to(dev)
    gl = torch.empty_like(logits)
    gr = torch.empty_like(ranges)
    log(f"differentiation inputs ready in {time.time() - t0:.1f}s: {keys.shape[0]} voxels")

    def fwd_bwd():
        forward()
        gmap.loss(keys, labels, samples, 1.0)
        for f in range(frames):
            gmap.backward_rays(ranges[f], dirs[f], poses[f], logits[f], gl[f], gr[f])

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            s = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - s)
        return float(np.median(ts)) * 1e3

    t_fwd = timed(forward)
    t_fb = timed(fwd_bwd)
    return {"workload": f"{frames} LiDAR ray sweeps x {ranges.shape[1]} rays, 20-class logits, map loss = "
                        "Dirichlet-predictive cross-entropy over all voxels + mean |D| at 10k surface samples",
            "fwd_ms": t_fwd, "fwd_bwd_ms": t_fb, "ratio": t_fb / t_fwd, "voxels": int(keys.shape[0]),
            "points_per_s_fwd_bwd": frames * ranges.shape[1] / (t_fb / 1e3)}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this integrator runs on one GPU; multi-GPU runs are not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    from paper_2512_12945_amd import slimvdb as sv
    from paper_2512_12945_amd import synth

    K, W = args.steps, args.warmup
    vs, tau, rmax, ncls = 0.1, 0.3, 50.0, 20
    scene = synth.StreetScene(seed=2)
    t0 = time.time()
    sweeps = scene.sweeps(range(W + K), workers=min(8, os.cpu_count() or 1))
    log(f"generated {W + K} sweeps in {time.time() - t0:.1f}s")
    dev = torch.device("cuda", 0)
    pts = [torch.from_numpy(s["points"]).to(dev) for s in sweeps]
    lab = [torch.from_numpy(s["label"]).to(dev) for s in sweeps]
    poses = [s["pose"] for s in sweeps]
    torch.cuda.synchronize()
    n_pts = sweeps[0]["points"].shape[0]

    gmap = sv.Map(vs, tau, 0.0, rmax, sv.SEM_CLOSED, ncls, 0, 0, max_leaves=1 << 18, max_voxels=1 << 24)

    # counts per sweep (deterministic): one untimed pass with stats
    per = []
    for i in range(W + K):
        gmap.integrate(pts[i], poses[i], lab[i], sv.IN_LABEL_I32)
        per.append(gmap.stats())
    gmap.reset()
    torch.cuda.synchronize()

    # timed pass: warm-up sweeps, then K timed sweeps with kernel events
    for i in range(W):
        gmap.integrate(pts[i], poses[i], lab[i], sv.IN_LABEL_I32)
    gmap.profile(True)
    gmap.profile_read()
    torch.cuda.synchronize()
    start = time.perf_counter()
    for i in range(W, W + K):
        gmap.integrate(pts[i], poses[i], lab[i], sv.IN_LABEL_I32)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - start
    kern = gmap.profile_read()
    gmap.profile(False)
    final = gmap.stats()
    assert final["voxels"] == per[-1]["voxels"], "timed pass diverged from the counting pass"

    # same K sweeps again without events, for the step time without event overhead
    gmap.reset()
    for i in range(W):
        gmap.integrate(pts[i], poses[i], lab[i], sv.IN_LABEL_I32)
    torch.cuda.synchronize()
    s2 = time.perf_counter()
    for i in range(W, W + K):
        gmap.integrate(pts[i], poses[i], lab[i], sv.IN_LABEL_I32)
    torch.cuda.synchronize()
    elapsed_noev = time.perf_counter() - s2

    timed = per[W:W + K]
    P = sum(s["pairs_last"] for s in timed)
    valid = sum(s["points_last"] - s["rejected_last"] for s in timed)
    u_old = sum(s["voxels_old_last"] for s in timed)
    u_new = sum(s["voxels_new_last"] for s in timed)
    S_v = 8 + 4 * ncls  # D, W and K float counts
    b_sem = 4           # int32 label
    bytes_points = n_pts * K * 12
    bytes_sem = n_pts * K * b_sem
    bytes_state = u_old * 2 * S_v + u_new * S_v
    b_alg = bytes_points + bytes_sem + bytes_state

    # dominant kernel and its algorithmic bytes
    kalg = {"ray_walk_emit": bytes_points, "leaf_plan": 0, "pair_bucket": 0, "leaf_fuse": bytes_sem + bytes_state,
            "frame_commit": 0}
    dom = max(kern, key=lambda k: kern[k][0])
    dom_ms, dom_n = kern[dom]
    dom_avg_s = dom_ms / 1e3 / max(dom_n, 1)
    dom_gbs = kalg[dom] / K / dom_avg_s / 1e9 if dom_avg_s > 0 else 0.0
    ms_step = elapsed_noev / K * 1e3

    result = {
        "metric": METRIC,
        "value": n_pts * K / elapsed_noev,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "lidar-street: 64x1024 sweeps (65,536 points), voxel 0.1 m, trunc 0.3 m, "
                               "20 classes as int32 labels, 10% flicker; map grows over the sweeps",
                   "points_per_step": n_pts, "voxel_size": vs, "sdf_trunc": tau, "num_classes": ncls,
                   "first_timed_sweep": W},
        "voxel_updates_per_s": P / elapsed_noev,
        "valid_points_per_s": valid / elapsed_noev,
        "ms_per_step_with_kernel_events": elapsed / K * 1e3,
        "alg_bytes_per_step": b_alg / K,
        "path_roofline_frac": (b_alg / elapsed_noev / 1e9) / HBM_PEAK_GBS,
        "kernel_ms_per_step": {k: v[0] / max(v[1], 1) for k, v in kern.items()},
        "roofline": {"kernel": dom, "bound": "hbm", "achieved": dom_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": dom_gbs / HBM_PEAK_GBS, "traffic": None,
                     "alg_bytes_per_launch": kalg[dom] / K},
    }

    if not args.no_diff:
        result["fwd_bwd"] = diff_bench(sv, synth, torch, scene, reps=args.diff_reps)
        log(f"fwd+bwd {result['fwd_bwd']}")

    if not args.no_cpu:
        import oracle  # test infrastructure: the CPU baseline leg only

        o = oracle.OracleMap(vs, tau, 0.0, rmax, oracle.SEM_CLOSED, ncls)
        done, tcpu = 0, 0.0
        while done < len(sweeps) and tcpu < args.cpu_seconds:
            s = sweeps[done]
            c0 = time.perf_counter()
            o.integrate(s["points"], s["pose"], s["label"], oracle.IN_LABEL_I32)
            tcpu += time.perf_counter() - c0
            done += 1
        result["cpu_baseline"] = {"value": n_pts * done / tcpu, "unit": "points/s", "cores": 1, "kind": "oracle",
                                  "sample": f"sweeps 0..{done - 1} of the same street ({done} x {n_pts} points), "
                                            f"single-threaded FP64 oracle, {tcpu:.1f} s"}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
