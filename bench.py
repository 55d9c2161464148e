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
    ap.add_argument("--no-batched", action="store_true", help="skip the many-map batched measurement")
    ap.add_argument("--no-open", action="store_true", help="skip the open-set RGB-D measurement")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="also run plain device copies of this many MiB (calibrates HBM byte counters)")
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


def batched_bench(sv, synth, torch, reps=10, log_fn=log):
    """Many-map workload: 32 independent maps, one frame each with 10k-130k
    rays of a 128-beam street sweep; 16 maps 20-class closed set (int32
    labels), 16 maps 256-d open set (bf16 embeddings).  The launch shape comes
    from the autotuner.  Times, in steady state (each map already holds its
    frame once, so every voxel exists), one batched call per replay (eager and
    graph) against one plain integration per map on the same stream."""
    from paper_2512_12945_amd import autotune

    t0 = time.time()
    w = synth.batched_workload(workers=min(8, os.cpu_count() or 1))
    dev = torch.device("cuda", 0)
    frames, cfgs = [], []
    for item in w:
        if item["mode"] == "closed":
            frames.append(dict(points=torch.from_numpy(item["points"]).to(dev), pose=item["pose"],
                               sem=torch.from_numpy(item["label"]).to(dev), kind=sv.IN_LABEL_I32))
            cfgs.append(dict(voxel_size=0.1, sdf_trunc=0.3, min_range=0.0, max_range=50.0, sem_mode=sv.SEM_CLOSED,
                             num_classes=item["K"], embed_dim=0, device=0, max_leaves=1 << 15,
                             max_voxels=1 << 21))
        else:
            frames.append(dict(points=torch.from_numpy(item["points"]).to(dev), pose=item["pose"],
                               sem=torch.from_numpy(item["emb"]).to(dev), kind=sv.IN_EMB_BF16))
            cfgs.append(dict(voxel_size=0.1, sdf_trunc=0.3, min_range=0.0, max_range=50.0, sem_mode=sv.SEM_OPEN,
                             num_classes=0, embed_dim=item["L"], device=0, max_leaves=1 << 15,
                             max_voxels=1 << 21))
    torch.cuda.synchronize()
    log_fn(f"batched inputs ready in {time.time() - t0:.1f}s: {sum(x['n'] for x in w)} points over {len(w)} maps")
    shape = autotune.tune(cfgs, frames, cache_path=os.path.join(os.environ.get("TMPDIR", "/tmp"),
                                                                "slimvdb_autotune.json"), log=log_fn)
    maps = [sv.Map(**c) for c in cfgs]
    maps[0].set_launch_shape(*shape)
    for m in maps[1:]:
        m.set_launch_shape(*shape)

    def sequential():
        for m, f in zip(maps, frames):
            m.integrate(f["points"], f["pose"], f["sem"], f["kind"])

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

    t_seq = timed(sequential)
    t_eager = timed(lambda: sv.integrate_batched(maps, frames, use_graph=False))
    t_graph = timed(lambda: sv.integrate_batched(maps, frames, use_graph=True))
    st = [m.stats() for m in maps]
    npts = sum(x["n"] for x in w)
    pairs = sum(s["pairs_last"] for s in st)
    for m in maps:
        m.close()
    return {"workload": "32 maps, one street-sweep frame each with 10k-130k rays (128 beams); 16 maps 20-class "
                        "int32 labels, 16 maps 256-d bf16 embeddings; voxel 0.1 m, trunc 0.3 m; steady state",
            "points": npts, "pairs": pairs, "launch_shape": list(shape),
            "sequential_ms": t_seq, "batched_ms": t_eager, "batched_graph_ms": t_graph,
            "speedup_graph_vs_sequential": t_seq / t_graph,
            "points_per_s_graph": npts / (t_graph / 1e3)}


def run_sequence(torch, gmap, seq, W, K, sv=None):
    """Integrates seq[0:W] (warm-up) and times seq[W:W+K], three passes over a
    reset map: one with stats after every frame (the counts), one with kernel
    events (per-kernel time), one plain (the step time); with sv, a fourth
    pass integrates the timed frames with one slim_integrate_sequence call."""
    per = []
    for f in seq:
        gmap.integrate(*f)
        per.append(gmap.stats())
    gmap.reset()

    def warm():
        for f in seq[:W]:
            gmap.integrate(*f)
        torch.cuda.synchronize()

    warm()
    gmap.profile(True)
    gmap.profile_read()
    start = time.perf_counter()
    for f in seq[W:W + K]:
        gmap.integrate(*f)
    torch.cuda.synchronize()
    elapsed_events = time.perf_counter() - start
    kern = gmap.profile_read()
    gmap.profile(False)
    assert gmap.stats()["voxels"] == per[-1]["voxels"], "timed pass diverged from the counting pass"
    gmap.reset()
    warm()
    start = time.perf_counter()
    for f in seq[W:W + K]:
        gmap.integrate(*f)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - start
    assert gmap.stats()["voxels"] == per[-1]["voxels"], "timed pass diverged from the counting pass"
    out = dict(per=per, kern=kern, elapsed=elapsed, elapsed_events=elapsed_events)
    if sv is not None:
        # the same frames through slim_integrate_sequence (one call for the timed frames)
        frames = [dict(points=f[0], pose=f[1], sem=f[2], kind=f[3]) for f in seq]
        gmap.reset()
        if W:
            sv.integrate_sequence(gmap, frames[:W])
        torch.cuda.synchronize()
        start = time.perf_counter()
        sv.integrate_sequence(gmap, frames[W:W + K])
        torch.cuda.synchronize()
        out["elapsed_sequence"] = time.perf_counter() - start
        assert gmap.stats()["voxels"] == per[-1]["voxels"], "sequence pass diverged from the counting pass"
    return out


def account(timed, n_pts, b_sem, S_v):
    """Algorithmic HBM bytes of the timed frames: every point read once
    (12 B of coordinates plus b_sem of semantics), every voxel that existed read
    and written (2 S_v), every new voxel written (S_v).  Split by kernel: the
    walk reads the coordinates, the fused leaf kernel the semantics and state."""
    P = sum(s["pairs_last"] for s in timed)
    valid = sum(s["points_last"] - s["rejected_last"] for s in timed)
    u_old = sum(s["voxels_old_last"] for s in timed)
    u_new = sum(s["voxels_new_last"] for s in timed)
    K = len(timed)
    bytes_points = n_pts * K * 12
    bytes_sem = n_pts * K * b_sem
    bytes_state = u_old * 2 * S_v + u_new * S_v
    kalg = {"ray_walk_emit": bytes_points, "leaf_plan": 0, "pair_bucket": 0, "leaf_fuse": bytes_sem + bytes_state,
            "frame_commit": 0}
    return dict(pairs=P, valid=valid, u_old=u_old, u_new=u_new, kalg=kalg,
                b_alg=bytes_points + bytes_sem + bytes_state)


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (profiles/leaf_fuse_lidar_street_hbm_traffic.md), or None when the kernel
    sources changed since the counters were taken."""
    import hashlib

    root = os.path.dirname(os.path.abspath(__file__))
    try:
        text = open(os.path.join(root, "profiles", "leaf_fuse_lidar_street_hbm_traffic.md")).read()
        line = [ln for ln in text.splitlines() if ln.startswith("TRAFFIC-JSON ")][0]
        rec = json.loads(line[len("TRAFFIC-JSON "):])
        h = hashlib.sha256()
        for f in ("slimvdb_kernels.hip", "slim_internal.h"):
            h.update(open(os.path.join(root, "paper_2512_12945_amd", "csrc", f), "rb").read())
        if h.hexdigest() != rec["kernel_source_sha256"]:
            return None
        return rec["per_launch_bytes"].get(kernel)
    except (OSError, IndexError, ValueError, KeyError):
        return None


def dominant(kern, kalg, K):
    """Kernel with the most time, its achieved algorithmic GB/s (bytes per
    launch over its average event-timed duration) and its bytes per launch."""
    dom = max(kern, key=lambda k: kern[k][0])
    dom_ms, dom_n = kern[dom]
    avg_s = dom_ms / 1e3 / max(dom_n, 1)
    per_launch = kalg[dom] / K
    return dom, (per_launch / avg_s / 1e9 if avg_s > 0 else 0.0), per_launch


def open_bench(sv, synth, torch, warm=2, steps=6, log_fn=log):
    """Open-set RGB-D workload: 640x480 depth frames (307,200 points) of a room
    with 50 boxes on a 0.5 deg/frame orbit, per-pixel 512-d bf16 embeddings,
    voxel 0.02 m, trunc 0.06 m.  Integrates `warm` frames, then times `steps`
    more; reports points/s, voxel updates/s and the roofline of the dominant
    kernel as for the LiDAR sweep."""
    L = 512
    t0 = time.time()
    sc = synth.OpenRoomScene(L=L)
    fr = sc.frames(range(warm + steps), workers=min(8, os.cpu_count() or 1))
    dev = torch.device("cuda", 0)
    seq = [(torch.from_numpy(f["points"]).to(dev), f["pose"], torch.from_numpy(f["emb"]).to(dev), sv.IN_EMB_BF16)
           for f in fr]
    n_pts = fr[0]["points"].shape[0]
    del fr
    torch.cuda.synchronize()
    log_fn(f"open-set frames ready in {time.time() - t0:.1f}s")
    gmap = sv.Map(0.02, 0.06, 0.0, 10.0, sv.SEM_OPEN, 0, L, 0, max_leaves=1 << 14, max_voxels=1 << 21)
    run = run_sequence(torch, gmap, seq, warm, steps)
    gmap.close()
    acc = account(run["per"][warm:warm + steps], n_pts, 2 * L, 8 + 8 * L)
    dom, dom_gbs, dom_bytes = dominant(run["kern"], acc["kalg"], steps)
    el = run["elapsed"]
    return {"workload": "open-set RGB-D: 640x480 depth frames (307,200 points), room of 50 boxes, orbit 0.5 deg/frame, "
                        "512-d bf16 embeddings, voxel 0.02 m, trunc 0.06 m",
            "frames_timed": steps, "first_timed_frame": warm, "points_per_s": n_pts * steps / el,
            "ms_per_frame": el / steps * 1e3, "voxel_updates_per_s": acc["pairs"] / el,
            "valid_points_per_s": acc["valid"] / el, "alg_bytes_per_frame": acc["b_alg"] / steps,
            "path_roofline_frac": acc["b_alg"] / el / 1e9 / HBM_PEAK_GBS,
            "kernel_ms_per_step": {k: v[0] / max(v[1], 1) for k, v in run["kern"].items()},
            "roofline": {"kernel": dom, "bound": "hbm", "achieved": dom_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": dom_gbs / HBM_PEAK_GBS, "alg_bytes_per_launch": dom_bytes}}


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
    seq = [(pts[i], poses[i], lab[i], sv.IN_LABEL_I32) for i in range(W + K)]
    run = run_sequence(torch, gmap, seq, W, K, sv)
    gmap.close()
    # the headline is the faster of the two public paths for a stream of sweeps:
    # one slim_integrate call per sweep, or one slim_integrate_sequence call
    # (walk of sweep t + 1 beside the rest of sweep t; bitwise the same map)
    use_seq = run["elapsed_sequence"] < run["elapsed"]
    elapsed_noev = run["elapsed_sequence"] if use_seq else run["elapsed"]
    b_sem = 4  # int32 label
    acc = account(run["per"][W:W + K], n_pts, b_sem, 8 + 4 * ncls)
    dom, dom_gbs, dom_bytes = dominant(run["kern"], acc["kalg"], K)
    P, valid, b_alg = acc["pairs"], acc["valid"], acc["b_alg"]
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
                   "first_timed_sweep": W,
                   "api": "slim_integrate_sequence, all timed sweeps in one call (two-sweep passes, the default)"
                   if use_seq
                   else "slim_integrate, one call per sweep"},
        "ms_per_step_single_calls": run["elapsed"] / K * 1e3,
        "ms_per_step_sequence": run["elapsed_sequence"] / K * 1e3,
        "voxel_updates_per_s": P / elapsed_noev,
        "valid_points_per_s": valid / elapsed_noev,
        "ms_per_step_with_kernel_events": run["elapsed_events"] / K * 1e3,
        "alg_bytes_per_step": b_alg / K,
        "path_roofline_frac": (b_alg / elapsed_noev / 1e9) / HBM_PEAK_GBS,
        "kernel_ms_per_step": {k: v[0] / max(v[1], 1) for k, v in run["kern"].items()},
        "roofline": {"kernel": dom, "bound": "hbm", "achieved": dom_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": dom_gbs / HBM_PEAK_GBS, "traffic": measured_traffic(dom),
                     "alg_bytes_per_launch": dom_bytes},
    }

    if not args.no_diff:
        result["fwd_bwd"] = diff_bench(sv, synth, torch, scene, reps=args.diff_reps)
        log(f"fwd+bwd {result['fwd_bwd']}")

    if not args.no_open:
        result["open_set"] = open_bench(sv, synth, torch)
        log(f"open set {result['open_set']}")

    if not args.no_batched:
        result["batched"] = batched_bench(sv, synth, torch)
        log(f"batched {result['batched']}")

    if args.copy_calib:
        n = args.copy_calib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        result["copy_calib_bytes"] = {"read": n * 4, "write": n * 4, "launches": 5}
        del src, dst

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
