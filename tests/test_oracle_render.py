"""Pins of the oracle's render (first surface per pixel, the map-viewing role of
Sec. III-E): a planar distance field seen along a line of voxel centres (exact
closed form), and an independent FP64 re-implementation -- its own walk in
world coordinates, lookups in the extract, the same detection rule -- on a
map of integrated room frames, compared wherever the FP64 and binary32 walks
cannot differ (checked by perturbing the ray)."""
import numpy as np

import oracle
from oracle.loss import KeyIndex, walk64
from paper_2512_12945_amd import synth


def _cam_pose(position, forward):
    return synth.pose_matrix(synth.camera_rotation(forward), np.asarray(position, float))


def test_plane_along_centre_line_closed_form():
    vs, X = 0.1, 3.2371
    m = oracle.OracleMap(vs, 0.3, 0.0, 100.0, oracle.SEM_CLOSED, 3)
    keys, tsdf = [], []
    for i in range(-5, 60):
        for j in range(-8, 9):
            for k in range(-8, 9):
                keys.append((i, j, k))
                tsdf.append(X - (i + 0.5) * np.float64(np.float32(vs)))  # planar field, positive in front
    keys = np.array(keys, np.int32)
    lab = np.full(len(keys), 2, np.int32)
    m.apply(keys, np.arange(len(keys), dtype=np.uint32), np.array(tsdf), lab, oracle.IN_LABEL_I32)
    # camera at the centre of voxel (0, 0, 0) looking along +x; the principal pixel's ray runs through centres
    pose = _cam_pose((0.05, 0.05, 0.05), (1.0, 0.0, 0.0))
    out = oracle.render(m, pose, 10.0, 10.0, 2.0, 1.0, 5, 3, 0.0, 20.0)
    o_x = np.float64(np.float32(0.05 - 0.0))  # the anchor is voxel 0; the origin is 0.05 inside it
    assert abs(out["depth"][1, 2] - (X - o_x)) < 1e-12
    # centres (i + 1/2) vs: the first with D <= 0 is the first i >= X / vs - 1/2
    assert tuple(out["key"][1, 2]) == (int(np.floor(X / vs - 0.5)) + 1, 0, 0)
    assert out["label"][1, 2] == 2
    assert np.isfinite(out["depth"]).all()  # every pixel meets the plane


def _fp64_render_pixel(ex, index, pose, intr, uv, near, far, vs, maxsteps, dirot=None):
    fx, fy, cx, cy = intr
    u_, v_ = uv
    dc = np.array([(u_ - cx) / fx, (v_ - cy) / fy, 1.0])
    R = pose[:3, :3] if dirot is None else dirot @ pose[:3, :3]
    d = R @ dc
    u = d / np.linalg.norm(d)
    o = pose[:3, 3]
    cells = walk64(o, u, near, far, vs, maxsteps)
    rows = index.find(np.asarray(cells, np.int64))
    prev, margin = None, np.inf
    for k, (cell, r) in enumerate(zip(cells, rows)):
        if r < 0:
            prev = None
            continue
        D = float(ex["D"][r])
        margin = min(margin, abs(D))
        sk = float(np.dot((np.asarray(cell) + 0.5) * vs - o, u))
        if prev is not None and prev[0] > 0 and D <= 0:
            return cells[:k + 1], prev[1] + (sk - prev[1]) * prev[0] / (prev[0] - D), cell, r, margin
        prev = (D, sk)
    return cells, np.nan, None, -1, margin


def test_render_matches_independent_fp64_version():
    vs = 0.05
    m = oracle.OracleMap(vs, 0.15, 0.0, 100.0, oracle.SEM_CLOSED, 5)
    for fr in synth.room_sequence(4, seed=5, yaw_span=1.0, width=48, height=36, f=40.0, cx=24.0, cy=18.0):
        m.integrate(fr["points"], fr["pose"], fr["label"], oracle.IN_LABEL_I32)
    ex = m.extract()
    index = KeyIndex(ex["keys"])
    pose = _cam_pose((2.0312, 1.9687, 1.4219), (0.9, 0.35, -0.1))
    intr, W, H, near, far = (14.0, 14.0, 11.5, 8.5), 24, 18, 0.05, 5.0
    vs32 = float(np.float32(vs))
    maxsteps = 3 * int(np.ceil((np.float64(np.float32(far)) - np.float64(np.float32(near))) / vs32)) + 4
    out = oracle.render(m, pose, *intr, W, H, near, far)
    eps = 1e-7
    rots = []
    for ax in range(3):
        for sgn in (-1, 1):
            w = np.zeros(3)
            w[ax] = sgn * eps
            K = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
            rots.append(np.eye(3) + K)
    checked = hits = 0
    for v_ in range(H):
        for u_ in range(W):
            cells, depth, cell, r, margin = _fp64_render_pixel(ex, index, pose, intr, (u_, v_), near, far, vs32,
                                                               maxsteps)
            robust = all(_fp64_render_pixel(ex, index, pose, intr, (u_, v_), near, far, vs32, maxsteps, Rp)[0]
                         == cells for Rp in rots)
            if not robust:
                continue
            checked += 1
            if cell is None:
                assert np.isnan(out["depth"][v_, u_]) and out["label"][v_, u_] == -1
                continue
            hits += 1
            assert tuple(out["key"][v_, u_]) == tuple(cell)
            assert out["label"][v_, u_] == int(np.argmax(ex["sem"][r]))
            assert abs(out["depth"][v_, u_] - depth) <= 1e-6 * depth
            assert out["margin"][v_, u_] == margin
    assert checked > 0.9 * W * H and hits > 0.5 * W * H, (checked, hits)
