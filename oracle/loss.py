"""FP64 map loss and gradients of the differentiation workload.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The loss of a map integrated from several frames of (range, direction, logits)
rays is

    L = (1/|V|) sum_v  -log p_v(y_v)          closed-set predictive, Eq. (7),
                                              p_v(i) = (a0 + c_vi) / (K a0 + sum_i c_vi)
      + (1/M') sum_s |D(v_s)|                 TSDF at surface samples

over all voxels v of the map (y_v the ground-truth class; a voxel whose label
is outside [0, K) contributes no cross-entropy term, but still counts in
1/|V|) and the M' surface samples s whose voxel v_s is in the map.  The map is
the batch conjugate posterior of all observations (Thm. 1; Eq. (1)-(2) with
unit weights), so

    c_vi = sum over observations j of v of softmax(l_j)_i
    D_v  = (sum over observations j of v of tsdf_j) / W_v

and the gradient of L with respect to a point's logits and range follows by
the chain rule through the softmax and through tsdf = min(sdf, tau), where
d sdf / d r = 1 along the fixed ray direction (p = o + r u).  The clamp's
derivative is decided on the binary32 signed distance, as the gate is.  The
gradient w.r.t. D uses sign(0) = 0.
"""
from __future__ import annotations

import numpy as np

from . import IN_LOGIT_F32


def rays_to_points(ranges, dirs):
    """Sensor-frame points r * dir, one binary32 product per component."""
    r = np.asarray(ranges, np.float32)
    d = np.asarray(dirs, np.float32).reshape(-1, 3)
    return (r[:, None] * d).astype(np.float32)


def softmax64(l):
    l = np.asarray(l, np.float64)
    e = np.exp(l - l.max(axis=-1, keepdims=True))
    return e / e.sum(axis=-1, keepdims=True)


def _pack(keys):
    k = np.asarray(keys, np.int64) + (1 << 20)
    return (k[:, 0] << 42) | (k[:, 1] << 21) | k[:, 2]


class KeyIndex:
    """Row of each voxel key in an extract."""

    def __init__(self, keys):
        packed = _pack(keys)
        self.order = np.argsort(packed, kind="stable")
        self.sorted = packed[self.order]

    def find(self, keys):
        q = _pack(keys)
        i = np.searchsorted(self.sorted, q)
        i = np.minimum(i, len(self.sorted) - 1)
        hit = (len(self.sorted) > 0) & (self.sorted[i] == q)
        return np.where(hit, self.order[i], -1)


def sample_keys(samples, voxel_size):
    """Voxel of each world sample: floor(x / vs) with a binary32 division."""
    s = np.asarray(samples, np.float32)
    return np.floor(s / np.float32(voxel_size)).astype(np.int64)


def map_loss(ex, y, samples, voxel_size, alpha0=1.0):
    """Loss and per-voxel adjoints dL/dc (M x K) and dL/dD (M) of an extracted map."""
    c = np.asarray(ex["sem"], np.float64)
    D = np.asarray(ex["D"], np.float64)
    M, K = c.shape
    y = np.asarray(y, np.int64)
    tot = K * alpha0 + c.sum(axis=1)
    # a ground-truth label outside [0, K) adds no cross-entropy term and no
    # dL/dc; the mean still runs over all M listed voxels
    ok = (y >= 0) & (y < K)
    yy = np.where(ok, y, 0)
    cy = c[np.arange(M), yy]
    ce = np.where(ok, -np.log((alpha0 + cy) / tot), 0.0)
    adj_c = np.repeat((1.0 / tot)[:, None], K, axis=1)
    adj_c[np.arange(M), yy] -= 1.0 / (alpha0 + cy)
    adj_c[~ok] = 0.0
    adj_c /= M
    idx = KeyIndex(ex["keys"]).find(sample_keys(samples, voxel_size))
    valid = idx >= 0
    Mp = int(valid.sum())
    cnt = np.bincount(idx[valid], minlength=M).astype(np.float64)
    l1 = np.abs(D[idx[valid]]).sum() / max(Mp, 1)
    adj_D = cnt * np.sign(D) / max(Mp, 1)
    return dict(loss=ce.mean() + l1, ce=ce.mean(), l1=l1, adj_c=adj_c, adj_D=adj_D, M=M, Mp=Mp, cnt=cnt, y=y)


def frame_gradients(omap, frame, ex, lo, index=None):
    """dL/dlogits (N x K) and dL/drange (N) of one frame, from the adjoints of
    map_loss `lo`.  `omap` supplies the frame's observation pairs (the same
    decision path that built the map)."""
    pts = rays_to_points(frame["ranges"], frame["dirs"])
    logits = np.asarray(frame["logits"], np.float32)
    pr = omap.frame_pairs(pts, frame["pose"], logits, IN_LOGIT_F32)
    index = index or KeyIndex(ex["keys"])
    v = index.find(pr["keys"])
    assert np.all(v >= 0), "every observed voxel is in the map"
    N, K = logits.shape
    G = np.zeros((N, K))
    np.add.at(G, pr["pid"], lo["adj_c"][v])
    p = softmax64(logits)
    g_logit = p * (G - (p * G).sum(axis=1, keepdims=True))
    sel = pr["sdf32"] < np.float32(omap.sdf_trunc)
    g_r = np.zeros(N)
    np.add.at(g_r, pr["pid"][sel], lo["adj_D"][v[sel]] / np.asarray(ex["W"], np.float64)[v[sel]])
    return g_logit, g_r, pr


# ---------------------------------------------------------------------------
# FP64-everywhere finite differences (independent of the binary32 decision path)
# ---------------------------------------------------------------------------


def walk64(o, u, t0, t1, vs, maxsteps):
    """Amanatides-Woo walk in FP64 over [t0, t1] of the ray o + t u (world
    coordinates, voxel size vs); ties step the lowest axis first."""
    c = [int(np.floor((o[a] + t0 * u[a]) / vs)) for a in range(3)]
    tm, td, st = [0.0] * 3, [0.0] * 3, [0] * 3
    for a in range(3):
        s = o[a] + t0 * u[a]
        if u[a] > 0:
            st[a], tm[a], td[a] = 1, t0 + ((c[a] + 1) * vs - s) / u[a], vs / u[a]
        elif u[a] < 0:
            st[a], tm[a], td[a] = -1, t0 + (c[a] * vs - s) / u[a], -vs / u[a]
        else:
            st[a], tm[a], td[a] = 0, np.inf, np.inf
    cells = []
    for _ in range(maxsteps):
        cells.append(tuple(c))
        ax = int(np.argmin(tm))
        if tm[ax] > t1:
            break
        c[ax] += st[ax]
        tm[ax] += td[ax]
    return cells


def ray64(frame, j, r=None):
    """FP64 geometry of point j: origin, unit direction, range along it."""
    R, t = np.asarray(frame["pose"])[:3, :3], np.asarray(frame["pose"])[:3, 3]
    d = R @ np.asarray(frame["dirs"][j], np.float64)
    rr = float(frame["ranges"][j]) if r is None else r
    n = np.linalg.norm(d)
    return t, d / n, rr * n


def kept_cells64(frame, j, vs, tau, maxsteps, r=None):
    """(cell, tsdf) of point j's band in FP64: cells whose projective signed
    distance exceeds -tau, tsdf = min(sdf, tau)."""
    o, u, rr = ray64(frame, j, r)
    p = o + rr * u
    out = []
    for cell in walk64(o, u, max(rr - tau, 0.0), rr + tau, vs, maxsteps):
        centre = (np.asarray(cell, np.float64) + 0.5) * vs
        s = float(np.dot(p - centre, u))
        if s > -tau:
            out.append((cell, min(s, tau), s))
    return out


def local_loss(ex, lo, index, frame, j, logits_j, cells, tsdf0, alpha0=1.0):
    """Loss terms of the voxels on point j's ray, with point j's contribution
    replaced: logits_j (K,) and the cells' tsdf values (list aligned with
    `cells`, which must be the voxels it observed in the map)."""
    rows = index.find(np.asarray([cl for cl, _ in cells], np.int64))
    c = np.asarray(ex["sem"], np.float64)[rows]
    D = np.asarray(ex["D"], np.float64)[rows]
    W = np.asarray(ex["W"], np.float64)[rows]
    K = c.shape[1]
    p0 = softmax64(np.asarray(frame["logits"][j], np.float64))
    p1 = softmax64(np.asarray(logits_j, np.float64))
    c = c - p0 + p1
    D = D + (np.asarray([ts for _, ts in cells]) - np.asarray(tsdf0)) / W
    y = lo["y"][rows]
    tot = K * alpha0 + c.sum(axis=1)
    ce = -np.log((alpha0 + c[np.arange(len(rows)), y]) / tot)
    return ce.sum() / lo["M"] + (lo["cnt"][rows] * np.abs(D)).sum() / max(lo["Mp"], 1)
