"""Helpers shared by the GPU parity tests: run the HIP path and the oracle on
the same seeded inputs and compare them (keys and W bit-exact; D within 1e-5
relative to max(|D|, tau); closed-set predictive within 1e-5 relative; open-set
mean and scatter within 1e-4 relative, see compare_maps)."""
import numpy as np
import torch

import oracle
from paper_2512_12945_amd import slimvdb as sv

ALPHA0 = 1.0


def cuda(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def make_pair(voxel_size, sdf_trunc, min_range=0.0, max_range=100.0, sem_mode=sv.SEM_NONE, K=0, L=0,
              max_leaves=1 << 16, max_voxels=1 << 22):
    g = sv.Map(voxel_size, sdf_trunc, min_range, max_range, sem_mode, K, L, 0, max_leaves, max_voxels)
    o = oracle.OracleMap(voxel_size, sdf_trunc, min_range, max_range, sem_mode, K, L)
    return g, o


def integrate_both(g, o, pts, pose, sem=None, kind=sv.IN_NONE):
    sem_t = None
    if sem is not None:
        sem_t = cuda(sem)
    g.integrate(cuda(pts), pose, sem_t, kind)
    ost = o.integrate(pts, pose, sem, kind)
    gst = g.stats()
    return gst, ost


def assert_stats_equal(gst, ost):
    assert gst["status_last"] == 0
    pairs = {"points_last": "points", "rejected_last": "rejected", "pairs_last": "pairs",
             "voxels_old_last": "u_old", "voxels_new_last": "u_new", "new_leaves_last": "new_leaves",
             "voxels": "voxels", "leaves": "leaves"}
    for gk, ok in pairs.items():
        assert gst[gk] == ost[ok], (gk, gst[gk], ost[ok])


def extract_np(g):
    ex = g.extract()
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in ex.items()}


def compare_maps(gx, ox, tau, sem_mode, K=0, L=0, exact_counts=False):
    """Keys and W bit-exact; D within 1e-5 max(|D|, tau); closed-set posterior
    predictive within 1e-5 max(p, 1e-3) (counts bit-exact for one-hot input);
    open-set m within 1e-4 max(|m|, max|m| of the voxel), beta within
    1e-4 max(beta, 1e-3 W).  Returns the observed worst errors."""
    assert gx["keys"].shape == ox["keys"].shape, (gx["keys"].shape, ox["keys"].shape)
    assert np.array_equal(gx["keys"], ox["keys"])
    assert np.array_equal(gx["W"].astype(np.float64), ox["W"])
    err = {}
    dD = np.abs(gx["D"].astype(np.float64) - ox["D"]) / np.maximum(np.abs(ox["D"]), tau)
    err["D"] = float(dD.max(initial=0))
    assert err["D"] <= 1e-5, err
    if sem_mode == sv.SEM_CLOSED:
        c_g = gx["sem"].astype(np.float64)
        c_o = ox["sem"]
        if exact_counts:
            assert np.array_equal(c_g, c_o)
        p_g = (ALPHA0 + c_g) / (K * ALPHA0 + c_g.sum(axis=1, keepdims=True))
        p_o = (ALPHA0 + c_o) / (K * ALPHA0 + c_o.sum(axis=1, keepdims=True))
        dp = np.abs(p_g - p_o) / np.maximum(p_o, 1e-3)
        err["p"] = float(dp.max(initial=0))
        dc = np.abs(c_g - c_o) / np.maximum(np.abs(c_o), 1.0)
        err["c"] = float(dc.max(initial=0))
        assert err["p"] <= 1e-5, err
        assert err["c"] <= 1e-5, err
    elif sem_mode == sv.SEM_OPEN:
        m_g, b_g = gx["sem"][:, :L].astype(np.float64), gx["sem"][:, L:].astype(np.float64)
        m_o, b_o = ox["sem"][:, :L], ox["sem"][:, L:]
        scale = np.maximum(np.abs(m_o), np.abs(m_o).max(axis=1, keepdims=True))
        err["m"] = float((np.abs(m_g - m_o) / np.maximum(scale, 1e-30)).max(initial=0))
        bscale = np.maximum(b_o, 1e-3 * ox["W"][:, None])
        err["beta"] = float((np.abs(b_g - b_o) / bscale).max(initial=0))
        assert err["m"] <= 1e-4, err
        assert err["beta"] <= 1e-4, err
    return err
