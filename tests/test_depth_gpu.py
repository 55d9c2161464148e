"""Depth-image ingest (slim_integrate_depth) on the GPU: the oracle integrates
the points of its own binary32 back-projection; keys, W and counters must
match bit for bit, D and semantics within the stated tolerances, and the GPU's
depth path must equal its point path on those points bitwise."""
import numpy as np
import pytest
import torch

import oracle
from paper_2512_12945_amd import slimvdb as sv
from paper_2512_12945_amd import synth

from _gpu_util import assert_stats_equal, compare_maps, cuda, extract_np, make_pair

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sv.load()


W_, H_, F, CX, CY = 96, 72, 78.75, 47.5, 35.5


def _frames(L, n=3):
    sc = synth.OpenRoomScene(seed=9, L=L, width=W_, height=H_, f=F, cx=CX, cy=CY, nboxes=12, deg_per_frame=10.0)
    out = []
    for t in range(n):
        fr = sc.frame(t)
        depth = fr["points"][:, 2].reshape(H_, W_).copy()
        depth[0, :5] = [0.0, -1.0, np.inf, np.nan, 1e-30]  # invalid and tiny depths
        out.append((depth, fr))
    return out


@pytest.mark.parametrize("mode", ["open", "closed"])
def test_depth_matches_oracle_and_point_path(mode):
    L, K = 32, 56
    print(f"depth ingest {mode}", flush=True)
    if mode == "open":
        g, o = make_pair(0.05, 0.15, 0.0, 100.0, sv.SEM_OPEN, 0, L)
        gp = sv.Map(0.05, 0.15, 0.0, 100.0, sv.SEM_OPEN, 0, L, 0, 1 << 16, 1 << 22)
    else:
        g, o = make_pair(0.05, 0.15, 0.0, 100.0, sv.SEM_CLOSED, K)
        gp = sv.Map(0.05, 0.15, 0.0, 100.0, sv.SEM_CLOSED, K, 0, 0, 1 << 16, 1 << 22)
    intr = (F, F, CX, CY)
    for depth, fr in _frames(L):
        if mode == "open":
            sem, kind = fr["emb"], sv.IN_EMB_BF16
        else:
            sem, kind = fr["obj"].astype(np.int32), sv.IN_LABEL_I32
        pts = oracle.depth_points(depth, *intr)
        g.integrate_depth(cuda(depth), intr, fr["pose"], cuda(sem), kind)
        gp.integrate(cuda(pts), fr["pose"], cuda(sem), kind)
        ost = o.integrate(pts, fr["pose"], sem, kind)
        gst = g.stats()
        assert_stats_equal(gst, ost)
        assert gst["rejected_last"] >= 4
    gx = extract_np(g)
    compare_maps(gx, o.extract(), 0.15, sv.SEM_OPEN if mode == "open" else sv.SEM_CLOSED, K=K, L=L,
                 exact_counts=mode == "closed")
    px = extract_np(gp)
    for k in gx:
        assert np.array_equal(gx[k], px[k]), k


def test_depth_rejects_bad_arguments():
    g = sv.Map(0.05, 0.15, 0.0, 100.0, sv.SEM_NONE, 0, 0, 0, 1 << 10, 1 << 16)
    d = torch.ones((4, 5), device="cuda")
    with pytest.raises(sv.SlimError):
        g.integrate_depth(d, (0.0, 1.0, 2.0, 2.0), np.eye(4))
    with pytest.raises(sv.SlimError):
        g.integrate_depth(d, (1.0, 1.0, float("nan"), 2.0), np.eye(4))
    with pytest.raises(sv.SlimError):
        g.integrate_depth(torch.ones((4096, 4096), device="cuda"), (1.0, 1.0, 2.0, 2.0), np.eye(4))
