"""Render (slim_render) on the GPU against the oracle's FP64 render of its own
map: where the oracle's sign decisions are clear of ties, hit or miss, the
voxel behind the surface and its label agree exactly and the depth within the
error the D tolerance allows; elsewhere the GPU's answer must be a valid one."""
import numpy as np
import pytest
import torch

import oracle
from oracle.loss import KeyIndex
from paper_2512_12945_amd import slimvdb as sv
from paper_2512_12945_amd import synth

from _gpu_util import cuda, integrate_both, make_pair

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sv.load()


@pytest.mark.parametrize("mode", [sv.SEM_CLOSED, sv.SEM_CLOSED_LAST])
def test_render_matches_oracle(mode):
    vs, tau, K = 0.05, 0.15, 5
    print(f"render mode {mode}", flush=True)
    g, o = make_pair(vs, tau, 0.0, 100.0, mode, K)
    for fr in synth.room_sequence(4, seed=5, yaw_span=1.0, width=64, height=48, f=53.3, cx=32.0, cy=24.0):
        integrate_both(g, o, fr["points"], fr["pose"], fr["label"], sv.IN_LABEL_I32)
    pose = synth.pose_matrix(synth.camera_rotation((0.9, 0.35, -0.1)), np.array([2.0312, 1.9687, 1.4219]))
    intr, W, H, near, far = (40.0, 40.0, 39.5, 29.5), 80, 60, 0.05, 6.0
    gout = g.render(pose, intr, W, H, near, far)
    torch.cuda.synchronize()
    oout = oracle.render(o, pose, *intr, W, H, near, far)
    gd, gk, gl = (gout[k].cpu().numpy() for k in ("depth", "key", "label"))
    od, ok, ol, om = oout["depth"], oout["key"], oout["label"], oout["margin"]
    clear = om > 1e-2 * tau
    ghit, ohit = np.isfinite(gd), np.isfinite(od)
    assert np.array_equal(ghit[clear], ohit[clear])
    both = clear & ohit
    assert np.array_equal(gk[both], ok[both])
    assert np.array_equal(gl[both], ol[both])
    assert np.all(gl[~ghit] == -1)
    tol = 2e-6 * od[both] + 1e-5 * tau * np.sqrt(3.0) * vs / om[both] + 1e-6
    err = np.abs(gd[both].astype(np.float64) - od[both])
    print(f"  {both.sum()} clear hits, {(~clear).sum()} near-tie pixels; max depth error {err.max():.2e} m",
          flush=True)
    assert np.all(err <= tol)
    assert both.sum() > 0.5 * W * H
    # near-tie pixels: any GPU surface lies on an observed voxel of the oracle's map
    ex = o.extract()
    idx = KeyIndex(ex["keys"])
    sel = ~clear & ghit
    if sel.any():
        assert np.all(idx.find(gk[sel].reshape(-1, 3)) >= 0)


def test_render_empty_map_and_bad_args():
    g = sv.Map(0.1, 0.3, 0.0, 50.0, sv.SEM_CLOSED, 4, 0, 0, 1 << 10, 1 << 16)
    out = g.render(np.eye(4), (10.0, 10.0, 8.0, 6.0), 16, 12, 0.1, 20.0)
    assert torch.isnan(out["depth"]).all() and (out["label"] == -1).all()
    with pytest.raises(sv.SlimError):
        g.render(np.eye(4), (10.0, 10.0, 8.0, 6.0), 16, 12, 5.0, 1.0)
