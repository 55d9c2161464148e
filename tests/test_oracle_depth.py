"""Pins of the oracle's depth-image back-projection (RGB-D input turned into
points, Sec. III-A): exact-arithmetic bounds, the synthetic camera's own
points, and rejection of invalid depths."""
import numpy as np

import oracle
from paper_2512_12945_amd import synth


def test_backprojection_within_rounding_of_exact():
    rng = np.random.default_rng(31)
    H, W, fx, fy, cx, cy = 37, 53, 41.3, 47.9, 26.5, 17.5
    d = rng.uniform(0.3, 9.0, (H, W)).astype(np.float32)
    pts = oracle.depth_points(d, fx, fy, cx, cy).astype(np.float64)
    v, u = np.mgrid[0:H, 0:W]
    f32 = lambda x: np.float64(np.float32(x))
    ex = np.stack([(u - f32(cx)) / f32(fx) * d, (v - f32(cy)) / f32(fy) * d, d.astype(np.float64)], -1).reshape(-1, 3)
    # u - cx is exact (cx has a half-integer binary32 value); a division and a product round once each
    bound = 2.0 * 2.0 ** -24 * np.abs(ex) + 1e-30
    assert np.all(np.abs(pts - ex) <= bound)
    assert np.array_equal(pts[:, 2], d.reshape(-1).astype(np.float64))


def test_backprojection_matches_synthetic_camera():
    sc = synth.OpenRoomScene(seed=3, L=8, width=64, height=48, f=52.5, cx=31.5, cy=23.5, nboxes=10)
    fr = sc.frame(0, with_embeddings=False)
    depth = fr["points"][:, 2].reshape(48, 64)  # NaN where the camera saw nothing valid
    pts = oracle.depth_points(depth, 52.5, 52.5, 31.5, 23.5)
    ok = np.isfinite(fr["points"]).all(axis=1)
    assert np.array_equal(ok, np.isfinite(pts).all(axis=1))
    np.testing.assert_allclose(pts[ok], fr["points"][ok], rtol=4 * 2.0 ** -24, atol=0)


def test_invalid_depths_are_rejected():
    d = np.array([[1.0, 0.0, -2.0], [np.nan, np.inf, 2.5]], np.float32)
    pts = oracle.depth_points(d, 10.0, 10.0, 1.0, 0.5)
    assert np.isfinite(pts[[0, 5]]).all() and np.isnan(pts[[1, 2, 3, 4]]).all()
    m = oracle.OracleMap(0.1, 0.3, 0.0, 100.0)
    st = m.integrate(pts, np.eye(4))
    assert st["points"] == 6 and st["rejected"] == 4
