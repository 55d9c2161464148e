"""Pins of the oracle's loss gradient (differentiation workload) against FP64
central finite differences computed with an independent FP64 voxel walk."""
import numpy as np
import pytest

import oracle
from oracle import loss as ol
from paper_2512_12945_amd import synth

VS, TAU = 0.1, 0.3


@pytest.fixture(scope="module")
def street_loss():
    sc = synth.StreetScene(seed=2)
    frames = [sc.ray_sweep(t) for t in range(3)]
    om = oracle.OracleMap(VS, TAU, 0.0, 50.0, oracle.SEM_CLOSED, 20)
    for fr in frames:
        om.integrate(ol.rays_to_points(fr["ranges"], fr["dirs"]), fr["pose"], fr["logits"], oracle.IN_LOGIT_F32)
    ex = om.extract()
    vs = np.float64(np.float32(VS))
    y = sc.nearest_class((ex["keys"] + 0.5) * vs)
    samples = sc.surface_samples(frames, count=3000)
    lo = ol.map_loss(ex, y, samples, VS)
    return sc, frames, om, ex, lo


def test_loss_terms_positive_and_consistent(street_loss):
    _, _, _, ex, lo = street_loss
    assert lo["Mp"] > 2000 and lo["M"] == len(ex["W"])
    assert lo["ce"] > 0 and lo["l1"] > 0
    # sum of adjoint counts equals the valid samples
    assert lo["cnt"].sum() == lo["Mp"]


def test_softmax_jacobian_rows_sum_to_zero(street_loss):
    _, frames, om, ex, lo = street_loss
    g_logit, g_r, _ = ol.frame_gradients(om, frames[1], ex, lo)
    scale = np.abs(g_logit).max()
    assert np.abs(g_logit.sum(axis=1)).max() < 1e-12 * max(scale, 1e-300) * 20
    assert np.all(g_r[~np.isfinite(frames[1]["ranges"])] == 0)


def test_fd_matches_analytic(street_loss):
    """256 points (as the differentiation workload states).  Central
    differences (h = 1e-6) of the local loss of a point, with the
    point's voxels recomputed by an FP64 walk; points whose FP64 voxel set differs
    from the binary32 one, changes under +-h, or sits near a clamp, gate or sign
    kink are redrawn."""
    sc, frames, om, ex, lo = street_loss
    index = ol.KeyIndex(ex["keys"])
    fr = frames[1]
    g_logit, g_r, pr = ol.frame_gradients(om, fr, ex, lo, index)
    vs, tau = om.voxel_size, om.sdf_trunc
    h = 1e-6
    rng = np.random.default_rng(5)
    cand = rng.permutation(np.nonzero(np.isfinite(fr["ranges"]))[0])
    gl_scale, gr_scale = np.abs(g_logit).max(), np.abs(g_r).max()
    checked, redrawn, worst = 0, 0, 0.0
    for j in cand:
        if checked == 256:
            break
        mine = pr["pid"] == j
        cells32 = sorted(map(tuple, pr["keys"][mine].tolist()))
        base = ol.kept_cells64(fr, j, vs, tau, om.maxsteps)
        plus = ol.kept_cells64(fr, j, vs, tau, om.maxsteps, r=float(fr["ranges"][j]) + h)
        minus = ol.kept_cells64(fr, j, vs, tau, om.maxsteps, r=float(fr["ranges"][j]) - h)
        same = [cl for cl, _, _ in base] == [cl for cl, _, _ in plus] == [cl for cl, _, _ in minus]
        rows = index.find(np.asarray([cl for cl, _, _ in base], np.int64)) if base else np.array([-1])
        stable = (sorted(cl for cl, _, _ in base) == cells32 and same and np.all(rows >= 0)
                  and all(abs(s - tau) > 1e-4 and abs(s + tau) > 1e-4 for _, _, s in base)
                  and np.all(np.abs(np.asarray(ex["D"])[rows]) > 1e-4))
        if not stable:
            redrawn += 1
            continue
        cells = [(cl, ts) for cl, ts, _ in base]
        ts0 = [ts for _, ts in cells]
        l0 = np.asarray(fr["logits"][j], np.float64)
        # a central difference of a sum of magnitude |L| carries a rounding error
        # of a few ulp(|L|) / (2h); the comparison allows that bound on top of 1e-6
        eps = np.finfo(np.float64).eps
        Lj = ol.local_loss(ex, lo, index, fr, j, l0, cells, ts0)
        fd_noise = 16 * eps * abs(Lj) / (2 * h)
        for k in (int(np.argmax(l0)), int(rng.integers(0, 20))):
            e = np.zeros(20)
            e[k] = h
            fd = (ol.local_loss(ex, lo, index, fr, j, l0 + e, cells, ts0)
                  - ol.local_loss(ex, lo, index, fr, j, l0 - e, cells, ts0)) / (2 * h)
            err = abs(fd - g_logit[j, k]) / (max(abs(g_logit[j, k]), 1e-3 * gl_scale) * 1e-6 + fd_noise) * 1e-6
            worst = max(worst, err)
            assert err < 1e-6, (j, k, fd, g_logit[j, k], fd_noise)
        cp = [(cl, ts) for cl, ts, _ in plus]
        cm = [(cl, ts) for cl, ts, _ in minus]
        fd = (ol.local_loss(ex, lo, index, fr, j, l0, cp, ts0) - ol.local_loss(ex, lo, index, fr, j, l0, cm, ts0)) / (2 * h)
        err = abs(fd - g_r[j]) / (max(abs(g_r[j]), 1e-3 * gr_scale) * 1e-6 + fd_noise) * 1e-6
        worst = max(worst, err)
        assert err < 1e-6, (j, fd, g_r[j], fd_noise)
        checked += 1
    assert checked == 256, (checked, redrawn)
    print(f"FD check: {checked} points, {redrawn} redrawn, worst relative error {worst:.2e}")


def test_labels_outside_classes_add_nothing(street_loss):
    """A ground-truth label outside [0, K) adds no cross-entropy term and no
    dL/dc; the mean still divides by every listed voxel.  Checked against the
    valid voxels' terms computed directly from the Dirichlet predictive."""
    _, _, _, ex, lo = street_loss
    y = lo["y"].copy()
    rng = np.random.default_rng(11)
    bad = rng.random(len(y)) < 0.3
    y[bad] = np.where(rng.random(int(bad.sum())) < 0.5, -1, 20)
    lo2 = ol.map_loss(ex, y, np.zeros((0, 3), np.float32), VS)
    c = np.asarray(ex["sem"], np.float64)
    ok = ~bad
    p = (1.0 + c[ok, lo["y"][ok]]) / (20.0 + c[ok].sum(axis=1))
    assert abs(lo2["ce"] - (-np.log(p)).sum() / len(y)) <= 1e-12 * lo2["ce"]
    assert np.all(lo2["adj_c"][bad] == 0.0)
    assert np.array_equal(lo2["adj_c"][ok], lo["adj_c"][ok])
