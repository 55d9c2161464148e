"""Semantic read-out (slim_predict) on the GPU against the oracle's FP64
read-out: Dirichlet predictive (Eq. (7)), prototype softmax, Student-t
variance (Eq. (15)), labels with the threshold, unobserved and invalid points."""
import numpy as np
import pytest
import torch

import oracle
from oracle import predictive as opred
from oracle.loss import KeyIndex, sample_keys
from paper_2512_12945_amd import slimvdb as sv
from paper_2512_12945_amd import synth

from _gpu_util import cuda, extract_np, integrate_both, make_pair

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sv.load()


def _queries(ox, vs, rng, extra=500):
    """Voxel centres of the map, random points around it (many unobserved), and a NaN point."""
    vs32 = np.float32(vs)
    cent = ((ox["keys"].astype(np.float32) + np.float32(0.5)) * vs32).astype(np.float32)
    lo, hi = cent.min(axis=0), cent.max(axis=0)
    rnd = rng.uniform(lo - 1.0, hi + 1.0, (extra, 3)).astype(np.float32)
    q = np.concatenate([cent, rnd, np.array([[np.nan, 0.0, 0.0]], np.float32)])
    idx = KeyIndex(ox["keys"]).find(np.where(np.isfinite(q), sample_keys(np.nan_to_num(q), vs), 0))
    idx[~np.isfinite(q).all(axis=1)] = -1
    return q, idx


def _check_labels(lab_g, p_o, W_o, threshold, rtol=1e-5):
    """Labels agree where the oracle's decision is clear; elsewhere the GPU's is valid."""
    top = p_o.max(axis=1)
    tol = rtol * np.maximum(top, 1e-3)
    want = opred.labels(p_o, W_o, threshold)
    srt = np.sort(p_o, axis=1)
    clear = (srt[:, -1] - srt[:, -2] > tol) & (np.abs(top - threshold) > tol)
    assert np.array_equal(lab_g[clear], want[clear])
    for i in np.flatnonzero(~clear):
        if lab_g[i] >= 0:
            assert p_o[i, lab_g[i]] >= top[i] - tol[i] and top[i] >= threshold - tol[i]
        else:
            assert W_o[i] <= 0 or top[i] <= threshold + tol[i]
    return int((~clear).sum())


def test_predict_closed():
    K, vs = 20, 0.1
    g, o = make_pair(vs, 0.3, 0.0, 50.0, sv.SEM_CLOSED, K)
    sc = synth.StreetScene(seed=2)
    for t in range(3):
        fr = sc.sweep(t, nrays=20_000)
        integrate_both(g, o, fr["points"], fr["pose"], fr["label"], sv.IN_LABEL_I32)
    ox = o.extract()
    q, idx = _queries(ox, vs, np.random.default_rng(21))
    for a0, thr in ((1.0, 0.0), (0.5, 0.6)):
        out = g.predict(cuda(q), alpha0=a0, threshold=thr)
        p_g, lab_g = out["prob"].cpu().numpy().astype(np.float64), out["label"].cpu().numpy()
        c = np.where(idx[:, None] >= 0, ox["sem"][np.maximum(idx, 0)], 0.0)
        p_o = opred.closed_predictive(c, a0)
        W_o = np.where(idx >= 0, ox["W"][np.maximum(idx, 0)], 0.0)
        err = np.abs(p_g - p_o) / np.maximum(p_o, 1e-3)
        print(f"closed alpha0 {a0}: max rel err {err.max():.2e}", flush=True)
        assert err.max() <= 1e-5
        nf = _check_labels(lab_g, p_o, W_o, thr)
        print(f"  labels checked, {nf} near-ties validated", flush=True)
        assert np.all(lab_g[idx < 0] == -1)


def test_predict_open_and_variance():
    L, vs = 64, 0.05
    sc = synth.OpenRoomScene(seed=9, L=L, width=80, height=60, f=65.6, cx=39.5, cy=29.5, nboxes=12,
                             deg_per_frame=10.0)
    g, o = make_pair(vs, 0.15, 0.0, 100.0, sv.SEM_OPEN, 0, L)
    for t in range(4):
        fr = sc.frame(t)
        integrate_both(g, o, fr["points"], fr["pose"], fr["emb"], sv.IN_EMB_BF16)
    ox = o.extract()
    q, idx = _queries(ox, vs, np.random.default_rng(22))
    protos = sc.proto.astype(np.float32)
    T, thr = 0.1, 0.1
    out = g.predict(cuda(q), temperature=T, threshold=thr, prototypes=cuda(protos), var=True)
    p_g, lab_g = out["prob"].cpu().numpy().astype(np.float64), out["label"].cpu().numpy()
    v_g = out["var"].cpu().numpy().astype(np.float64)
    obs = idx >= 0
    m_o, b_o, W_o = ox["sem"][idx[obs], :L], ox["sem"][idx[obs], L:], ox["W"][idx[obs]]
    p_o = np.zeros_like(p_g)
    p_o[obs] = opred.cosine_softmax(m_o, protos.astype(np.float64), T)
    err = np.abs(p_g - p_o) / np.maximum(p_o, 1e-3)
    print(f"open: max rel err of class probabilities {err.max():.2e}", flush=True)
    assert err.max() <= 1e-4
    Wq = np.where(obs, ox["W"][np.maximum(idx, 0)], 0.0)
    nf = _check_labels(lab_g, p_o, Wq, thr, rtol=1e-4)
    print(f"  labels checked, {nf} near-ties validated", flush=True)
    _, _, _, var_o = opred.student_t(m_o, b_o, W_o)
    fin = np.isfinite(var_o)
    assert np.array_equal(np.isfinite(v_g[obs]), fin)
    assert np.all(np.isnan(v_g[~obs]))
    # beta carries the 1e-4 tolerance of the integration; the read-out adds a few roundings
    Wc = W_o[:, None] * np.ones_like(var_o)
    floor = 1e-3 * 2.0 * (Wc + 1.0) / np.maximum(Wc - 2.0, 1.0)  # the beta floor 1e-3 W, carried through
    verr = np.abs(v_g[obs][fin] - var_o[fin]) / np.maximum(var_o, floor)[fin]
    print(f"  Student-t variance: max rel err {verr.max(initial=0):.2e} over {fin.sum()} components", flush=True)
    assert verr.max(initial=0) <= 2e-4


def test_predict_last_modes():
    K, vs = 8, 0.1
    g, o = make_pair(vs, 0.3, 0.0, 50.0, sv.SEM_CLOSED_LAST, K)
    sc = synth.StreetScene(seed=2)
    rng = np.random.default_rng(23)
    for t in range(2):
        fr = sc.sweep(t, nrays=10_000)
        integrate_both(g, o, fr["points"], fr["pose"], rng.integers(0, K, fr["points"].shape[0]).astype(np.int32),
                       sv.IN_LABEL_I32)
    ox = o.extract()
    q, idx = _queries(ox, vs, rng)
    out = g.predict(cuda(q), threshold=0.5)
    lab = out["label"].cpu().numpy()
    want = np.where(idx >= 0, ox["sem"][np.maximum(idx, 0), 0], -1).astype(np.int64)
    assert np.array_equal(lab, want)
    p = out["prob"].cpu().numpy()
    assert np.array_equal(p.argmax(axis=1)[idx >= 0], want[idx >= 0]) and np.all(p.sum(axis=1)[idx >= 0] == 1.0)
    with pytest.raises(sv.SlimError):
        g.predict(cuda(q), var=True)


def test_predict_rejects_bad_params():
    g = sv.Map(0.1, 0.3, 0.0, 50.0, sv.SEM_CLOSED, 4, 0, 0, 1 << 10, 1 << 16)
    q = torch.zeros((4, 3), device="cuda")
    with pytest.raises(sv.SlimError):
        g.predict(q, alpha0=0.0)
    go = sv.Map(0.1, 0.3, 0.0, 50.0, sv.SEM_OPEN, 0, 8, 0, 1 << 10, 1 << 16)
    with pytest.raises(sv.SlimError):
        go.predict(q, temperature=0.0, prototypes=torch.ones((3, 8), device="cuda"))
    gn = sv.Map(0.1, 0.3, 0.0, 50.0, sv.SEM_NONE, 0, 0, 0, 1 << 10, 1 << 16)
    with pytest.raises(sv.SlimError):
        gn.predict(q)
