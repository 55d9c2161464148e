"""Non-Bayesian mode (SLIM-VDB* of Sec. IV) on the GPU against the oracle:
keys, W and the stored class index or embedding bit-exact, D within the
Eq. (1)-(2) tolerance, and D, W bitwise equal to the Bayesian map's."""
import numpy as np
import pytest
import torch

import oracle
from paper_2512_12945_amd import slimvdb as sv
from paper_2512_12945_amd import synth

from _gpu_util import assert_stats_equal, compare_maps, cuda, extract_np, integrate_both, make_pair

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sv.load()


def _street(n_frames=3, nrays=20_000):
    sc = synth.StreetScene(seed=2)
    return [sc.sweep(t, nrays=nrays) for t in range(n_frames)]


@pytest.mark.parametrize("kind", [sv.IN_LABEL_I32, sv.IN_PROB_F32, sv.IN_LOGIT_F32])
def test_last_closed_matches_oracle(kind):
    K = 20
    print(f"last closed kind {kind}", flush=True)
    g, o = make_pair(0.1, 0.3, 0.0, 50.0, sv.SEM_CLOSED_LAST, K)
    gb = sv.Map(0.1, 0.3, 0.0, 50.0, sv.SEM_CLOSED, K, 0, 0, 1 << 16, 1 << 22)
    rng = np.random.default_rng([11, kind])
    for fr in _street():
        n = fr["points"].shape[0]
        if kind == sv.IN_LABEL_I32:
            sem = fr["label"]
        else:
            x = rng.integers(0, 4, (n, K)).astype(np.float32)  # many exact ties
            sem = x / np.float32(3.0) if kind == sv.IN_PROB_F32 else x
        gst, ost = integrate_both(g, o, fr["points"], fr["pose"], sem, kind)
        assert_stats_equal(gst, ost)
        gb.integrate(cuda(fr["points"]), fr["pose"], cuda(sem), kind)
    gx, ox = extract_np(g), o.extract()
    compare_maps(gx, ox, 0.3, sv.SEM_CLOSED_LAST)
    assert np.array_equal(gx["sem"][:, 0].astype(np.float64), ox["sem"][:, 0])
    bx = extract_np(gb)
    assert np.array_equal(gx["D"], bx["D"]) and np.array_equal(gx["W"], bx["W"])


@pytest.mark.parametrize("kind,L", [(sv.IN_EMB_BF16, 64), (sv.IN_EMB_F32, 40)])
def test_last_open_matches_oracle(kind, L):
    print(f"last open kind {kind} L {L}", flush=True)
    sc = synth.OpenRoomScene(seed=9, L=L, width=80, height=60, f=65.6, cx=39.5, cy=29.5, nboxes=12,
                             deg_per_frame=10.0)
    g, o = make_pair(0.05, 0.15, 0.0, 100.0, sv.SEM_OPEN_LAST, 0, L)
    for t in range(3):
        fr = sc.frame(t)
        z = fr["emb"] if kind == sv.IN_EMB_BF16 else synth.bf16_bits_to_float(fr["emb"]) * np.float32(1.25)
        gst, ost = integrate_both(g, o, fr["points"], fr["pose"], z, kind)
        assert_stats_equal(gst, ost)
    gx, ox = extract_np(g), o.extract()
    compare_maps(gx, ox, 0.15, sv.SEM_OPEN_LAST)
    assert np.array_equal(gx["sem"].astype(np.float64), ox["sem"])


def test_last_modes_reject_loss():
    g = sv.Map(0.1, 0.3, 0.0, 50.0, sv.SEM_CLOSED_LAST, 5, 0, 0, 1 << 10, 1 << 16)
    keys = torch.zeros((1, 3), dtype=torch.int32, device="cuda")
    with pytest.raises(sv.SlimError):
        g.loss(keys, torch.zeros(1, dtype=torch.int32, device="cuda"), torch.zeros((1, 3), device="cuda"), 1.0)
