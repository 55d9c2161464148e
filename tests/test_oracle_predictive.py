"""Pins of the oracle's semantic read-out (Eq. (7), Eq. (15), the prototype
softmax and T_p of Sec. III-D) against library routines and the law of total
variance under the normal-inverse-gamma posterior."""
import numpy as np
import pytest
from scipy import special, stats
from sklearn.metrics.pairwise import cosine_similarity

from oracle import predictive as pr


def test_closed_predictive_is_dirichlet_mean():
    rng = np.random.default_rng(1)
    c = rng.integers(0, 9, (50, 7)).astype(np.float64)
    c[0] = 0.0  # unobserved voxel: the prior predictive, uniform
    for a0 in (1.0, 0.25):
        p = pr.closed_predictive(c, a0)
        for i in range(len(c)):
            np.testing.assert_allclose(p[i], stats.dirichlet.mean(a0 + c[i]), rtol=1e-14)
    np.testing.assert_allclose(pr.closed_predictive(c[:1], 1.0)[0], np.full(7, 1 / 7), rtol=1e-15)
    np.testing.assert_allclose(pr.closed_predictive(np.array([[5.0]]), 1.0), [[1.0]])  # K = 1


def test_student_t_matches_nig_total_variance():
    # lambda = 2 nu = W, beta = half the sum of squared deviations of W samples
    rng = np.random.default_rng(2)
    for W in (3, 4, 7, 30):
        z = rng.normal(0.3, 0.2, (W, 5))
        m = z.mean(axis=0, keepdims=True)
        beta = 0.5 * ((z - m) ** 2).sum(axis=0, keepdims=True)
        loc, scale2, dof, var = pr.student_t(m, beta, [W])
        lam, nu = float(W), W / 2.0
        # Var z = E[sigma^2] (1 + 1/lambda), sigma^2 ~ InvGamma(nu, beta), mu | sigma^2 ~ N(m, sigma^2 / lambda)
        e_s2 = np.array([stats.invgamma(a=nu, scale=b).mean() for b in beta[0]])
        np.testing.assert_allclose(var[0], e_s2 * (1.0 + 1.0 / lam), rtol=1e-12)
        # and the Student-t of Eq. (15) has that variance and mean m
        t = stats.t(df=dof[0], loc=loc[0], scale=np.sqrt(scale2[0]))
        np.testing.assert_allclose(t.var(), var[0], rtol=1e-12)
        np.testing.assert_allclose(t.mean(), m[0], rtol=1e-15)


def test_student_t_degenerate():
    loc, scale2, dof, var = pr.student_t(np.zeros((4, 2)), np.ones((4, 2)), [0, 1, 2, 3])
    assert np.all(np.isnan(var[:3])) and np.all(np.isfinite(var[3]))
    assert np.all(np.isnan(scale2[0])) and np.all(np.isfinite(scale2[1:]))


def test_cosine_softmax_matches_library():
    rng = np.random.default_rng(3)
    m = rng.normal(size=(40, 16))
    q = rng.normal(size=(9, 16))
    for T in (0.1, 1.0):
        want = special.softmax(cosine_similarity(m, q) / T, axis=1)
        np.testing.assert_allclose(pr.cosine_softmax(m, q, T), want, rtol=1e-12, atol=1e-300)


def test_labels_threshold_and_ties():
    p = np.array([[0.2, 0.5, 0.3], [0.4, 0.4, 0.2], [0.34, 0.33, 0.33], [0.1, 0.8, 0.1]])
    W = np.array([1.0, 2.0, 1.0, 0.0])
    assert pr.labels(p, W, 0.0).tolist() == [1, 0, 0, -1]
    assert pr.labels(p, W, 0.35).tolist() == [1, 0, -1, -1]
