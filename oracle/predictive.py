"""FP64 read-out of a map's semantic posterior at query time.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Closed set: the posterior predictive of the Dirichlet over class probabilities
(Eq. (7)) with a symmetric prior alpha0 added to the stored counts c:
p_i = (alpha0 + c_i) / (K alpha0 + sum_i c_i).

Open set: each embedding component has the Student-t predictive of Eq. (15)
with 2 nu = lambda = W (Sec. III-D): location m, squared scale
beta (lambda + 1) / (lambda nu) = 2 beta (W + 1) / W^2 and 2 nu = W degrees
of freedom; its variance (dof / (dof - 2)) scale^2 = 2 beta (W + 1) / (W (W - 2))
exists for W > 2 (the paper states the conditions on lambda; with lambda = 2 nu
they are the degrees-of-freedom conditions).  Class probabilities: a softmax
over the cosine similarities between the predictive mean and class prototypes,
divided by a temperature; a voxel whose largest class probability is below the
threshold T_p (0.1 in Sec. III-D) gets no label.

Labels are the first index of the largest probability; unobserved voxels
(W = 0) get label -1.
"""
from __future__ import annotations

import numpy as np


def closed_predictive(counts, alpha0=1.0):
    c = np.asarray(counts, np.float64)
    K = c.shape[1]
    return (alpha0 + c) / (K * alpha0 + c.sum(axis=1, keepdims=True))


def student_t(m, beta, W):
    """(location, squared scale, degrees of freedom, variance) per component;
    variance NaN where W <= 2, everything NaN where W = 0."""
    m = np.asarray(m, np.float64)
    b = np.asarray(beta, np.float64)
    W = np.asarray(W, np.float64)[:, None]
    lam, nu = W, W / 2.0
    with np.errstate(divide="ignore", invalid="ignore"):
        scale2 = b * (lam + 1.0) / (lam * nu)
        dof = np.broadcast_to(2.0 * nu, b.shape)
        var = np.where(dof > 2.0, dof / (dof - 2.0) * scale2, np.nan)
    scale2 = np.where(W > 0, scale2, np.nan)
    return m, scale2, dof, var


def cosine_softmax(mean, prototypes, temperature):
    """Class probabilities: softmax over cos(mean, prototype_j) / temperature."""
    m = np.asarray(mean, np.float64)
    q = np.asarray(prototypes, np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        cos = (m @ q.T) / (np.linalg.norm(m, axis=1, keepdims=True) * np.linalg.norm(q, axis=1)[None, :])
    s = cos / temperature
    e = np.exp(s - s.max(axis=1, keepdims=True))
    return e / e.sum(axis=1, keepdims=True)


def labels(prob, W, threshold=0.0):
    """First argmax, or -1 where unobserved or below the threshold."""
    prob = np.asarray(prob, np.float64)
    lab = np.argmax(prob, axis=1).astype(np.int64)
    top = prob.max(axis=1)
    lab[(np.asarray(W) <= 0) | ~(top >= threshold)] = -1
    return lab
