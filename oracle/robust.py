"""Huber robust loss by iteratively reweighted least squares (oracle; test
infrastructure).

Not part of the paper, whose objective is plain squared loss (Sec. 4,
F(x) = 1/2 sum ||r_i||^2).  Added for the outlier workload.  Reading used:
the loss acts on s = ||r_i||^2 of the 2-D residual,

    rho(s) = s                      for s <= delta^2
    rho(s) = 2 delta sqrt(s) - delta^2   otherwise,

F = 1/2 sum rho(s_i), and each LM linearisation scales the residual and its
Jacobian rows by sqrt(w_i) with w_i = rho'(s_i) = min(1, delta / ||r_i||)
(no second-order correction term).
"""
from __future__ import annotations

import math

import numpy as np


def rho(s, delta):
    s = np.asarray(s, dtype=np.float64)
    return np.where(s <= delta * delta, s, 2.0 * delta * np.sqrt(s) - delta * delta)


def weight(s, delta):
    """rho'(s)."""
    s = np.asarray(s, dtype=np.float64)
    return np.where(s <= delta * delta, 1.0, delta / np.sqrt(np.maximum(s, 1e-300)))


def cost(r, delta=None):
    """F = 1/2 sum rho(||r_i||^2) with a correctly rounded sum (math.fsum).
    delta None means the plain squared loss of Sec. 4.  A sum beyond the
    float64 range is +inf (a trial state whose cost is not finite is then
    rejected by the LM loop), and a NaN term gives NaN."""
    s = np.sum(np.asarray(r, dtype=np.float64) ** 2, axis=1)
    terms = s if delta is None else rho(s, delta)
    try:
        return 0.5 * math.fsum(terms.tolist())
    except OverflowError:  # finite terms whose exact sum exceeds the float64 range
        return math.inf


def reweight(r, Jp, Jl, delta=None):
    """IRLS: returns sqrt(w) r, sqrt(w) J_p, sqrt(w) J_l and w."""
    if delta is None:
        return r, Jp, Jl, np.ones(r.shape[0])
    s = np.sum(r * r, axis=1)
    w = weight(s, delta)
    sw = np.sqrt(w)
    return r * sw[:, None], Jp * sw[:, None, None], Jl * sw[:, None, None], w
