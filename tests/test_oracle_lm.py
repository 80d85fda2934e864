"""Pins of the oracle's LM loop and Huber loss (CPU)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import camera, lm, robust
from oracle_fixtures import c1, rel, tiny

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_defaults_follow_paper_settings():
    g = json.load(open(os.path.join(GOLDEN, "lm_settings.json")))
    o = lm.LMOptions()
    assert o.lambda0 == g["lambda0"]
    assert o.max_iters == g["max_lm_iterations"]
    assert o.func_tol == g["relative_function_tolerance"]
    assert o.m == g["max_inner_iterations"]
    assert o.eps == g["epsilon"]


def test_lm_accepted_costs_decrease_and_match_dense_solver():
    P = c1()
    opts = lm.LMOptions(max_iters=50)
    ser = lm.lm(P.cams, P.lms, P.obs_cam, P.obs_lm, P.obs, opts, solver="series")
    den = lm.lm(P.cams, P.lms, P.obs_cam, P.obs_lm, P.obs, opts, solver="dense")
    acc = [it.cost_new for it in ser.iterations if it.accepted]
    assert all(b < a for a, b in zip(acc, acc[1:]))
    assert ser.converged and den.converged
    f_ser = min(acc)
    f_den = min(it.cost_new for it in den.iterations if it.accepted)
    assert abs(f_ser - f_den) <= 1e-6 * f_den
    # the optimum sits near the noise floor: 1/2 chi^2 with 2N - dof degrees of freedom
    dof = 2 * len(P.obs_cam) - 9 * P.n_cams - 3 * P.n_lms
    assert 0.3 * dof < f_den < 0.7 * dof


def test_rejected_step_raises_damping():
    """Far from the optimum (0.8 rad rotation error), with lambda0 tiny and a
    single series term, steps fail; every failure multiplies lambda by nu and
    doubles nu, every success applies the Nielsen factor."""
    P = tiny()
    opts = lm.LMOptions(lambda0=1e-12, m=0, eps=0.0, max_iters=12)
    cams = P.cams.copy()
    cams[:, 1] += 0.8
    res = lm.lm(cams, P.lms, P.obs_cam, P.obs_lm, P.obs, opts)
    lams = [it.lam for it in res.iterations]
    nu = 2.0
    for a, b, it in zip(lams, lams[1:], res.iterations):
        if it.accepted:
            expect = a * max(1 / 3, 1 - (2 * it.gain - 1) ** 3)
            nu = 2.0
        else:
            expect = a * nu
            nu *= 2.0
        assert b == pytest.approx(min(max(expect, 1e-16), 1e16), rel=1e-12)
    assert any(not it.accepted for it in res.iterations)
    assert any(it.accepted for it in res.iterations)


def test_cost_threshold():
    assert lm.cost_threshold(10.0, 2.0, 0.0) == 2.0
    assert lm.cost_threshold(10.0, 2.0, 1.0) == 10.0
    assert lm.cost_threshold(10.0, 2.0, 0.01) == pytest.approx(2.08)


def test_model_decrease_equals_quadratic_difference():
    P = tiny()
    rng = np.random.default_rng(0)
    dxp = rng.normal(size=(P.n_cams, 9)) * 1e-3
    dxl = rng.normal(size=(P.n_lms, 3)) * 1e-2
    L = lm.model_decrease(P.r, P.Jp, P.Jl, P.obs_cam, P.obs_lm, dxp, dxl)
    e = np.einsum("nkj,nj->nk", P.Jp, dxp[P.obs_cam]) + np.einsum("nkj,nj->nk", P.Jl, dxl[P.obs_lm])
    direct = 0.5 * np.sum(P.r ** 2) - 0.5 * np.sum((P.r + e) ** 2)
    assert L == pytest.approx(direct, rel=1e-9)


# ---------------------------------------------------------------- Huber ----

def test_huber_continuity_and_derivative():
    d = 3.0
    s0 = d * d
    eps = 1e-9
    assert robust.rho(s0 - eps, d) == pytest.approx(robust.rho(s0 + eps, d), abs=1e-8)
    assert robust.weight(s0 * (1 - 1e-12), d) == pytest.approx(robust.weight(s0 * (1 + 1e-12), d), rel=1e-9)
    for s in [0.5, 4.0, 9.5, 100.0, 1e4]:
        h = 1e-6 * s
        fd = (robust.rho(s + h, d) - robust.rho(s - h, d)) / (2 * h)
        assert robust.weight(s, d) == pytest.approx(fd, rel=1e-7)


def test_irls_gradient_is_robust_cost_gradient():
    """sum_i w_i J_i^T r_i is the gradient of F = 1/2 sum rho(||r_i||^2)."""
    P = tiny()
    delta = 2.0
    cams, lms = P.scene.cams_gt, P.scene.lms_gt
    obs = P.obs.copy()
    obs[::3] += 25.0  # make some residuals outliers
    r = camera.residuals(cams, lms, P.obs_cam, P.obs_lm, obs)
    Jp, Jl = camera.jacobians(cams, lms, P.obs_cam, P.obs_lm)
    rw, Jpw, Jlw, w = robust.reweight(r, Jp, Jl, delta)
    assert np.any(w < 1.0) and np.any(w == 1.0)
    g_lm = np.zeros((P.n_lms, 3))
    np.add.at(g_lm, P.obs_lm, np.einsum("nki,nk->ni", Jlw, rw))
    for l in range(P.n_lms):
        for j in range(3):
            h = 1e-6
            lp, lmn = lms.copy(), lms.copy()
            lp[l, j] += h
            lmn[l, j] -= h
            Fp = robust.cost(camera.residuals(cams, lp, P.obs_cam, P.obs_lm, obs), delta)
            Fm = robust.cost(camera.residuals(cams, lmn, P.obs_cam, P.obs_lm, obs), delta)
            assert (Fp - Fm) / (2 * h) == pytest.approx(g_lm[l, j], rel=1e-5, abs=1e-6)


def test_cost_is_half_sum_of_squares_without_loss():
    P = tiny()
    assert robust.cost(P.r) == pytest.approx(0.5 * float(np.sum(P.r ** 2)), rel=1e-14)
    assert math.isfinite(P.F)


def test_cost_beyond_float64_range_is_infinite():
    """A trial state so far off that the sum of its squared residuals leaves
    the float64 range has an infinite cost (every term is finite, only the
    sum overflows), so the LM loop, which accepts a step only if F(x + dx) is
    finite, rejects it instead of failing."""
    huge = np.full((4, 2), 7e153)  # each term 9.8e307, their sum past 1.8e308
    assert np.all(np.isfinite(np.sum(huge ** 2, axis=1)))
    assert math.isinf(robust.cost(huge))
    assert math.isfinite(robust.cost(huge, 3.0))  # Huber terms grow like |r| and stay summable
    nan = np.array([[1.0, 2.0], [np.nan, 0.0]])
    assert math.isnan(robust.cost(nan))
