"""Levenberg-Marquardt outer loop (oracle; test infrastructure).

Sec. 5.1 "LM loop": start with damping 1e-4, update lambda on success or
failure of a step, at most 50 iterations, stop early at a relative function
tolerance of 1e-6; the series uses at most 20 inner iterations and eps = 0.01.

Readings where Sec. 5.1 is silent:
  * lambda update (Nielsen): on success lambda *= max(1/3, 1 - (2 rho - 1)^3),
    nu = 2; on failure lambda *= nu, nu *= 2; lambda clamped to [1e-16, 1e16].
  * gain ratio rho = (F(x) - F(x + dx)) / (L(0) - L(dx)) with the undamped
    linear model L(dx) = 1/2 ||r + J dx||^2 evaluated explicitly from J dx
    (dx is inexact, so the normal equations cannot shorten it); the model
    decrease is summed per observation as -(r.e + e.e/2), e = J dx.
  * a step is accepted iff F(x + dx) is finite, the model decrease is
    positive and rho > eta = 1e-3.
  * after an accepted step the loop ends when (F_old - F_new) / F_old < 1e-6;
    a rejected step never ends it.  Every iteration, accepted or not, counts
    towards the 50.
  * with the Huber loss the residual and Jacobian entering the model are the
    reweighted ones of robust.reweight, and F is the robust cost.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import camera, dense, post, robust, schur


@dataclasses.dataclass
class LMOptions:
    lambda0: float = 1e-4
    max_iters: int = 50
    func_tol: float = 1e-6
    m: int = 20
    eps: float = 0.01
    eta: float = 1e-3
    huber_delta: float | None = None
    damping: str = "marquardt"
    lambda_min: float = 1e-16
    lambda_max: float = 1e16


@dataclasses.dataclass
class LMIteration:
    cost: float            # F(x) before the step
    cost_new: float        # F(x + dx)
    model_decrease: float  # L(0) - L(dx)
    gain: float            # rho
    accepted: bool
    lam: float             # damping used for this step
    stop_order: int        # highest power of P in the series (or -1 for dense)


@dataclasses.dataclass
class LMResult:
    cams: np.ndarray
    lms: np.ndarray
    iterations: list
    converged: bool

    @property
    def costs(self):
        return [it.cost for it in self.iterations]


def linearize(cams, lms, obs_cam, obs_lm, obs_xy, delta=None):
    """F(x), reweighted r, J_p, J_l at the state."""
    r = camera.residuals(cams, lms, obs_cam, obs_lm, obs_xy)
    Jp, Jl = camera.jacobians(cams, lms, obs_cam, obs_lm)
    F = robust.cost(r, delta)
    rw, Jpw, Jlw, _ = robust.reweight(r, Jp, Jl, delta)
    return F, rw, Jpw, Jlw


def model_decrease(rw, Jp, Jl, obs_cam, obs_lm, dxp, dxl):
    """L(0) - L(dx) = -sum_i (r_i . e_i + e_i . e_i / 2), e_i = J_p dx_c + J_l dx_l."""
    e = np.einsum("nkj,nj->nk", Jp, dxp[obs_cam]) + np.einsum("nkj,nj->nk", Jl, dxl[obs_lm])
    terms = -(np.sum(rw * e, axis=1) + 0.5 * np.sum(e * e, axis=1))
    return math.fsum(terms.tolist())


def step_direction(rw, Jp, Jl, obs_cam, obs_lm, n_cams, n_lms, lam, opts, solver="series", cluster=None):
    if solver == "clustered":  # PoST's per-cluster series (Sec. 5.3)
        sol = post.solve_clustered(Jp, Jl, rw, obs_cam, obs_lm, n_cams, n_lms, lam, opts.m, opts.eps, cluster,
                                   opts.damping)
        return sol.dxp, sol.dxl, max(sol.stop_orders, default=0)
    if solver == "series":
        sol = schur.solve(Jp, Jl, rw, obs_cam, obs_lm, n_cams, n_lms, lam, opts.m, opts.eps,
                          opts.damping)
        return sol.dxp, sol.dxl, sol.series.stop_order
    if solver == "dense":
        J = dense.dense_jacobian(Jp, Jl, obs_cam, obs_lm, n_cams, n_lms)
        dxp, dxl, _, _ = dense.full_step(J, rw, lam, n_cams, opts.damping)
        return dxp.reshape(n_cams, 9), dxl.reshape(n_lms, 3), -1
    raise ValueError(solver)


def lm(cams0, lms0, obs_cam, obs_lm, obs_xy, opts: LMOptions | None = None, solver="series",
       callback=None, cluster=None, progress=None) -> LMResult:
    """callback(iteration, cams_new, lms_new) after every iteration;
    progress(stage) after the linearisation, the step and the trial cost of
    every iteration (for reporting only)."""
    opts = opts or LMOptions()
    report = progress or (lambda stage: None)
    cams = np.array(cams0, dtype=np.float64)
    lms = np.array(lms0, dtype=np.float64)
    n_cams, n_lms = cams.shape[0], lms.shape[0]
    lam, nu = opts.lambda0, 2.0
    F, rw, Jp, Jl = linearize(cams, lms, obs_cam, obs_lm, obs_xy, opts.huber_delta)
    report("linearised")
    its = []
    converged = False
    for it in range(opts.max_iters):
        cl = cluster(it) if callable(cluster) else cluster  # clusters drawn per iteration (Sec. 5.3)
        dxp, dxl, order = step_direction(rw, Jp, Jl, obs_cam, obs_lm, n_cams, n_lms, lam, opts, solver, cl)
        report("step")
        cams_new = cams + dxp
        lms_new = lms + dxl
        r_new = camera.residuals(cams_new, lms_new, obs_cam, obs_lm, obs_xy)
        F_new = robust.cost(r_new, opts.huber_delta)
        report("trial cost")
        L = model_decrease(rw, Jp, Jl, obs_cam, obs_lm, dxp, dxl)
        if math.isfinite(F_new) and L > 0.0:
            rho = (F - F_new) / L
        else:
            rho = -math.inf
        accepted = rho > opts.eta
        its.append(LMIteration(F, F_new, L, rho, accepted, lam, order))
        if callback is not None:
            callback(its[-1], cams_new, lms_new)
        if accepted:
            rel = (F - F_new) / F if F > 0 else 0.0
            cams, lms = cams_new, lms_new
            lam = lam * max(1.0 / 3.0, 1.0 - (2.0 * rho - 1.0) ** 3)
            nu = 2.0
            lam = min(max(lam, opts.lambda_min), opts.lambda_max)
            if rel < opts.func_tol:
                converged = True
                break
            F, rw, Jp, Jl = linearize(cams, lms, obs_cam, obs_lm, obs_xy, opts.huber_delta)
            report("linearised")
        else:
            lam = min(max(lam * nu, opts.lambda_min), opts.lambda_max)
            nu = 2.0 * nu
    return LMResult(cams, lms, its, converged)


def cost_threshold(f0, fstar, tau):
    """f_tau = f* + tau (f0 - f*)  (Sec. 5, "Performance Profiles")."""
    return fstar + tau * (f0 - fstar)
