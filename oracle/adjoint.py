"""Implicit differentiation of one damped step (oracle; test infrastructure).

An extension of the method: the paper solves the damped step, it does not
differentiate it.  The step of Sec. 4.1 (eq. normal) at a fixed state,

    H dx = -g,   H = J^T J + lam D,   g = J^T r,   r = pi(state; theta) - o,

is taken with lam and the damping diagonal D held fixed (D is computed from
the undamped blocks at the state and then treated as a constant); theta are
the camera intrinsics (f, k1, k2), o the observed pixels.  Squared loss only.

For an upstream gradient gbar of dx = (dx_p, dx_l), with z = H^-1 gbar
(H is symmetric):

    d<gbar, dx>/do_i    = J_i z_i
    d<gbar, dx>/dtheta  = -z^T  d/dtheta [ J^T (J dx + r) ]   at fixed dx

since dx = -H^-1 g gives d dx = -H^-1 (dH dx + dg), dH dx + dg =
d[J^T J dx + J^T r] (lam D is constant), and dg/do_i = -J_i^T.

The truncated series (Sec. 4.3, eqs. S_approx, x_approx, with back-
substitution) is a linear map dx_m = -Ht_m^-1 g whose Ht_m^-1 is symmetric,
so the observation gradient J_i (Ht_m^-1 gbar)_i is exact for it, and the
intrinsic gradient with z_m = Ht_m^-1 gbar is the implicit-differentiation
estimate, exact as m grows.

Here z comes either from a dense LAPACK solve of H (m = None) or from the
matrix-free series of `schur.solve` run on the right-hand side -gbar; the
derivative d/dtheta [J^T (J dx + r)] is taken by the complex-step method over
the analytic Jacobian code of `camera` (real-analytic in theta).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg

from . import camera, dense, normal, schur

INTRINSICS = (6, 7, 8)


def linearize(cams, lms, obs_cam, obs_lm, obs_xy):
    """r [N,2], J_p [N,2,9], J_l [N,2,3] (squared loss)."""
    r = camera.residuals(cams, lms, obs_cam, obs_lm, obs_xy)
    Jp, Jl = camera.jacobians(cams, lms, obs_cam, obs_lm)
    return r, Jp, Jl


def damping_diagonals(cams, lms, obs_cam, obs_lm, obs_xy, mode="marquardt"):
    """D at the state, as (dp [n_c,9], dl [n_l,3]) (Sec. 4.1, Marquardt reading)."""
    r, Jp, Jl = linearize(cams, lms, obs_cam, obs_lm, obs_xy)
    U, V, _, _ = normal.assemble(Jp, Jl, r, obs_cam, obs_lm, cams.shape[0], lms.shape[0])
    return normal.damping_diagonals(U, V, mode)


def _dense_H(Jp, Jl, obs_cam, obs_lm, n_c, n_l, lam, diagonals):
    J = dense.dense_jacobian(Jp, Jl, obs_cam, obs_lm, n_c, n_l)
    d = np.concatenate([diagonals[0].ravel(), diagonals[1].ravel()])
    return J, J.T @ J + lam * np.diag(d)


def _solve(Jp, Jl, r, obs_cam, obs_lm, n_c, n_l, lam, m, diagonals, rhs):
    """Solution of H x = -rhs (rhs = (g_p, g_l)): dense if m is None, else the
    order-m series with back-substitution."""
    if m is None:
        J, H = _dense_H(Jp, Jl, obs_cam, obs_lm, n_c, n_l, lam, diagonals)
        g = np.concatenate([rhs[0].ravel(), rhs[1].ravel()])
        x = -scipy.linalg.cho_solve(scipy.linalg.cho_factor(H), g)
        return x[:9 * n_c].reshape(n_c, 9), x[9 * n_c:].reshape(n_l, 3)
    res = schur.solve(Jp, Jl, r, obs_cam, obs_lm, n_c, n_l, lam, m, 0.0, rhs=rhs, diagonals=diagonals)
    return res.dxp, res.dxl


def step(cams, lms, obs_cam, obs_lm, obs_xy, lam, m=None, diagonals=None, mode="marquardt"):
    """The damped step (dx_p, dx_l) with D fixed to `diagonals` (default: D at the state)."""
    if diagonals is None:
        diagonals = damping_diagonals(cams, lms, obs_cam, obs_lm, obs_xy, mode)
    r, Jp, Jl = linearize(cams, lms, obs_cam, obs_lm, obs_xy)
    U, V, bp, bl = normal.assemble(Jp, Jl, r, obs_cam, obs_lm, cams.shape[0], lms.shape[0])
    return _solve(Jp, Jl, r, obs_cam, obs_lm, cams.shape[0], lms.shape[0], lam, m, diagonals, (bp, bl))


@dataclasses.dataclass
class Adjoint:
    dxp: np.ndarray        # the step [n_c, 9]
    dxl: np.ndarray        # [n_l, 3]
    zp: np.ndarray         # z = H^-1 gbar (or Ht_m^-1 gbar), camera part [n_c, 9]
    zl: np.ndarray         # landmark part [n_l, 3]
    grad_obs: np.ndarray   # [N, 2]
    grad_intr: np.ndarray  # [n_c, 3]  (f, k1, k2)


def adjoint(cams, lms, obs_cam, obs_lm, obs_xy, lam, gbar_p, gbar_l, m=None, diagonals=None, mode="marquardt",
            h=1e-30):
    """Gradients of <gbar, dx> with respect to o and the intrinsics."""
    cams = np.asarray(cams, dtype=np.float64)
    lms = np.asarray(lms, dtype=np.float64)
    n_c, n_l = cams.shape[0], lms.shape[0]
    if diagonals is None:
        diagonals = damping_diagonals(cams, lms, obs_cam, obs_lm, obs_xy, mode)
    r, Jp, Jl = linearize(cams, lms, obs_cam, obs_lm, obs_xy)
    U, V, bp, bl = normal.assemble(Jp, Jl, r, obs_cam, obs_lm, n_c, n_l)
    dxp, dxl = _solve(Jp, Jl, r, obs_cam, obs_lm, n_c, n_l, lam, m, diagonals, (bp, bl))
    # z: the solution of H z = gbar, i.e. of H x = -(-gbar)
    zp, zl = _solve(Jp, Jl, r, obs_cam, obs_lm, n_c, n_l, lam, m, diagonals, (-gbar_p, -gbar_l))
    grad_obs = np.einsum("nkj,nj->nk", Jp, zp[obs_cam]) + np.einsum("nkj,nj->nk", Jl, zl[obs_lm])
    # d/dtheta_k of phi_i = J_i^T (J_i dx_i + r_i) by the complex step, all
    # cameras' parameter k perturbed at once (phi_i depends on its own camera only)
    grad_intr = np.zeros((n_c, 3))
    for col, k in enumerate(INTRINSICS):
        cz = cams.astype(np.complex128)
        cz[:, k] += 1j * h
        lz = lms.astype(np.complex128)
        rz = camera.residuals(cz, lz, obs_cam, obs_lm, obs_xy)
        Jpz, Jlz = camera.jacobians(cz, lz, obs_cam, obs_lm)
        e = np.einsum("nkj,nj->nk", Jpz, dxp[obs_cam]) + np.einsum("nkj,nj->nk", Jlz, dxl[obs_lm]) + rz
        phip = np.imag(np.einsum("nki,nk->ni", Jpz, e)) / h
        phil = np.imag(np.einsum("nki,nk->ni", Jlz, e)) / h
        contrib = np.einsum("ni,ni->n", phip, zp[obs_cam]) + np.einsum("ni,ni->n", phil, zl[obs_lm])
        np.add.at(grad_intr[:, col], obs_cam, -contrib)
    return Adjoint(dxp, dxl, zp, zl, grad_obs, grad_intr)
