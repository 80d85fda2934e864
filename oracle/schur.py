"""Schur complement, power-series solve and back-substitution (oracle; test
infrastructure).

W = J_p^T J_l is never formed: products are taken per observation i = (c, l),
whose block of W is W_cl = J_{p,i}^T J_{l,i} (Sec. 4.1).

  W s   : u_c = sum over observations of camera c of J_p^T (J_l s_l)
  W^T v : t_l = sum over observations of landmark l of J_l^T (J_p v_c)

Reduced camera system (Sec. 4.2, eqs. Sx and Schur):
  S = U - W V^-1 W^T,  b~ = b_p - W V^-1 b_l,  S dx_p = -b~.

Power series (Sec. 4.3, eqs. inverse, S_approx, x_approx): with
P = U^-1 W V^-1 W^T,
  x(m) = - sum_{i=0..m} P^i U^-1 b~,
built as v_0 = -U^-1 b~, v_i = P v_{i-1}, x(i) = x(i-1) + v_i.

Stop rule (Sec. 4.3, eq. qcriterion): after order i >= 1 stop when
(i + 1) ||x(i) - x(i-1)||_2 / ||x(i)||_2 < eps.  Readings: norms are taken
over all camera parameters in the unscaled variables; the comparison is
strict; eps = 0 disables the rule (fixed order m); ||x(i)|| = 0 stops.
m is the highest power of P, so x(m) has m + 1 terms.

Back-substitution (Sec. 4.2, eq. back_substitution): the paper prints
dx_l = -V^-1(-b_l + W^T dx_p).  The second block row of eq. normal gives
W^T dx_p + V dx_l = -b_l, i.e. dx_l = -V^-1 (b_l + W^T dx_p); that sign is
used (the printed one does not reproduce the full solve of eq. normal).
"""
from __future__ import annotations

import dataclasses

import numpy as np


def apply_W(Jp, Jl, obs_cam, obs_lm, s, n_cams):
    """u = W s  [n_c, 9]."""
    z = np.einsum("nkj,nj->nk", Jl, s[obs_lm])
    u = np.zeros((n_cams, 9))
    np.add.at(u, obs_cam, np.einsum("nki,nk->ni", Jp, z))
    return u


def apply_Wt(Jp, Jl, obs_cam, obs_lm, v, n_lms):
    """t = W^T v  [n_l, 3]."""
    q = np.einsum("nkj,nj->nk", Jp, v[obs_cam])
    t = np.zeros((n_lms, 3))
    np.add.at(t, obs_lm, np.einsum("nki,nk->ni", Jl, q))
    return t


def block_matvec(A, x):
    return np.einsum("nij,nj->ni", A, x)


def reduced_rhs(Jp, Jl, obs_cam, obs_lm, bp, bl, Vinv):
    """b~ = b_p - W V^-1 b_l."""
    return bp - apply_W(Jp, Jl, obs_cam, obs_lm, block_matvec(Vinv, bl), bp.shape[0])


def apply_P(Jp, Jl, obs_cam, obs_lm, Uinv, Vinv, v):
    """P v = U^-1 W V^-1 W^T v."""
    t = apply_Wt(Jp, Jl, obs_cam, obs_lm, v, Vinv.shape[0])
    u = apply_W(Jp, Jl, obs_cam, obs_lm, block_matvec(Vinv, t), Uinv.shape[0])
    return block_matvec(Uinv, u)


@dataclasses.dataclass
class SeriesResult:
    x: np.ndarray            # x(i*) [n_c, 9]
    iterates: list           # x(0), ..., x(i*)
    stop_order: int          # i*: the highest power of P included
    stopped_by_rule: bool    # True if the eps rule ended the series before m


def power_series(Jp, Jl, obs_cam, obs_lm, Uinv, Vinv, btilde, m, eps=0.0):
    """x(m) of eq. x_approx with the stop rule of eq. qcriterion."""
    v = -block_matvec(Uinv, btilde)
    x = v.copy()
    iterates = [x.copy()]
    stop_order = 0
    stopped = False
    for i in range(1, m + 1):
        v = apply_P(Jp, Jl, obs_cam, obs_lm, Uinv, Vinv, v)
        x = x + v
        iterates.append(x.copy())
        stop_order = i
        if eps > 0.0:
            nx = np.linalg.norm(x.ravel())
            nv = np.linalg.norm(v.ravel())
            if nx == 0.0 or (i + 1) * nv < eps * nx:
                stopped = i < m
                break
    return SeriesResult(x, iterates, stop_order, stopped)


def back_substitute(Jp, Jl, obs_cam, obs_lm, bl, Vinv, dxp):
    """dx_l = -V^-1 (b_l + W^T dx_p)."""
    t = apply_Wt(Jp, Jl, obs_cam, obs_lm, dxp, bl.shape[0])
    return -block_matvec(Vinv, bl + t)


def reduced_residual(Jp, Jl, obs_cam, obs_lm, Ul, Vinv, btilde, x):
    """|S x + b~|_2 / |b~|_2 with S x = U_lambda x - W V^-1 W^T x (eq. Schur),
    matrix-free: how far a camera step is from solving the reduced camera
    system."""
    t = apply_Wt(Jp, Jl, obs_cam, obs_lm, x, Vinv.shape[0])
    u = apply_W(Jp, Jl, obs_cam, obs_lm, block_matvec(Vinv, t), Ul.shape[0])
    res = block_matvec(Ul, x) - u + btilde
    return float(np.linalg.norm(res.ravel()) / np.linalg.norm(btilde.ravel()))


@dataclasses.dataclass
class Solve:
    dxp: np.ndarray
    dxl: np.ndarray
    btilde: np.ndarray
    Uinv: np.ndarray
    Vinv: np.ndarray
    series: SeriesResult
    Ul: np.ndarray = None    # damped camera blocks
    not_spd: int = 0         # damped blocks that took the diagonal fallback


def solve(Jp, Jl, r, obs_cam, obs_lm, n_cams, n_lms, lam, m, eps=0.0,
          damping="marquardt", rhs=None, diagonals=None, landmark_blocks=None):
    """One damped step: blocks, damped inverses, b~, series, back-substitution.

    rhs: optional (g_p, g_l) replacing (b_p, b_l) (the right-hand side of
    eq. normal is then -(g_p, g_l)); the blocks always come from J.
    diagonals: optional fixed damping diagonals (d_p [n_c,9], d_l [n_l,3])
    replacing those taken from the blocks.
    landmark_blocks: optional (V [n_l,3,3], b_l [n_l,3]) replacing the
    undamped landmark blocks assembled from J (damping is taken from them).
    A damped block that is not positive definite is inverted through its
    damping diagonal alone (normal.damped_inverse); not_spd counts them.
    """
    from . import normal

    U, V, bp, bl = normal.assemble(Jp, Jl, r, obs_cam, obs_lm, n_cams, n_lms)
    if landmark_blocks is not None:
        V, bl = (np.asarray(a, dtype=np.float64) for a in landmark_blocks)
    if rhs is not None:
        bp, bl = rhs
    dp, dl = normal.damping_diagonals(U, V, damping) if diagonals is None else diagonals
    Ul, Vl = normal.damp(U, V, lam, dp, dl)
    Uinv, bad_u = normal.damped_inverse(Ul, lam * dp)
    Vinv, bad_v = normal.damped_inverse(Vl, lam * dl)
    bt = reduced_rhs(Jp, Jl, obs_cam, obs_lm, bp, bl, Vinv)
    ser = power_series(Jp, Jl, obs_cam, obs_lm, Uinv, Vinv, bt, m, eps)
    dxl = back_substitute(Jp, Jl, obs_cam, obs_lm, bl, Vinv, ser.x)
    return Solve(ser.x, dxl, bt, Uinv, Vinv, ser, Ul, int(bad_u.sum() + bad_v.sum()))
