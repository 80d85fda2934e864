"""Normal-equation blocks and damping (oracle; test infrastructure).

Sec. 4.1, eq. normal: H [dx_p; dx_l] = -[b_p; b_l] with

    U_lambda = J_p^T J_p + lambda D_p^T D_p     (block diagonal, 9x9 per camera)
    V_lambda = J_l^T J_l + lambda D_l^T D_l     (block diagonal, 3x3 per landmark)
    W        = J_p^T J_l
    b_p = J_p^T r,   b_l = J_l^T r.

The paper calls D_p, D_l "diagonal damping matrices" without fixing them.
Reading used: Marquardt damping, D^T D = diag(J^T J) clamped to [1e-6, 1e32]
(the form used by the solvers the paper says it is in line with, Sec. 5.1);
plain identity damping (D = I) is the alternative.
"""
from __future__ import annotations

import numpy as np

DIAG_MIN = 1e-6
DIAG_MAX = 1e32


def assemble(Jp, Jl, r, obs_cam, obs_lm, n_cams, n_lms):
    """Undamped blocks U [n_c,9,9], V [n_l,3,3] and b_p [n_c,9], b_l [n_l,3]."""
    U = np.zeros((n_cams, 9, 9))
    V = np.zeros((n_lms, 3, 3))
    bp = np.zeros((n_cams, 9))
    bl = np.zeros((n_lms, 3))
    np.add.at(U, obs_cam, np.einsum("nki,nkj->nij", Jp, Jp))
    np.add.at(V, obs_lm, np.einsum("nki,nkj->nij", Jl, Jl))
    np.add.at(bp, obs_cam, np.einsum("nki,nk->ni", Jp, r))
    np.add.at(bl, obs_lm, np.einsum("nki,nk->ni", Jl, r))
    return U, V, bp, bl


def damping_diagonals(U, V, mode="marquardt"):
    """D_p^T D_p and D_l^T D_l as diagonals [n_c,9], [n_l,3]."""
    if mode == "marquardt":
        dp = np.clip(np.diagonal(U, axis1=1, axis2=2), DIAG_MIN, DIAG_MAX)
        dl = np.clip(np.diagonal(V, axis1=1, axis2=2), DIAG_MIN, DIAG_MAX)
        return dp.copy(), dl.copy()
    if mode == "identity":
        return np.ones(U.shape[:2]), np.ones(V.shape[:2])
    raise ValueError(mode)


def damp(U, V, lam, dp, dl):
    """U_lambda = U + lambda diag(dp), V_lambda = V + lambda diag(dl)."""
    Ul = U.copy()
    Vl = V.copy()
    i9 = np.arange(9)
    i3 = np.arange(3)
    Ul[:, i9, i9] += lam * dp
    Vl[:, i3, i3] += lam * dl
    return Ul, Vl


def block_inverse(A):
    """Inverse of every SPD block (LAPACK through numpy.linalg.inv)."""
    if A.shape[0] == 0:
        return A.copy()
    return np.linalg.inv(A)


def _not_positive_definite(A):
    """[n] bool: blocks whose Cholesky factorisation (LAPACK) meets a pivot
    that is not positive, or that hold a non-finite entry."""
    n = A.shape[0]
    bad = ~np.all(np.isfinite(A.reshape(n, -1)), axis=1)
    idx = np.nonzero(~bad)[0]
    try:
        np.linalg.cholesky(A[idx])
    except np.linalg.LinAlgError:
        for i in idx:
            try:
                np.linalg.cholesky(A[i])
            except np.linalg.LinAlgError:
                bad[i] = True
    return bad


def damped_inverse(A, lam_d):
    """Inverses of the damped blocks A = B + lambda diag(d)  [n,k,k], with
    lam_d = lambda d  [n,k].

    Sec. 4.1 takes U_lambda and V_lambda to be positive definite, which holds
    for Gram blocks once lambda d > 0; a block set from elsewhere, or one with
    non-finite entries, need not be.  Reading for that case: a block whose
    Cholesky factorisation meets a pivot that is not positive, or whose inverse
    is not finite, is replaced by the inverse of its damping diagonal alone,
    diag(1 / (lambda d_j)), with 0 where lambda d_j is not positive.

    Returns (inverses [n,k,k], fell_back [n] bool)."""
    n, k = A.shape[0], A.shape[1]
    inv = np.zeros_like(A, dtype=np.float64)
    bad = _not_positive_definite(A)
    good = np.nonzero(~bad)[0]
    if good.size:
        inv[good] = np.linalg.inv(A[good])
    bad |= ~np.all(np.isfinite(inv.reshape(n, -1)), axis=1)
    if bad.any():
        e = np.asarray(lam_d, dtype=np.float64)[bad]
        pos = e > 0.0
        diag = np.where(pos, 1.0 / np.where(pos, e, 1.0), 0.0)
        inv[bad] = 0.0
        inv[np.nonzero(bad)[0][:, None], np.arange(k)[None, :], np.arange(k)[None, :]] = diag
    return inv, bad
