"""Dense reference quantities for tiny problems (oracle; test infrastructure).

Forms the full system of eq. normal (Sec. 4.1) and the reduced camera system
(Sec. 4.2) as dense matrices, so that the matrix-free path can be checked
against LAPACK solves, and the spectral statements of the paper can be
evaluated directly:

  Sec. 3, Prop. 1       (I - M)^-1 = sum_{i<=m} M^i + R,  R = M^{m+1} (I - M)^-1
  Sec. 4.3, Lemma 1     eigenvalues of P = U^-1 W V^-1 W^T lie in [0, 1)
  Sec. 4.3, Prop. 2     x(m) - dx_p = R_m b~,  R_m = sum_{i>m} P^i U^-1

Only for problems small enough for dense (9 n_c + 3 n_l)^2 matrices.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def dense_jacobian(Jp, Jl, obs_cam, obs_lm, n_cams, n_lms):
    """J = [J_p J_l] as a dense (2N) x (9 n_c + 3 n_l) matrix."""
    n = Jp.shape[0]
    J = np.zeros((2 * n, 9 * n_cams + 3 * n_lms))
    for i in range(n):
        c, l = int(obs_cam[i]), int(obs_lm[i])
        J[2 * i:2 * i + 2, 9 * c:9 * c + 9] = Jp[i]
        J[2 * i:2 * i + 2, 9 * n_cams + 3 * l:9 * n_cams + 3 * l + 3] = Jl[i]
    return J


def damping_matrix(J, n_cams, mode="marquardt"):
    """diag(D^T D) for the whole state (same reading as normal.damping_diagonals)."""
    if mode == "identity":
        return np.ones(J.shape[1])
    return np.clip(np.sum(J * J, axis=0), 1e-6, 1e32)


def split(H, n_cams):
    k = 9 * n_cams
    return H[:k, :k], H[:k, k:], H[k:, k:]


def full_step(J, r, lam, n_cams, mode="marquardt"):
    """dx = -H^-1 J^T r by a dense Cholesky solve of eq. normal."""
    d = damping_matrix(J, n_cams, mode)
    H = J.T @ J + lam * np.diag(d)
    g = J.T @ r.reshape(-1)
    dx = -scipy.linalg.cho_solve(scipy.linalg.cho_factor(H), g)
    k = 9 * n_cams
    return dx[:k], dx[k:], H, g


def schur_parts(J, r, lam, n_cams, mode="marquardt"):
    """Dense U, W, V (damped), S, b~, g = (b_p, b_l)."""
    d = damping_matrix(J, n_cams, mode)
    H = J.T @ J + lam * np.diag(d)
    g = J.T @ r.reshape(-1)
    U, W, V = split(H, n_cams)
    k = 9 * n_cams
    bp, bl = g[:k], g[k:]
    Vinv = np.linalg.inv(V)
    S = U - W @ Vinv @ W.T
    bt = bp - W @ Vinv @ bl
    return U, W, V, S, bt, bp, bl


def schur_step(J, r, lam, n_cams, mode="marquardt"):
    """dx_p = -S^-1 b~ by dense Cholesky of the reduced camera system."""
    U, W, V, S, bt, bp, bl = schur_parts(J, r, lam, n_cams, mode)
    dxp = -scipy.linalg.cho_solve(scipy.linalg.cho_factor(S), bt)
    dxl = -np.linalg.solve(V, bl + W.T @ dxp)
    return dxp, dxl


def P_matrix(J, r, lam, n_cams, mode="marquardt"):
    U, W, V, S, bt, bp, bl = schur_parts(J, r, lam, n_cams, mode)
    return np.linalg.solve(U, W @ np.linalg.solve(V, W.T)), U, S, bt


def symmetric_P(J, r, lam, n_cams, mode="marquardt"):
    """U^-1/2 W V^-1 W^T U^-1/2, similar to P and symmetric (Lemma 1 proof)."""
    U, W, V, S, bt, bp, bl = schur_parts(J, r, lam, n_cams, mode)
    w, Q = np.linalg.eigh(U)
    Uih = Q @ np.diag(w ** -0.5) @ Q.T
    Ph = Uih @ W @ np.linalg.solve(V, W.T) @ Uih
    return 0.5 * (Ph + Ph.T)


def S_tilde(P, U, m):
    """S~_{-1}(m) = sum_{i=0..m} P^i U^-1 (eq. S_approx)."""
    Uinv = np.linalg.inv(U)
    term = Uinv.copy()
    acc = Uinv.copy()
    for _ in range(m):
        term = P @ term
        acc = acc + term
    return acc


def series_remainder(M, m):
    """R = sum_{i>m} M^i = M^{m+1} (I - M)^-1 (Prop. 1)."""
    n = M.shape[0]
    return np.linalg.matrix_power(M, m + 1) @ np.linalg.inv(np.eye(n) - M)


def spectral_radius(A):
    return float(np.max(np.abs(np.linalg.eigvals(A))))
