"""Preconditioned conjugate gradients on the reduced camera system (oracle;
test infrastructure: only tests/, smoke() and the benchmark's CPU leg use it).

The paper compares, in its Fig. 2 (Sec. 2), the power series of the inverse
Schur complement used as a preconditioner of CG on S x = -b~ (eq. Sx) with
the Schur-Jacobi preconditioner: M^-1 = S~(m) = sum_{i<=m} P^i U^-1
(eq. S_approx, 4m products per application) against the inverted 9 x 9
diagonal blocks of S.  CG (Hestenes and Stiefel) is written out here with
x_0 = 0:

    r = b - S x, z = M^-1 r, p = z
    repeat: q = S p, alpha = (r.z) / (p.q), x += alpha p, r -= alpha q,
            stop when |r| <= tol |b|, z = M^-1 r,
            beta = (r.z)_new / (r.z)_old, p = z + beta p

Blocks, damping and the reduced right-hand side are those of the power-series
solve (schur.solve), so both solvers work on the same damped system.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import normal, schur


def schur_apply(Jp, Jl, obs_cam, obs_lm, Ul, Vinv, x):
    """S x = U_lambda x - W V_lambda^-1 W^T x (eq. Schur), matrix-free."""
    t = schur.apply_Wt(Jp, Jl, obs_cam, obs_lm, x, Vinv.shape[0])
    u = schur.apply_W(Jp, Jl, obs_cam, obs_lm, schur.block_matvec(Vinv, t), Ul.shape[0])
    return schur.block_matvec(Ul, x) - u


def schur_jacobi_blocks(Jp, Jl, obs_cam, obs_lm, Ul, Vinv):
    """The 9 x 9 diagonal blocks of S: U_c - sum_l W_cl V_l^-1 W_cl^T, with
    W_cl the sum of J_p^T J_l over the observations of camera c and landmark l."""
    n_cams = Ul.shape[0]
    Wcl = {}
    for i in range(Jp.shape[0]):
        key = (int(obs_cam[i]), int(obs_lm[i]))
        w = Jp[i].T @ Jl[i]
        Wcl[key] = Wcl[key] + w if key in Wcl else w
    S = Ul.copy()
    for (c, l), w in Wcl.items():
        S[c] -= w @ Vinv[l] @ w.T
    assert S.shape[0] == n_cams
    return S


def power_series_precond(Jp, Jl, obs_cam, obs_lm, Uinv, Vinv, r, m):
    """S~(m) r = sum_{i<=m} P^i U^-1 r (the series of schur.power_series run on
    b~ = -r, which returns -sum P^i U^-1 b~)."""
    return schur.power_series(Jp, Jl, obs_cam, obs_lm, Uinv, Vinv, -r, m, 0.0).x


@dataclasses.dataclass
class PCGResult:
    x: np.ndarray            # the solution estimate, shaped like b
    iterations: int          # CG iterations performed
    residuals: list          # |r_k| / |b| for k = 0..iterations
    converged: bool
    iterates: list           # x_1, ..., x_iterations
    alphas: list             # step lengths alpha_1..alpha_k
    betas: list              # direction updates beta_1..beta_{k-1}


def pcg(apply_S, b, apply_M, tol, max_iters):
    """CG on S x = b with preconditioner z = apply_M(r), from x_0 = 0."""
    nb = float(np.linalg.norm(b.ravel()))
    x = np.zeros_like(b)
    if nb == 0.0:
        return PCGResult(x, 0, [0.0], True, [], [], [])
    r = b.copy()
    z = apply_M(r)
    p = z.copy()
    rz = float(np.sum(r * z))
    res, xs, alphas, betas = [1.0], [], [], []
    for k in range(1, max_iters + 1):
        q = apply_S(p)
        alpha = rz / float(np.sum(p * q))
        x = x + alpha * p
        r = r - alpha * q
        res.append(float(np.linalg.norm(r.ravel())) / nb)
        xs.append(x.copy())
        alphas.append(alpha)
        if res[-1] <= tol:
            return PCGResult(x, k, res, True, xs, alphas, betas)
        z = apply_M(r)
        rz_new = float(np.sum(r * z))
        betas.append(rz_new / rz)
        p = z + betas[-1] * p
        rz = rz_new
    return PCGResult(x, max_iters, res, False, xs, alphas, betas)


def lanczos_tridiagonal(alphas, betas):
    """The k x k Lanczos matrix of M^-1 S implied by k CG steps: diagonal
    1/alpha_j + beta_{j-1}/alpha_{j-1}, off-diagonal sqrt(beta_j)/alpha_j.
    Its eigenvalues (Ritz values) approach the extreme eigenvalues of M^-1 S,
    so their ratio estimates the condition number kappa(M^-1 S) of Fig. 2."""
    k = len(alphas)
    T = np.zeros((k, k))
    for j in range(k):
        T[j, j] = 1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0)
        if j + 1 < k:
            T[j, j + 1] = T[j + 1, j] = np.sqrt(betas[j]) / alphas[j]
    return T


def condition_estimate(alphas, betas):
    """lambda_max / lambda_min of the Lanczos matrix (1.0 for no steps)."""
    if not alphas:
        return 1.0
    ev = np.linalg.eigvalsh(lanczos_tridiagonal(alphas, betas))
    return float(ev[-1] / ev[0])


@dataclasses.dataclass
class PCGSolve:
    dxp: np.ndarray
    dxl: np.ndarray
    btilde: np.ndarray
    result: PCGResult


def solve_pcg(Jp, Jl, r, obs_cam, obs_lm, n_cams, n_lms, lam, precond, m, tol, max_iters,
              damping="marquardt"):
    """One damped step with the camera step from PCG on S dx_p = -b~.
    precond: "schur_jacobi", "power" (order m) or "none"."""
    U, V, bp, bl = normal.assemble(Jp, Jl, r, obs_cam, obs_lm, n_cams, n_lms)
    dp, dl = normal.damping_diagonals(U, V, damping)
    Ul, Vl = normal.damp(U, V, lam, dp, dl)
    Uinv, _ = normal.damped_inverse(Ul, lam * dp)
    Vinv, _ = normal.damped_inverse(Vl, lam * dl)
    bt = schur.reduced_rhs(Jp, Jl, obs_cam, obs_lm, bp, bl, Vinv)

    def apply_S(x):
        return schur_apply(Jp, Jl, obs_cam, obs_lm, Ul, Vinv, x)

    if precond == "schur_jacobi":
        Minv = normal.block_inverse(schur_jacobi_blocks(Jp, Jl, obs_cam, obs_lm, Ul, Vinv))

        def apply_M(x):
            return schur.block_matvec(Minv, x)
    elif precond == "power":
        def apply_M(x):
            return power_series_precond(Jp, Jl, obs_cam, obs_lm, Uinv, Vinv, x, m)
    elif precond == "none":
        def apply_M(x):
            return x.copy()
    else:
        raise ValueError(f"unknown preconditioner {precond}")
    res = pcg(apply_S, -bt, apply_M, tol, max_iters)
    dxl = schur.back_substitute(Jp, Jl, obs_cam, obs_lm, bl, Vinv, res.x)
    return PCGSolve(res.x, dxl, bt, res)
