"""Pins of the oracle's preconditioned conjugate gradients on the reduced
camera system (Sec. 2, Fig. 2; CG of Hestenes and Stiefel), on the CPU.

They check it against what the mathematics fixes independently of the
oracle's own CG code:
  * the dense Schur complement and a LAPACK Cholesky solve of eq. Sx;
  * the diagonal blocks of the dense S (Schur-Jacobi);
  * S~(m) S = I - P^{m+1} (eq. S_approx), so the preconditioned spectrum is
    1 - eig(P)^{m+1};
  * the optimality of CG: the k-th iterate minimises the S-norm of the error
    over the Krylov space span{z, (M^-1 S) z, ..., (M^-1 S)^{k-1} z},
    z = M^-1 b, computed here by a dense projection;
  * finite termination: CG ends in at most n steps on a well-conditioned
    n x n matrix;
  * the Lanczos matrix from the CG coefficients: after n steps its
    eigenvalues are those of M^-1 S."""
import numpy as np
import pytest
import scipy.linalg

from oracle import dense, normal, pcg, schur
from oracle_fixtures import c1, rel, tiny


def _parts(P, lam):
    U, V, bp, bl = normal.assemble(P.Jp, P.Jl, P.r, P.obs_cam, P.obs_lm, P.n_cams, P.n_lms)
    dp, dl = normal.damping_diagonals(U, V)
    Ul, Vl = normal.damp(U, V, lam, dp, dl)
    Uinv, Vinv = normal.block_inverse(Ul), normal.block_inverse(Vl)
    bt = schur.reduced_rhs(P.Jp, P.Jl, P.obs_cam, P.obs_lm, bp, bl, Vinv)
    return Ul, Uinv, Vinv, bt


def _dense(P, lam):
    J = dense.dense_jacobian(P.Jp, P.Jl, P.obs_cam, P.obs_lm, P.n_cams, P.n_lms)
    return J, dense.schur_parts(J, P.r, lam, P.n_cams)


@pytest.mark.parametrize("lam", [1e-3, 1.0])
def test_schur_apply_and_jacobi_blocks_match_dense_S(lam):
    P = tiny()
    Ul, Uinv, Vinv, bt = _parts(P, lam)
    J, (U, W, V, S, btd, bp, bl) = _dense(P, lam)
    x = np.random.default_rng(1).standard_normal((P.n_cams, 9))
    got = pcg.schur_apply(P.Jp, P.Jl, P.obs_cam, P.obs_lm, Ul, Vinv, x)
    assert rel(got.ravel(), S @ x.ravel()) <= 1e-12
    blocks = pcg.schur_jacobi_blocks(P.Jp, P.Jl, P.obs_cam, P.obs_lm, Ul, Vinv)
    for c in range(P.n_cams):
        assert rel(blocks[c], S[9 * c:9 * c + 9, 9 * c:9 * c + 9]) <= 1e-12
    assert rel(bt.ravel(), btd) <= 1e-12


def test_jacobi_blocks_with_repeated_camera_landmark_pairs():
    """Two observations of one landmark by one camera add inside W_cl before
    the product W_cl V^-1 W_cl^T (a cross term the per-observation sum misses)."""
    P = tiny()
    keep = np.concatenate([np.arange(len(P.obs_cam)), [0, 3]])
    Jp, Jl = P.Jp[keep], P.Jl[keep]
    oc, ol, r = P.obs_cam[keep], P.obs_lm[keep], P.r[keep]
    J = dense.dense_jacobian(Jp, Jl, oc, ol, P.n_cams, P.n_lms)
    U, W, V, S, *_ = dense.schur_parts(J, r, 0.1, P.n_cams)
    U_, V_, _, _ = normal.assemble(Jp, Jl, r, oc, ol, P.n_cams, P.n_lms)
    dp, dl = normal.damping_diagonals(U_, V_)
    Ul, Vl = normal.damp(U_, V_, 0.1, dp, dl)
    blocks = pcg.schur_jacobi_blocks(Jp, Jl, oc, ol, Ul, normal.block_inverse(Vl))
    for c in range(P.n_cams):
        assert rel(blocks[c], S[9 * c:9 * c + 9, 9 * c:9 * c + 9]) <= 1e-12


@pytest.mark.parametrize("m", [0, 1, 3, 8])
def test_power_preconditioner_spectrum(m):
    """S~(m) S = I - P^{m+1}: the eigenvalues of the preconditioned matrix are
    1 - mu^{m+1} for the eigenvalues mu of P, all in (0, 1]."""
    P = tiny()
    lam = 1e-2
    Ul, Uinv, Vinv, bt = _parts(P, lam)
    J, (U, W, V, S, *_rest) = _dense(P, lam)
    n = 9 * P.n_cams
    # the matrix-free preconditioner applied to the columns of S
    cols = [pcg.power_series_precond(P.Jp, P.Jl, P.obs_cam, P.obs_lm, Uinv, Vinv,
                                     S[:, j].reshape(P.n_cams, 9), m).ravel() for j in range(n)]
    MS = np.stack(cols, axis=1)
    Pm = np.linalg.solve(U, W @ np.linalg.solve(V, W.T))
    assert rel(MS, np.eye(n) - np.linalg.matrix_power(Pm, m + 1)) <= 1e-10
    mu = np.sort(np.linalg.eigvals(Pm).real)
    ev = np.sort(np.linalg.eigvals(MS).real)
    assert np.allclose(ev, np.sort(1.0 - mu ** (m + 1)), atol=1e-10)
    assert ev.min() > 0.0 and ev.max() <= 1.0 + 1e-12


@pytest.mark.parametrize("precond", ["none", "schur_jacobi", "power"])
@pytest.mark.parametrize("lam", [1e-3, 1.0])
def test_pcg_solution_matches_cholesky(precond, lam):
    P = c1()
    out = pcg.solve_pcg(P.Jp, P.Jl, P.r, P.obs_cam, P.obs_lm, P.n_cams, P.n_lms, lam,
                        precond, 4, 1e-12, 2000)
    assert out.result.converged
    J, (U, W, V, S, bt, bp, bl) = _dense(P, lam)
    dxp = -scipy.linalg.cho_solve(scipy.linalg.cho_factor(S), bt)
    dxl = -np.linalg.solve(V, bl + W.T @ dxp)
    # |x - x*| / |x*| <= kappa(S) |r| / |b|, plus rounding of the dense solve
    ev = np.linalg.eigvalsh(S)
    bound = ev[-1] / ev[0] * out.result.residuals[-1] + 1e-11
    assert rel(out.dxp.ravel(), dxp) <= bound
    assert rel(out.dxl.ravel(), dxl) <= 10 * bound


@pytest.mark.parametrize("precond,m", [("none", 0), ("schur_jacobi", 0), ("power", 0), ("power", 2)])
def test_pcg_iterates_are_krylov_minimisers(precond, m):
    """x_k = argmin over x in K_k(M^-1 S, M^-1 b) of (x - x*)^T S (x - x*),
    by a dense projection onto an orthonormal Krylov basis."""
    P = tiny()
    lam = 1e-2
    Ul, Uinv, Vinv, bt = _parts(P, lam)
    J, (U, W, V, S, btd, *_rest) = _dense(P, lam)
    n = 9 * P.n_cams
    if precond == "none":
        Minv = np.eye(n)
    elif precond == "schur_jacobi":
        Minv = np.zeros((n, n))
        for c in range(P.n_cams):
            s = slice(9 * c, 9 * c + 9)
            Minv[s, s] = np.linalg.inv(S[s, s])
    else:
        Minv = dense.S_tilde(np.linalg.solve(U, W @ np.linalg.solve(V, W.T)), U, m)
    out = pcg.solve_pcg(P.Jp, P.Jl, P.r, P.obs_cam, P.obs_lm, P.n_cams, P.n_lms, lam,
                        precond, m, 0.0, 5)
    b = -btd
    z = Minv @ b
    K = [z]
    for _ in range(4):
        K.append(Minv @ (S @ K[-1]))
    for k in range(1, 6):
        Q, _ = np.linalg.qr(np.stack(K[:k], axis=1))
        y = np.linalg.solve(Q.T @ S @ Q, Q.T @ b)
        assert rel(out.result.iterates[k - 1].ravel(), Q @ y) <= 1e-8, k


def test_cg_terminates_and_lanczos_recovers_spectrum():
    """Without a preconditioner CG solves S x = b; on a well-conditioned n x n
    matrix with n distinct eigenvalues it ends within n steps (up to
    rounding), and the n x n Lanczos matrix of its coefficients has that
    matrix's spectrum."""
    P = tiny()
    lam = 1.0
    J, (U, W, V, S, btd, *_rest) = _dense(P, lam)
    res = pcg.pcg(lambda x: S @ x, -btd, lambda x: x.copy(), 1e-10, 2000)
    assert res.converged
    ev = np.linalg.eigvalsh(S)
    assert rel(res.x, np.linalg.solve(S, -btd)) <= ev[-1] / ev[0] * 1e-10 + 1e-12
    n = 12
    d = np.linspace(1.0, 4.0, n)
    Q, _ = np.linalg.qr(np.random.default_rng(5).standard_normal((n, n)))
    A = Q @ np.diag(d) @ Q.T
    b = np.random.default_rng(6).standard_normal(n)
    r = pcg.pcg(lambda x: A @ x, b, lambda x: x.copy(), 1e-12, 4 * n)
    assert r.converged and r.iterations <= n + 1
    r = pcg.pcg(lambda x: A @ x, b, lambda x: x.copy(), 0.0, n)
    T = pcg.lanczos_tridiagonal(r.alphas, r.betas)
    assert np.allclose(np.linalg.eigvalsh(T), d, atol=1e-8)
    assert abs(pcg.condition_estimate(r.alphas, r.betas) - 4.0) <= 1e-8


def test_condition_estimate_approaches_dense_kappa():
    """On c1 the Ritz-value ratio after convergence is close to the dense
    kappa(M^-1 S) for Schur-Jacobi and for the power series with m = 2."""
    P = c1()
    lam = 1e-2
    J, (U, W, V, S, *_rest) = _dense(P, lam)
    n = S.shape[0]
    Pm = np.linalg.solve(U, W @ np.linalg.solve(V, W.T))
    Mj = np.zeros((n, n))
    for c in range(P.n_cams):
        s = slice(9 * c, 9 * c + 9)
        Mj[s, s] = np.linalg.inv(S[s, s])
    for precond, m, Minv in [("schur_jacobi", 0, Mj), ("power", 2, dense.S_tilde(Pm, U, 2))]:
        ev = np.sort(np.linalg.eigvals(Minv @ S).real)
        kappa = ev[-1] / ev[0]
        out = pcg.solve_pcg(P.Jp, P.Jl, P.r, P.obs_cam, P.obs_lm, P.n_cams, P.n_lms, lam,
                            precond, m, 1e-12, 2000)
        est = pcg.condition_estimate(out.result.alphas, out.result.betas)
        assert est <= kappa * (1 + 1e-6)
        assert est >= 0.9 * kappa, (precond, est, kappa)


def test_iterations_fall_with_series_order():
    """Fig. 2 (b): a higher order m of the power-series preconditioner needs
    fewer CG iterations, and already m = 1 needs no more than Schur-Jacobi's
    U-block part (m = 0 is block Jacobi on U)."""
    P = c1()
    lam = 1e-2
    its = {}
    for m in [0, 1, 2, 4, 8]:
        out = pcg.solve_pcg(P.Jp, P.Jl, P.r, P.obs_cam, P.obs_lm, P.n_cams, P.n_lms, lam,
                            "power", m, 1e-8, 2000)
        assert out.result.converged
        its[m] = out.result.iterations
    seq = [its[m] for m in sorted(its)]
    assert all(a >= b for a, b in zip(seq, seq[1:])), its
    assert its[8] < its[0]


def test_order_zero_is_block_jacobi_on_U():
    P = tiny()
    Ul, Uinv, Vinv, bt = _parts(P, 0.1)
    x = np.random.default_rng(2).standard_normal((P.n_cams, 9))
    got = pcg.power_series_precond(P.Jp, P.Jl, P.obs_cam, P.obs_lm, Uinv, Vinv, x, 0)
    want = np.stack([np.linalg.solve(Ul[c], x[c]) for c in range(P.n_cams)])
    assert rel(got, want) <= 1e-12


def test_zero_rhs_and_unknown_preconditioner():
    res = pcg.pcg(lambda x: 2 * x, np.zeros((3, 9)), lambda x: x, 1e-8, 10)
    assert res.converged and res.iterations == 0 and not np.any(res.x)
    P = tiny()
    with pytest.raises(ValueError):
        pcg.solve_pcg(P.Jp, P.Jl, P.r, P.obs_cam, P.obs_lm, P.n_cams, P.n_lms, 0.1, "ilu", 0, 1e-8, 10)
