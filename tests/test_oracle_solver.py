"""Pins of the oracle's normal equations, Schur complement and power series
(CPU).  They check the matrix-free oracle against a brute-force Jacobian of
the whole residual vector, LAPACK solves of eq. normal, and the spectral
statements of Sec. 3 (Prop. 1) and Sec. 4.3 (Lemma 1, Prop. 2)."""
import numpy as np
import pytest

from oracle import camera, dense, normal, schur
from oracle_fixtures import c1, rel, tiny

LAMBDAS = [1e-4, 1e-2, 1.0]


def _full_fd_jacobian(P, h=1e-6):
    """Central differences of the stacked residual vector w.r.t. the whole state."""
    x0 = np.concatenate([P.cams.ravel(), P.lms.ravel()])
    nc = P.cams.size

    def res(x):
        c = x[:nc].reshape(P.cams.shape)
        l = x[nc:].reshape(P.lms.shape)
        return camera.residuals(c, l, P.obs_cam, P.obs_lm, P.obs).ravel()

    J = np.zeros((2 * len(P.obs_cam), x0.size))
    for j in range(x0.size):
        step = h * max(1.0, abs(x0[j]))
        xp, xm = x0.copy(), x0.copy()
        xp[j] += step
        xm[j] -= step
        J[:, j] = (res(xp) - res(xm)) / (2 * step)
    return J, res(x0)


def test_blocks_match_brute_force_jacobian():
    P = tiny()
    J, r = _full_fd_jacobian(P)
    H = J.T @ J
    g = J.T @ r
    U, V, bp, bl = normal.assemble(P.Jp, P.Jl, P.r, P.obs_cam, P.obs_lm, P.n_cams, P.n_lms)
    k = 9 * P.n_cams
    for c in range(P.n_cams):
        assert rel(U[c], H[9 * c:9 * c + 9, 9 * c:9 * c + 9]) < 1e-6
    for l in range(P.n_lms):
        assert rel(V[l], H[k + 3 * l:k + 3 * l + 3, k + 3 * l:k + 3 * l + 3]) < 1e-6
    assert rel(bp.ravel(), g[:k]) < 1e-6 and rel(bl.ravel(), g[k:]) < 1e-6
    # W = J_p^T J_l through the matrix-free products
    rng = np.random.default_rng(0)
    s = rng.normal(size=(P.n_lms, 3))
    v = rng.normal(size=(P.n_cams, 9))
    W = H[:k, k:]
    assert rel(schur.apply_W(P.Jp, P.Jl, P.obs_cam, P.obs_lm, s, P.n_cams).ravel(), W @ s.ravel()) < 1e-6
    assert rel(schur.apply_Wt(P.Jp, P.Jl, P.obs_cam, P.obs_lm, v, P.n_lms).ravel(), W.T @ v.ravel()) < 1e-6


def test_marquardt_damping_clamps_empty_columns():
    U = np.zeros((2, 9, 9))
    U[0] = np.eye(9) * 4.0
    V = np.ones((1, 3, 3))
    dp, dl = normal.damping_diagonals(U, V)
    assert np.all(dp[0] == 4.0) and np.all(dp[1] == normal.DIAG_MIN) and np.all(dl == 1.0)


@pytest.mark.parametrize("lam,mode", [(1e-4, "marquardt"), (1e-2, "marquardt"), (1.0, "marquardt"),
                                      (1e-2, "identity"), (1.0, "identity")])
def test_schur_and_back_substitution_equal_full_solve(lam, mode):
    # (identity damping at 1e-4 leaves H too ill-conditioned for a 1e-9 comparison
    # of two dense solvers)
    P = c1()
    J = dense.dense_jacobian(P.Jp, P.Jl, P.obs_cam, P.obs_lm, P.n_cams, P.n_lms)
    dxp, dxl, _, _ = dense.full_step(J, P.r, lam, P.n_cams, mode)
    sp, sl = dense.schur_step(J, P.r, lam, P.n_cams, mode)
    assert rel(sp, dxp) < 1e-9 and rel(sl, dxl) < 1e-9
    # matrix-free back-substitution with the exact dx_p
    U, V, bp, bl = normal.assemble(P.Jp, P.Jl, P.r, P.obs_cam, P.obs_lm, P.n_cams, P.n_lms)
    dp, dl = normal.damping_diagonals(U, V, mode)
    _, Vl = normal.damp(U, V, lam, dp, dl)
    Vinv = normal.block_inverse(Vl)
    mf = schur.back_substitute(P.Jp, P.Jl, P.obs_cam, P.obs_lm, bl, Vinv, dxp.reshape(-1, 9))
    assert rel(mf, dxl) < 1e-9
    # the sign printed in eq. back_substitution (-b_l) does not reproduce the solve
    t = schur.apply_Wt(P.Jp, P.Jl, P.obs_cam, P.obs_lm, dxp.reshape(-1, 9), P.n_lms)
    printed = -schur.block_matvec(Vinv, -bl + t)
    assert rel(printed, dxl) > 1e-3


def test_series_converges_to_full_solve_at_large_order():
    P = c1()
    J = dense.dense_jacobian(P.Jp, P.Jl, P.obs_cam, P.obs_lm, P.n_cams, P.n_lms)
    dxp, dxl, _, _ = dense.full_step(J, P.r, 1.0, P.n_cams)
    sol = schur.solve(P.Jp, P.Jl, P.r, P.obs_cam, P.obs_lm, P.n_cams, P.n_lms, 1.0, 80, 0.0)
    assert rel(sol.dxp, dxp) < 1e-10 and rel(sol.dxl, dxl) < 1e-10


@pytest.mark.parametrize("lam", LAMBDAS)
@pytest.mark.parametrize("m", [0, 1, 5, 20])
def test_series_error_closed_form(lam, m):
    """x(m) - dx_p = -P^{m+1} dx_p (Prop. 2: x(m) - dx_p = R_m b~, R_m = P^{m+1} S^-1)."""
    P = c1()
    J = dense.dense_jacobian(P.Jp, P.Jl, P.obs_cam, P.obs_lm, P.n_cams, P.n_lms)
    dxp, _, _, _ = dense.full_step(J, P.r, lam, P.n_cams)
    Pm, U, S, bt = dense.P_matrix(J, P.r, lam, P.n_cams)
    sol = schur.solve(P.Jp, P.Jl, P.r, P.obs_cam, P.obs_lm, P.n_cams, P.n_lms, lam, m, 0.0)
    err = sol.dxp.ravel() - dxp
    pred = -np.linalg.matrix_power(Pm, m + 1) @ dxp
    assert np.linalg.norm(err - pred) <= 1e-9 * np.linalg.norm(dxp)
    if m == 0:
        Uinv = np.linalg.inv(U)
        assert rel(sol.dxp.ravel(), -Uinv @ bt) < 1e-12


@pytest.mark.parametrize("lam,m", [(1e-2, 0), (1e-2, 5), (1.0, 3), (1.0, 40)])
def test_reduced_residual_closed_form(lam, m):
    """S x(m) + b~ = U P^{m+1} U^-1 b~ (the series sums the first m+1 terms of
    (I - P)^-1, Sec. 3 Prop. 1), evaluated with dense matrices."""
    P = c1()
    J = dense.dense_jacobian(P.Jp, P.Jl, P.obs_cam, P.obs_lm, P.n_cams, P.n_lms)
    Pm, U, S, bt = dense.P_matrix(J, P.r, lam, P.n_cams)
    sol = schur.solve(P.Jp, P.Jl, P.r, P.obs_cam, P.obs_lm, P.n_cams, P.n_lms, lam, m, 0.0)
    got = schur.reduced_residual(P.Jp, P.Jl, P.obs_cam, P.obs_lm, sol.Ul, sol.Vinv, sol.btilde, sol.dxp)
    pred = U @ np.linalg.matrix_power(Pm, m + 1) @ np.linalg.solve(U, bt)
    want = np.linalg.norm(pred) / np.linalg.norm(bt)
    assert abs(got - want) <= 1e-8 * want + 1e-14, (got, want)
    # the dense solution of the reduced system has no residual
    exact = -np.linalg.solve(S, bt)
    zero = schur.reduced_residual(P.Jp, P.Jl, P.obs_cam, P.obs_lm, sol.Ul, sol.Vinv, sol.btilde,
                                  exact.reshape(P.n_cams, 9))
    assert zero < 1e-9


@pytest.mark.parametrize("lam", [1e-4, 1e-2, 1.0, 100.0])
@pytest.mark.parametrize("mode", ["marquardt", "identity"])
def test_lemma1_eigenvalues_in_unit_interval(lam, mode):
    P = c1()
    J = dense.dense_jacobian(P.Jp, P.Jl, P.obs_cam, P.obs_lm, P.n_cams, P.n_lms)
    Ph = dense.symmetric_P(J, P.r, lam, P.n_cams, mode)
    ev = np.linalg.eigvalsh(Ph)
    assert ev.min() > -1e-10 and ev.max() < 1.0
    Pm, _, _, _ = dense.P_matrix(J, P.r, lam, P.n_cams, mode)
    evn = np.linalg.eigvals(Pm)
    assert np.max(np.abs(evn.imag)) < 1e-8
    np.testing.assert_allclose(np.sort(evn.real), np.sort(ev), atol=1e-8)


def test_spectral_radius_regime_at_initial_damping():
    """Fig. 4 caption: rho(M) is just below 1 at lambda0 = 1e-4 (0.999858 and
    0.999879 on two BAL problems).  Qualitative regime only: same order of 1 - rho."""
    import json, os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "spectral_radius.json")))
    P = c1()
    J = dense.dense_jacobian(P.Jp, P.Jl, P.obs_cam, P.obs_lm, P.n_cams, P.n_lms)
    rho = float(np.linalg.eigvalsh(dense.symmetric_P(J, P.r, 1e-4, P.n_cams)).max())
    assert 0.999 < rho < 1.0
    assert 0.999 < gold["ladybug_49"] < 1.0 and 0.999 < gold["trafalgar_193"] < 1.0


@pytest.mark.parametrize("lam", [1e-2, 1.0])
@pytest.mark.parametrize("m", [0, 3, 10])
def test_prop1_remainder(lam, m):
    """R = sum_{i>m} M^i = M^{m+1}(I - M)^-1.  For the symmetric similar matrix
    the spectral norm equals rho and the bound of eq. bounded is attained with
    equality; for P itself rho(R) = rho^{m+1} / (1 - rho) exactly."""
    P = c1()
    J = dense.dense_jacobian(P.Jp, P.Jl, P.obs_cam, P.obs_lm, P.n_cams, P.n_lms)
    Ph = dense.symmetric_P(J, P.r, lam, P.n_cams)
    rho = float(np.linalg.eigvalsh(Ph).max())
    bound = rho ** (m + 1) / (1 - rho)
    Rh = dense.series_remainder(Ph, m)
    assert np.linalg.norm(Rh, 2) <= bound * (1 + 1e-8)
    assert abs(np.linalg.norm(Rh, 2) - bound) <= 1e-6 * bound
    # the remainder sums the tail: (I - M)^-1 - sum_{i<=m} M^i
    n = Ph.shape[0]
    partial = sum(np.linalg.matrix_power(Ph, i) for i in range(m + 1))
    assert rel(Rh, np.linalg.inv(np.eye(n) - Ph) - partial) < 1e-9
    Pm, _, _, _ = dense.P_matrix(J, P.r, lam, P.n_cams)
    R = dense.series_remainder(Pm, m)
    assert abs(dense.spectral_radius(R) - bound) <= 1e-6 * bound


def test_convergence_rate_in_U_norm():
    """||x(m) - dx_p||_U <= rho^{m+1} ||dx_p||_U and the error ratio tends to rho."""
    P = c1()
    lam = 1e-2
    J = dense.dense_jacobian(P.Jp, P.Jl, P.obs_cam, P.obs_lm, P.n_cams, P.n_lms)
    dxp, _, _, _ = dense.full_step(J, P.r, lam, P.n_cams)
    Pm, U, S, bt = dense.P_matrix(J, P.r, lam, P.n_cams)
    rho = float(np.linalg.eigvalsh(dense.symmetric_P(J, P.r, lam, P.n_cams)).max())
    w, Q = np.linalg.eigh(U)
    Uh = Q @ np.diag(np.sqrt(w)) @ Q.T
    unorm = lambda y: np.linalg.norm(Uh @ y)
    sol = schur.solve(P.Jp, P.Jl, P.r, P.obs_cam, P.obs_lm, P.n_cams, P.n_lms, lam, 400, 0.0)
    errs = [unorm(x.ravel() - dxp) for x in sol.series.iterates]
    e0 = unorm(dxp)
    for m, e in enumerate(errs):
        assert e <= rho ** (m + 1) * e0 * (1 + 1e-6) + 1e-12 * e0
    ratio = errs[300] / errs[299]
    assert abs(ratio - rho) < 1e-3


def test_truncated_inverse_is_symmetric():
    P = c1()
    J = dense.dense_jacobian(P.Jp, P.Jl, P.obs_cam, P.obs_lm, P.n_cams, P.n_lms)
    Pm, U, S, bt = dense.P_matrix(J, P.r, 1e-2, P.n_cams)
    St = dense.S_tilde(Pm, U, 7)
    assert np.linalg.norm(St - St.T) <= 1e-10 * np.linalg.norm(St)


def test_identity_damping_large_lambda_gives_scaled_gradient():
    P = c1()
    lam = 1e14
    sol = schur.solve(P.Jp, P.Jl, P.r, P.obs_cam, P.obs_lm, P.n_cams, P.n_lms, lam, 5, 0.0,
                      damping="identity")
    assert rel(sol.dxp, -sol.btilde / lam) < 1e-6


def test_stop_rule_first_order_meeting_criterion():
    """eq. qcriterion: the series stops at the first order i >= 1 with
    (i + 1) ||x(i) - x(i-1)|| / ||x(i)|| < eps."""
    P = c1()
    eps = 0.05
    full = schur.solve(P.Jp, P.Jl, P.r, P.obs_cam, P.obs_lm, P.n_cams, P.n_lms, 1.0, 60, 0.0)
    it = full.series.iterates
    crit = [(i + 1) * np.linalg.norm(it[i] - it[i - 1]) / np.linalg.norm(it[i]) for i in range(1, 61)]
    expect = 1 + next(i for i, c in enumerate(crit) if c < eps)
    sol = schur.solve(P.Jp, P.Jl, P.r, P.obs_cam, P.obs_lm, P.n_cams, P.n_lms, 1.0, 60, eps)
    assert sol.series.stop_order == expect and sol.series.stopped_by_rule
    assert rel(sol.dxp, it[expect]) < 1e-14
