"""Pins of the oracle's inverse for damped blocks that are not positive
definite (CPU only).

Sec. 4.1 takes U_lambda and V_lambda to be positive definite.  Where a block
is not (set from elsewhere, or holding a non-finite entry), the reading used is
that its inverse is replaced by the inverse of its damping diagonal alone,
diag(1 / (lambda d_j)), 0 where lambda d_j is not positive; the step is then
the exact step of the system in which that damped block is lambda diag(d)."""
import math

import numpy as np
import pytest

from oracle import dense, lm, normal, schur
from oracle_fixtures import c1, rel


def _spd(rng, k, cond=1e3):
    Q, _ = np.linalg.qr(rng.normal(size=(k, k)))
    ev = np.geomspace(1.0, cond, k)
    return Q @ np.diag(ev) @ Q.T


def test_positive_definite_blocks_are_inverted_exactly():
    rng = np.random.default_rng(0)
    for k in (3, 9):
        A = np.stack([_spd(rng, k) for _ in range(5)])
        inv, bad = normal.damped_inverse(A, np.ones((5, k)))
        assert not bad.any()
        for a, b in zip(A, inv):
            assert np.abs(a @ b - np.eye(k)).max() < 1e-11


def test_indefinite_3x3_takes_the_damping_diagonal():
    # eigenvalues 3.01, -0.99, 1.01: indefinite with a positive diagonal
    A = np.array([[[1.01, 2.0, 0.0], [2.0, 1.01, 0.0], [0.0, 0.0, 1.01]]])
    assert np.linalg.eigvalsh(A[0]).min() < 0.0
    lam_d = np.array([[0.01, 0.02, 0.04]])
    inv, bad = normal.damped_inverse(A, lam_d)
    assert bad.tolist() == [True]
    np.testing.assert_array_equal(inv[0], np.diag([100.0, 50.0, 25.0]))


def test_indefinite_9x9_takes_the_damping_diagonal_with_zero_entries():
    rng = np.random.default_rng(1)
    Q, _ = np.linalg.qr(rng.normal(size=(9, 9)))
    A = (Q @ np.diag([5.0, 4.0, 3.0, 2.0, 1.0, 0.5, 0.2, -0.3, 1.5]) @ Q.T)[None]
    lam_d = np.array([[0.5, 0.25, 2.0, 0.0, 1.0, 4.0, 8.0, 0.125, 1.0]])
    inv, bad = normal.damped_inverse(A, lam_d)
    assert bad.tolist() == [True]
    want = np.diag([2.0, 4.0, 0.5, 0.0, 1.0, 0.25, 0.125, 8.0, 1.0])
    np.testing.assert_array_equal(inv[0], want)


def test_zero_pivot_and_non_finite_blocks_fall_back():
    # positive semidefinite and singular: the second Cholesky pivot is exactly 0
    A0 = np.array([[1.0, 1.0, 0.0], [1.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    A1 = np.eye(3)
    A1[1, 2] = A1[2, 1] = math.nan
    A = np.stack([A0, A1])
    inv, bad = normal.damped_inverse(A, np.full((2, 3), 0.5))
    assert bad.tolist() == [True, True]
    np.testing.assert_array_equal(inv, np.stack([2.0 * np.eye(3)] * 2))


def test_only_the_failing_block_of_a_stack_falls_back():
    rng = np.random.default_rng(2)
    good0, good1 = _spd(rng, 3), _spd(rng, 3)
    badb = np.array([[1.0, 3.0, 0.0], [3.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    A = np.stack([good0, badb, good1])
    inv, bad = normal.damped_inverse(A, np.ones((3, 3)))
    assert bad.tolist() == [False, True, False]
    assert np.abs(inv[0] @ good0 - np.eye(3)).max() < 1e-12
    assert np.abs(inv[2] @ good1 - np.eye(3)).max() < 1e-12
    np.testing.assert_array_equal(inv[1], np.eye(3))


def _indefinite_landmark_case(lam):
    """c1 with landmark 7's undamped V replaced by an indefinite block whose
    diagonal is ten times the largest diagonal entry of the true block, so
    that lambda diag(d) dominates the true damped block (lambda = 1) and the
    system stays positive definite."""
    P = c1()
    U, V, bp, bl = normal.assemble(P.Jp, P.Jl, P.r, P.obs_cam, P.obs_lm, P.n_cams, P.n_lms)
    l = 7
    a = 10.0 * np.diag(V[l]).max()
    Vb = V.copy()
    Vb[l] = np.array([[a, 2.0 * a, 0.0], [2.0 * a, a, 0.0], [0.0, 0.0, a]])
    return P, U, V, Vb, bp, bl, l


def test_step_with_fallback_equals_dense_solve_of_the_modified_system():
    """The series with a large order and the back-substitution reach the dense
    LAPACK solve of eq. normal in which the damped block of landmark 7 is
    lambda diag(d_7) (d from the replaced block's diagonal)."""
    lam = 1.0
    P, U, V, Vb, bp, bl, l = _indefinite_landmark_case(lam)
    sol = schur.solve(P.Jp, P.Jl, P.r, P.obs_cam, P.obs_lm, P.n_cams, P.n_lms, lam, 200, 0.0,
                      landmark_blocks=(Vb, bl))
    assert sol.not_spd == 1
    J = dense.dense_jacobian(P.Jp, P.Jl, P.obs_cam, P.obs_lm, P.n_cams, P.n_lms)
    d = dense.damping_matrix(J, P.n_cams)
    H = J.T @ J + lam * np.diag(d)
    k = 9 * P.n_cams + 3 * l
    dl = np.clip(np.diag(Vb[l]), normal.DIAG_MIN, normal.DIAG_MAX)
    H[k:k + 3, k:k + 3] = lam * np.diag(dl)
    g = J.T @ P.r.reshape(-1)
    assert np.linalg.eigvalsh(H).min() > 0.0
    dx = -np.linalg.solve(H, g)
    assert rel(sol.dxp, dx[:9 * P.n_cams]) < 1e-10
    assert rel(sol.dxl, dx[9 * P.n_cams:]) < 1e-10
    # with the true block no fallback is taken
    ok = schur.solve(P.Jp, P.Jl, P.r, P.obs_cam, P.obs_lm, P.n_cams, P.n_lms, lam, 5, 0.0,
                     landmark_blocks=(V, bl))
    assert ok.not_spd == 0


def test_lm_rejects_a_step_with_a_non_finite_observation():
    """One observation is NaN: F is NaN, so no step has a finite gain ratio;
    every step is rejected and lambda grows by nu = 2, 4, 8, ..."""
    P = c1()
    obs = P.obs.copy()
    obs[5, 1] = math.nan
    opts = lm.LMOptions(max_iters=3, m=5)
    res = lm.lm(P.cams, P.lms, P.obs_cam, P.obs_lm, obs, opts)
    assert [it.accepted for it in res.iterations] == [False, False, False]
    assert all(math.isnan(it.cost) for it in res.iterations)
    assert [it.lam for it in res.iterations] == pytest.approx([1e-4, 2e-4, 8e-4])
    np.testing.assert_array_equal(res.cams, P.cams)
