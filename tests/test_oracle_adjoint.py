"""Pins of the oracle's adjoint of the damped step against brute force:
central differences of the step itself (linear in o, smooth in the
intrinsics), the symmetry of the truncated inverse, and the limit m -> inf."""
import functools

import numpy as np
import pytest

from paper_2204_12834_amd import synth
from oracle import adjoint, camera, schur


@functools.lru_cache(maxsize=None)
def tiny():
    s = synth.ring_scene(6, 120, (2, 5), seed=3, name="adj_tiny")
    obs = camera.project(s.cams_gt, s.lms_gt, s.obs_cam, s.obs_lm) + s.noise
    rng = np.random.default_rng(1)
    gp = rng.normal(size=(s.n_cams, 9))
    gl = rng.normal(size=(s.n_lms, 3))
    D = adjoint.damping_diagonals(s.cams0, s.lms0, s.obs_cam, s.obs_lm, obs)
    return s, obs, gp, gl, D


def _L(s, obs, gp, gl, D, lam, m, cams=None):
    dp, dl = adjoint.step(s.cams0 if cams is None else cams, s.lms0, s.obs_cam, s.obs_lm, obs, lam, m=m,
                          diagonals=D)
    return float(np.sum(gp * dp) + np.sum(gl * dl))


@pytest.mark.parametrize("m,lam", [(None, 1.0), (None, 1e-2), (3, 1e-2), (12, 1.0)])
def test_observation_gradient_is_exact(m, lam):
    """The step is linear in o, so central differences are exact up to
    rounding, for the dense step and for a truncated series alike."""
    s, obs, gp, gl, D = tiny()
    A = adjoint.adjoint(s.cams0, s.lms0, s.obs_cam, s.obs_lm, obs, lam, gp, gl, m=m, diagonals=D)
    rng = np.random.default_rng(5)
    for i in rng.choice(s.n_obs, 8, replace=False):
        for k in range(2):
            h = 1e-2
            op, om = obs.copy(), obs.copy()
            op[i, k] += h
            om[i, k] -= h
            fd = (_L(s, op, gp, gl, D, lam, m) - _L(s, om, gp, gl, D, lam, m)) / (2 * h)
            assert abs(fd - A.grad_obs[i, k]) <= 1e-7 * max(abs(fd), 1e-3), (i, k, fd, A.grad_obs[i, k])


def test_intrinsic_gradient_matches_central_differences():
    s, obs, gp, gl, D = tiny()
    lam = 1.0
    A = adjoint.adjoint(s.cams0, s.lms0, s.obs_cam, s.obs_lm, obs, lam, gp, gl, m=None, diagonals=D)
    scale = np.abs(A.grad_intr).max()
    for c in range(s.n_cams):
        for col, k in enumerate(adjoint.INTRINSICS):
            h = 1e-6 * max(1.0, abs(s.cams0[c, k]))
            cp, cm = s.cams0.copy(), s.cams0.copy()
            cp[c, k] += h
            cm[c, k] -= h
            fd = (_L(s, obs, gp, gl, D, lam, None, cp) - _L(s, obs, gp, gl, D, lam, None, cm)) / (2 * h)
            assert abs(fd - A.grad_intr[c, col]) <= 1e-6 * max(abs(fd), 1e-3 * scale), (c, k, fd,
                                                                                         A.grad_intr[c, col])


def test_truncated_inverse_is_symmetric_operator():
    """<a, Ht_m^-1 b> = <b, Ht_m^-1 a> for the matrix-free series with
    back-substitution: the reason the adjoint reuses the forward solve."""
    s, obs, gp, gl, D = tiny()
    r, Jp, Jl = adjoint.linearize(s.cams0, s.lms0, s.obs_cam, s.obs_lm, obs)
    rng = np.random.default_rng(7)
    a = (rng.normal(size=(s.n_cams, 9)), rng.normal(size=(s.n_lms, 3)))
    b = (rng.normal(size=(s.n_cams, 9)), rng.normal(size=(s.n_lms, 3)))
    for m in [0, 2, 7]:
        Ha = schur.solve(Jp, Jl, r, s.obs_cam, s.obs_lm, s.n_cams, s.n_lms, 1e-2, m, rhs=a, diagonals=D)
        Hb = schur.solve(Jp, Jl, r, s.obs_cam, s.obs_lm, s.n_cams, s.n_lms, 1e-2, m, rhs=b, diagonals=D)
        lhs = np.sum(a[0] * Hb.dxp) + np.sum(a[1] * Hb.dxl)
        rhs = np.sum(b[0] * Ha.dxp) + np.sum(b[1] * Ha.dxl)
        assert abs(lhs - rhs) <= 1e-11 * abs(lhs), (m, lhs, rhs)


def test_series_adjoint_tends_to_dense():
    s, obs, gp, gl, D = tiny()
    A = adjoint.adjoint(s.cams0, s.lms0, s.obs_cam, s.obs_lm, obs, 1.0, gp, gl, m=None, diagonals=D)
    errs = []
    for m in [2, 8, 30]:
        B = adjoint.adjoint(s.cams0, s.lms0, s.obs_cam, s.obs_lm, obs, 1.0, gp, gl, m=m, diagonals=D)
        errs.append(np.abs(B.grad_intr - A.grad_intr).max() / np.abs(A.grad_intr).max())
        assert np.abs(B.zp - A.zp).max() <= 2 * errs[-1] * np.abs(A.zp).max() + 1e-12
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-9, errs
