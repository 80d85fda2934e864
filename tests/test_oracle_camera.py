"""Pins of the oracle's camera model and Jacobian blocks (CPU).

The paper prints no projection values, so the pins are special cases with a
closed form, an independent library rotation (scipy), and derivatives by the
complex-step method and central differences."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import camera
from oracle_fixtures import c1, rel


def _random_rotvecs(rng, n):
    axes = rng.normal(size=(n, 3))
    axes /= np.linalg.norm(axes, axis=1, keepdims=True)
    angles = np.concatenate([rng.uniform(0, np.pi, n - 4), [1e-13, 1e-9, 1e-5, np.pi - 1e-6]])
    return axes * angles[:, None]


def test_rotation_matches_scipy():
    rng = np.random.default_rng(0)
    w = _random_rotvecs(rng, 64)
    X = rng.normal(size=(64, 3)) * 5
    ref = Rotation.from_rotvec(w).apply(X)
    np.testing.assert_allclose(camera.rotate(w, X), ref, rtol=0, atol=1e-13)


def _scene_point(cam, Pc):
    """World point whose camera-frame coordinates are Pc (scipy rotation)."""
    R = Rotation.from_rotvec(cam[0:3]).as_matrix()
    return R.T @ (Pc - cam[3:6])


def test_optical_axis_projects_to_origin():
    cam = np.array([0.3, -0.2, 0.5, 1.0, 2.0, -3.0, 500.0, 1e-3, -2e-3])
    X = _scene_point(cam, np.array([0.0, 0.0, -7.0]))
    px = camera.project(cam[None], X[None], [0], [0])
    np.testing.assert_allclose(px, 0.0, atol=1e-10)


def test_pinhole_reduction_and_distortion():
    rng = np.random.default_rng(1)
    cams = np.concatenate([_random_rotvecs(rng, 16), rng.normal(size=(16, 3)),
                           rng.uniform(400, 600, (16, 1)), np.zeros((16, 2))], axis=1)
    Pc = np.column_stack([rng.normal(size=(16, 2)), -rng.uniform(2, 9, 16)])
    X = np.array([_scene_point(cams[i], Pc[i]) for i in range(16)])
    idx = np.arange(16)
    pin = -cams[:, 6:7] * Pc[:, 0:2] / Pc[:, 2:3]
    np.testing.assert_allclose(camera.project(cams, X, idx, idx), pin, rtol=1e-12)
    cams[:, 7] = 0.01
    cams[:, 8] = -0.002
    p = -Pc[:, 0:2] / Pc[:, 2:3]
    r2 = np.sum(p * p, axis=1)
    dist = (1 + 0.01 * r2 - 0.002 * r2 ** 2)[:, None] * pin
    np.testing.assert_allclose(camera.project(cams, X, idx, idx), dist, rtol=1e-12)


def test_mirrored_points_give_mirrored_pixels():
    cam = np.array([0.1, 0.7, -0.4, 0.5, 0.0, 1.0, 520.0, 2e-3, 1e-3])
    a = _scene_point(cam, np.array([0.4, -0.3, -5.0]))
    b = _scene_point(cam, np.array([-0.4, 0.3, -5.0]))
    pa = camera.project(cam[None], a[None], [0], [0])
    pb = camera.project(cam[None], b[None], [0], [0])
    np.testing.assert_allclose(pa, -pb, rtol=1e-12)


def test_jacobians_match_complex_step():
    P = c1()
    Jp, Jl = camera.jacobians(P.cams, P.lms, P.obs_cam, P.obs_lm)
    Jpc, Jlc = camera.complex_step_jacobians(P.cams, P.lms, P.obs_cam, P.obs_lm)
    ep = np.linalg.norm(Jp - Jpc, axis=(1, 2)) / np.linalg.norm(Jpc, axis=(1, 2))
    el = np.linalg.norm(Jl - Jlc, axis=(1, 2)) / np.linalg.norm(Jlc, axis=(1, 2))
    assert ep.max() < 1e-12 and el.max() < 1e-12


def test_jacobians_match_central_differences():
    P = c1()
    Jp, Jl = camera.jacobians(P.cams, P.lms, P.obs_cam, P.obs_lm)
    Jpf, Jlf = camera.central_difference_jacobians(P.cams, P.lms, P.obs_cam, P.obs_lm)
    assert rel(Jp, Jpf) < 1e-6 and rel(Jl, Jlf) < 1e-6


@pytest.mark.parametrize("angle", [0.0, 1e-12, 1e-7, 1e-3])
def test_rotation_derivative_small_angles(angle):
    """At omega = 0, d(R X)/d omega = -[X]x; small angles stay continuous."""
    rng = np.random.default_rng(2)
    axis = rng.normal(size=3)
    axis /= np.linalg.norm(axis)
    cam = np.concatenate([axis * angle, [0.2, -0.1, 8.0], [480.0, 0.0, 0.0]])
    X = np.array([[0.3, -0.4, -1.0]])
    Jp, _ = camera.jacobians(cam[None], X, [0], [0])
    Jpc, _ = camera.complex_step_jacobians(cam[None], X, [0], [0])
    np.testing.assert_allclose(Jp, Jpc, rtol=1e-10, atol=1e-9)
    if angle == 0.0:
        # dpi/dP times -[X]x
        Jt = Jp[0, :, 3:6]
        Xs = X[0]
        skew = np.array([[0, -Xs[2], Xs[1]], [Xs[2], 0, -Xs[0]], [-Xs[1], Xs[0], 0]])
        np.testing.assert_allclose(Jp[0, :, 0:3], Jt @ (-skew), rtol=1e-12, atol=1e-12)
