"""The synthetic workloads' initial state (CPU only).

The initial state perturbs each camera about its own centre: centre moved by
N(0, 0.1^2 I) world units, orientation by a rotation of angle-axis
N(0, 0.01^2 I), translation t0 = -R0 c0 (App. B perturbs camera positions).
A perturbation of the angle-axis vector at fixed t would instead move a
camera's centre by about 0.01 |t|, tens of units on the long vehicle path."""
import math

import numpy as np
import pytest

from oracle import camera
from paper_2204_12834_amd import synth


def _centres(cams):
    # c = -R^T t, with R from the oracle's rotation of the unit vectors
    eye = np.eye(3)
    n = cams.shape[0]
    R = np.stack([camera.rotate(cams[:, 0:3], np.broadcast_to(eye[j], (n, 3))) for j in range(3)], axis=2)
    return -np.einsum("nji,nj->ni", R, cams[:, 3:6]), R


@pytest.mark.parametrize("name", ["c1", "c2", "c3", "c5", "c4"])
def test_initial_state_is_in_front_of_every_camera(name):
    scenes = synth.config(name)
    for s in scenes if isinstance(scenes, list) else [scenes]:
        P = camera.camera_points(s.cams0, s.lms0, s.obs_cam, s.obs_lm)
        assert P[:, 2].max() < -0.1, (s.name, P[:, 2].max())


@pytest.mark.parametrize("name", ["c2", "c3"])
def test_initial_perturbation_moves_centres_by_the_stated_sigma(name):
    s = synth.config(name)
    c_gt, R_gt = _centres(s.cams_gt)
    c0, R0 = _centres(s.cams0)
    shift = np.linalg.norm(c0 - c_gt, axis=1)
    # |N(0, s^2 I_3)| has mean s * 2 sqrt(2/pi) (chi distribution, 3 dof)
    mean = 0.1 * 2.0 * math.sqrt(2.0 / math.pi)
    assert abs(shift.mean() - mean) < 0.05 * mean
    assert shift.max() < 0.6
    # relative rotation R0 R^T: angle ~ |N(0, 0.01^2 I_3)|
    Rrel = np.einsum("nij,nkj->nik", R0, R_gt)
    ang = np.arccos(np.clip((np.trace(Rrel, axis1=1, axis2=2) - 1.0) / 2.0, -1.0, 1.0))
    assert abs(ang.mean() - 0.01 * 2.0 * math.sqrt(2.0 / math.pi)) < 0.1 * 0.016
    # intrinsics start at ground truth
    np.testing.assert_array_equal(s.cams0[:, 6:9], s.cams_gt[:, 6:9])


def test_angle_axis_initial_state_is_the_earlier_one():
    """x0 = "angle-axis" (kept to reproduce measurements made with the earlier
    initial state) adds the noise to the angle-axis vector and to t; it draws
    the same numbers in the same order as the default, so landmarks, noise
    and the camera noise itself are shared."""
    kw = dict(n_cams=60, n_lms=3000, seed=5, name="x0")
    a = synth.city_scene(**kw)
    b = synth.city_scene(**kw, x0="angle-axis")
    np.testing.assert_array_equal(a.lms0, b.lms0)
    np.testing.assert_array_equal(a.noise, b.noise)
    d = b.cams0 - b.cams_gt
    assert np.all(d[:, 6:9] == 0.0)
    assert abs(d[:, 0:3].std() - 0.01) < 0.002 and abs(d[:, 3:6].std() - 0.1) < 0.02
    # the centre then moves by about 0.01 |t|, more than the default's 0.1
    c_gt, _ = _centres(b.cams_gt)
    shift_b = np.linalg.norm(_centres(b.cams0)[0] - c_gt, axis=1)
    shift_a = np.linalg.norm(_centres(a.cams0)[0] - c_gt, axis=1)
    t = np.linalg.norm(b.cams_gt[:, 3:6], axis=1)
    assert np.median(shift_b / t) > 0.005 and np.median(shift_a) < 0.2
    with pytest.raises(ValueError):
        synth.city_scene(**kw, x0="other")
