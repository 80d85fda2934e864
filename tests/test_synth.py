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
