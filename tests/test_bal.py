"""The BAL text reader and writer: exact round trips, a hand-written fixture
(tests/golden/bal_tiny.txt, invented values in the format's layout: header
"cameras points observations", one "camera point x y" line per observation,
then 9 values per camera and 3 per point), malformed files, and the format's
documented camera model against the oracle's projection."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from paper_2204_12834_amd import bal, synth
from oracle import camera

GOLDEN = __file__.rsplit("/", 1)[0] + "/golden/bal_tiny.txt"


def test_fixture_values():
    p = bal.read(GOLDEN)
    assert (p.n_cams, p.n_lms, p.n_obs) == (2, 3, 5)
    np.testing.assert_array_equal(p.obs_cam, [0, 0, 1, 1, 0])
    np.testing.assert_array_equal(p.obs_lm, [0, 1, 0, 2, 2])
    np.testing.assert_array_equal(p.obs_xy[3], [21.75, 0.5])
    np.testing.assert_array_equal(p.cams[0], [0.01, -0.02, 0.005, 0.1, -0.2, -8.0, 500.0, -0.001, 0.0002])
    np.testing.assert_array_equal(p.cams[1, 6:], [480.0, 0.0005, -0.0001])
    np.testing.assert_array_equal(p.lms[2], [1.1, 0.6, -0.8])
    assert p.obs_cam.dtype == np.int32 and p.obs_xy.dtype == np.float64


def test_format_camera_model_is_the_oracle_model():
    """P = R(w) X + t (Rodrigues), p = -P_xy / P_z, f (1 + k1 |p|^2 + k2 |p|^4) p."""
    p = bal.read(GOLDEN)
    ref = []
    for c, l in zip(p.obs_cam, p.obs_lm):
        w, t, (f, k1, k2) = p.cams[c, :3], p.cams[c, 3:6], p.cams[c, 6:]
        P = Rotation.from_rotvec(w).apply(p.lms[l]) + t
        q = -P[:2] / P[2]
        n = q @ q
        ref.append(f * (1.0 + k1 * n + k2 * n * n) * q)
    out = camera.project(p.cams, p.lms, p.obs_cam, p.obs_lm)
    np.testing.assert_allclose(out, np.array(ref), rtol=1e-13, atol=1e-10)


@pytest.mark.parametrize("suffix", ["txt", "txt.bz2"])
def test_round_trip_is_exact(tmp_path, suffix):
    s = synth.config("c1")
    obs = camera.project(s.cams_gt, s.lms_gt, s.obs_cam, s.obs_lm) + s.noise
    p = bal.from_scene(s, obs)
    path = str(tmp_path / f"c1.{suffix}")
    bal.write(path, p)
    q = bal.read(path)
    for a in ["obs_cam", "obs_lm", "obs_xy", "cams", "lms"]:
        np.testing.assert_array_equal(getattr(q, a), getattr(p, a))


def _write(tmp_path, text):
    path = str(tmp_path / "bad.txt")
    with open(path, "w") as f:
        f.write(text)
    return path


def test_malformed_files_raise(tmp_path):
    good = open(GOLDEN).read()
    with pytest.raises(ValueError):  # one value missing
        bal.read(_write(tmp_path, good.rsplit("\n", 2)[0] + "\n"))
    with pytest.raises(ValueError):  # camera index out of range
        bal.read(_write(tmp_path, good.replace("1 2 21.75", "2 2 21.75")))
    with pytest.raises(ValueError):  # non-integral point index
        bal.read(_write(tmp_path, good.replace("0 1 3.0", "0 1.5 3.0")))
    with pytest.raises(ValueError):  # header
        bal.read(_write(tmp_path, "2 x 5\n"))
