"""Edge cases of the HIP path: empty and ragged inputs, long segments that
span several 64-wide chunks, cameras split into many pieces, empty landmarks
and cameras, no observations at all, and out-of-range indices."""
import dataclasses

import numpy as np
import pytest

from paper_2204_12834_amd import synth
from gpu_common import Case, log, np_, rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _ragged_scene():
    """100 cameras on a ring; landmark 0 seen 150 times (with repeated
    cameras), landmark 1 seen 70 times, landmarks 2..5 unobserved, landmark 6
    seen once, the rest 2..6 times; camera 99 sees nothing."""
    base = synth.ring_scene(100, 400, (2, 6), seed=11, name="ragged")
    rng = np.random.default_rng(3)
    keep = (base.obs_cam != 99) & ~np.isin(base.obs_lm, [0, 1, 2, 3, 4, 5, 6])
    cams = [base.obs_cam[keep]]
    lms = [base.obs_lm[keep]]
    cams.append(rng.integers(0, 99, 150)); lms.append(np.zeros(150, np.int64))
    cams.append(rng.permutation(99)[:70]); lms.append(np.ones(70, np.int64))
    cams.append(np.array([5])); lms.append(np.array([6]))
    oc = np.concatenate(cams).astype(np.int32)
    ol = np.concatenate(lms).astype(np.int32)
    perm = rng.permutation(oc.size)
    oc, ol = oc[perm], ol[perm]
    noise = rng.normal(size=(oc.size, 2))
    return dataclasses.replace(base, obs_cam=oc, obs_lm=ol, noise=noise, outlier=np.zeros(oc.size, bool))


@pytest.mark.parametrize("piece,ranges", [(0, 0), (64, 0), (100, 0), (64, 8)])
@pytest.mark.parametrize("precision,records", [("f64", "jacobian"), ("f32", "jacobian"), ("f64", "point"),
                                               ("f32", "point")])
def test_ragged_segments_and_empty_entities(piece, ranges, precision, records):
    log(f"ragged piece={piece} ranges={ranges} {precision} {records}")
    case = Case(_ragged_scene())
    s = case.scene
    prob = case.problem(precision, piece_size=piece, lm_ranges=ranges, records=records)
    cams, lms = case.state()
    cost = prob.linearize(cams, lms)
    assert abs(cost.item() - case.F) <= 1e-12 * case.F
    tol = 1e-10 if precision == "f64" else 1e-4
    for lam in [1e-3, 1.0]:
        dxp, dxl, _ = prob.power_solve(lam, 15, 0.0)
        ref = case.solve(lam, 15)
        assert rel(np_(dxp), ref.dxp) <= tol and rel(np_(dxl), ref.dxl) <= tol
        dxl_ = np_(dxl)
        assert np.all(dxl_[2:6] == 0.0)        # unobserved landmarks do not move
        assert np.all(np_(dxp)[99] == 0.0)     # nor does the camera without observations


def test_no_observations():
    from paper_2204_12834_amd.solver import Problem
    prob = Problem(np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros((0, 2)), 3, 5, device="cuda")
    cams = torch.zeros(3, 9, dtype=torch.float64, device="cuda")
    cams[:, 5] = -5.0
    cams[:, 6] = 500.0
    lms = torch.zeros(5, 3, dtype=torch.float64, device="cuda")
    cost = prob.linearize(cams, lms)
    dxp, dxl, _ = prob.power_solve(1e-2, 5, 0.0)
    assert cost.item() == 0.0
    assert torch.all(dxp == 0) and torch.all(dxl == 0)


def test_out_of_range_index_is_rejected():
    from paper_2204_12834_amd._lib import PobaError
    from paper_2204_12834_amd.solver import Problem
    oc = np.array([0, 1, 2], np.int32)
    ol = np.array([0, 7, 1], np.int32)  # landmark 7 of 4
    with pytest.raises(PobaError) as e:
        Problem(oc, ol, np.zeros((3, 2)), 3, 4, device="cuda")
    assert e.value.code == 2


def test_single_observation_landmarks_and_single_camera():
    """A one-camera problem: every landmark seen once (V is singular without
    damping; the damped block is SPD)."""
    rng = np.random.default_rng(4)
    base = synth.ring_scene(1, 50, (1, 1), seed=9, name="single")
    case = Case(base)
    prob = case.problem("f64")
    cams, lms = case.state()
    prob.linearize(cams, lms)
    dxp, dxl, info = prob.power_solve(1e-2, 10, 0.0)
    ref = case.solve(1e-2, 10)
    assert rel(np_(dxp), ref.dxp) <= 1e-10 and rel(np_(dxl), ref.dxl) <= 1e-10
