"""Failure paths of the HIP path: damped blocks that are not positive
definite, and non-finite observations.  Both are ordinary numeric paths: the
kernels flag them in the device status word and carry on.

Sec. 4.1 takes U_lambda and V_lambda to be positive definite.  Reading for a
block that is not (set from outside, or holding a non-finite entry): its
inverse is that of its damping diagonal alone, diag(1 / (lambda d_j)), 0
where lambda d_j <= 0, and POBA_ERR_NOT_SPD is raised; the oracle follows the
same reading (normal.damped_inverse), so the step still matches it.  A
non-finite residual makes the cost non-finite, raises POBA_ERR_NONFINITE and
the LM step is rejected with the state left as it was."""
import functools

import numpy as np
import pytest

from paper_2204_12834_amd import synth
from gpu_common import Case, log, np_, observations, rel
from oracle import lm as olm
from oracle import normal, schur

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NOT_SPD, NONFINITE = 4, 8


@functools.lru_cache(maxsize=None)
def c1():
    return Case(synth.config("c1"))


def _indefinite_blocks(case, which):
    """The undamped landmark blocks V, b_l of the initial state, with the
    landmarks in `which` given indefinite blocks of positive diagonal (so
    that Marquardt damping keeps them indefinite at small lambda)."""
    s = case.scene
    _, V, _, bl = normal.assemble(case.Jp, case.Jl, case.r, s.obs_cam, s.obs_lm, s.n_cams, s.n_lms)
    V = V.copy()
    for k, l in enumerate(which):
        a = np.trace(V[l]) / 3.0
        # eigenvalues 3a, -a, a (k = 0) or a, a, -2a (k = 1): one pivot turns negative
        V[l] = a * (np.array([[1.0, 2.0, 0.0], [2.0, 1.0, 0.0], [0.0, 0.0, 1.0]]) if k % 2 == 0 else
                    np.array([[1.0, 0.0, 1.5], [0.0, 1.0, 1.5], [1.5, 1.5, 1.0]]))
    return V, bl


@pytest.mark.parametrize("precision,records", [("f64", "jacobian"), ("f32", "jacobian"), ("f64", "point"),
                                               ("f32", "point")])
def test_indefinite_landmark_block_falls_back_to_damping_diagonal(precision, records):
    case = c1()
    s = case.scene
    which = [3, 400]
    V, bl = _indefinite_blocks(case, which)
    prob = case.problem(precision, records=records)
    cams, lms = case.state()
    prob.linearize(cams, lms)
    prob.set_landmark_blocks(torch.tensor(V, device="cuda"), torch.tensor(bl, device="cuda"))
    from paper_2204_12834_amd.solver import read_solve_info
    tol = 1e-10 if precision == "f64" else 1e-4
    for lam in [1e-3, 1e-1]:
        dxp, dxl, info = prob.power_solve(lam, 10, 0.0)
        inf = read_solve_info(info)
        ref = schur.solve(case.Jp, case.Jl, case.r, s.obs_cam, s.obs_lm, s.n_cams, s.n_lms, lam, 10,
                          landmark_blocks=(V, bl))
        assert ref.not_spd == len(which)
        ep, el = rel(np_(dxp), ref.dxp), rel(np_(dxl), ref.dxl)
        log(f"indefinite V {precision} {records} lam={lam}: status {inf['status']} dx_p {ep:.2e} dx_l {el:.2e}")
        assert inf["status"] & NOT_SPD
        assert ep <= tol and el <= tol
        # the fallback inverse on the flagged landmarks: dx_l = -diag(1/(lam d)) (b_l + W^T dx_p)
        d = np.clip(np.diagonal(V[which], axis1=1, axis2=2), normal.DIAG_MIN, normal.DIAG_MAX)
        t = schur.apply_Wt(case.Jp, case.Jl, s.obs_cam, s.obs_lm, ref.dxp, s.n_lms)[which]
        want = -(bl[which] + t) / (lam * d)
        assert rel(np_(dxl)[which], want) <= tol


def test_positive_definite_blocks_leave_status_clear():
    case = c1()
    s = case.scene
    _, V, _, bl = normal.assemble(case.Jp, case.Jl, case.r, s.obs_cam, s.obs_lm, s.n_cams, s.n_lms)
    prob = case.problem("f64")
    cams, lms = case.state()
    prob.linearize(cams, lms)
    prob.set_landmark_blocks(torch.tensor(V, device="cuda"), torch.tensor(bl, device="cuda"))
    from paper_2204_12834_amd.solver import read_solve_info
    dxp, dxl, info = prob.power_solve(1e-3, 10, 0.0)
    assert read_solve_info(info)["status"] == 0
    ref = case.solve(1e-3, 10)
    assert rel(np_(dxp), ref.dxp) <= 1e-10 and rel(np_(dxl), ref.dxl) <= 1e-10
    # the flag of a solve does not outlive it: an indefinite block, then the real ones again
    Vb, blb = _indefinite_blocks(case, [7])
    prob.set_landmark_blocks(torch.tensor(Vb, device="cuda"), torch.tensor(blb, device="cuda"))
    _, _, info = prob.power_solve(1e-3, 10, 0.0)
    assert read_solve_info(info)["status"] & NOT_SPD
    prob.set_landmark_blocks(torch.tensor(V, device="cuda"), torch.tensor(bl, device="cuda"))
    _, _, info = prob.power_solve(1e-3, 10, 0.0)
    assert read_solve_info(info)["status"] == 0


@pytest.mark.parametrize("precision,records", [("f64", "jacobian"), ("f32", "jacobian"), ("f32", "point")])
def test_nonfinite_observation_rejects_the_step(precision, records):
    from paper_2204_12834_amd.solver import LMOptions, read_lm_state
    case = c1()
    s = case.scene
    obs = case.obs.copy()
    obs[17, 1] = np.nan
    from paper_2204_12834_amd.solver import Problem
    prob = Problem(s.obs_cam, s.obs_lm, obs, s.n_cams, s.n_lms, precision=precision, records=records,
                   device="cuda")
    cams, lms = case.state()
    c0, l0 = np_(cams).copy(), np_(lms).copy()
    o = LMOptions(max_iters=5)
    st = prob.lm_init(o)
    prob.lm_step(cams, lms, st, o)
    g = read_lm_state(st)
    log(f"nan observation {precision} {records}: {g}")
    assert g["status"] & NONFINITE
    assert g["accepted"] == 0 and not np.isfinite(g["cost"])
    assert np.array_equal(np_(cams), c0) and np.array_equal(np_(lms), l0)


def test_nonfinite_observation_stays_in_its_problem():
    """A batch of three problems with a NaN observation in the middle one:
    that problem is flagged and rejected, the other two take the oracle's
    first LM step."""
    from paper_2204_12834_amd.solver import LMOptions, Problem, read_lm_states
    scenes = [synth.ring_scene(nc, nl, (2, 6), seed=40 + k, name=f"nf{k}")
              for k, (nc, nl) in enumerate([(10, 300), (12, 400), (9, 250)])]
    cat, co, lo = synth.concat_scenes(scenes)
    obs_k = [observations(sc) for sc in scenes]
    obs_k[1][5, 0] = np.inf
    prob = Problem(cat.obs_cam, cat.obs_lm, np.concatenate(obs_k), cat.n_cams, cat.n_lms, precision="f64",
                   prob_cam_off=co, prob_lm_off=lo, device="cuda")
    cams = torch.tensor(cat.cams0, device="cuda")
    lms = torch.tensor(cat.lms0, device="cuda")
    opts = olm.LMOptions(max_iters=1, m=20, eps=0.0)
    o = LMOptions(lambda0=opts.lambda0, func_tol=opts.func_tol, eps=opts.eps, eta=opts.eta, m=opts.m,
                  max_iters=opts.max_iters)
    st = prob.lm_init(o)
    prob.lm_step(cams, lms, st, o)
    states = read_lm_states(st)
    assert states[1]["status"] & NONFINITE and states[1]["accepted"] == 0
    cams_, lms_ = np_(cams), np_(lms)
    np.testing.assert_array_equal(cams_[co[1]:co[2]], cat.cams0[co[1]:co[2]])
    np.testing.assert_array_equal(lms_[lo[1]:lo[2]], cat.lms0[lo[1]:lo[2]])
    for k in [0, 2]:
        sc = scenes[k]
        ref = olm.lm(sc.cams0, sc.lms0, sc.obs_cam, sc.obs_lm, obs_k[k], opts)
        it = ref.iterations[0]
        assert states[k]["status"] == 0
        assert states[k]["accepted"] == int(it.accepted)
        assert abs(states[k]["cost_new"] - it.cost_new) <= 1e-9 * it.cost_new
        assert rel(cams_[co[k]:co[k + 1]], ref.cams) < 1e-8 and rel(lms_[lo[k]:lo[k + 1]], ref.lms) < 1e-8
