"""A problem read from a BAL file runs through the same handle and LM steps
and follows the oracle's LM loop (Sec. 5.1) on the same data."""
import numpy as np
import pytest

from paper_2204_12834_amd import bal, synth
from gpu_common import log, np_, rel
from oracle import camera, lm as olm

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("records", ["jacobian", "point"])
def test_bal_file_lm_matches_oracle(tmp_path, records):
    from paper_2204_12834_amd.solver import LMOptions, Problem, read_lm_state
    s = synth.config("c1")
    obs = camera.project(s.cams_gt, s.lms_gt, s.obs_cam, s.obs_lm) + s.noise
    path = str(tmp_path / "ring.txt.bz2")
    bal.write(path, bal.from_scene(s, obs))
    p = bal.read(path)
    log(f"bal {p.n_cams} cams {p.n_lms} lms {p.n_obs} obs, {records}")
    opts = olm.LMOptions(max_iters=6, m=20, eps=0.0)
    ref = olm.lm(p.cams, p.lms, p.obs_cam, p.obs_lm, p.obs_xy, opts)
    prob = Problem(p.obs_cam, p.obs_lm, p.obs_xy, p.n_cams, p.n_lms, precision="f64", device="cuda",
                   records=records)
    cams = torch.tensor(p.cams, device="cuda")
    lms = torch.tensor(p.lms, device="cuda")
    o = LMOptions(lambda0=opts.lambda0, func_tol=opts.func_tol, eps=opts.eps, eta=opts.eta, m=opts.m,
                  max_iters=opts.max_iters)
    st = prob.lm_init(o)
    costs = []
    for _ in range(len(ref.iterations)):
        prob.lm_step(cams, lms, st, o)
        costs.append(read_lm_state(st)["cost_new"])
    for g, it in zip(costs, ref.iterations):
        assert abs(g - it.cost_new) <= 1e-9 * it.cost_new
    assert rel(np_(cams), ref.cams) < 1e-8 and rel(np_(lms), ref.lms) < 1e-8
