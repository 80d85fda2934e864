"""Batched problems (poba_batch_create) and LM iterations captured in a HIP
graph.  Invariant: every problem of a batch gets the result it would get on
its own (oracle per problem; solo GPU handles for LM trajectories)."""
import functools

import numpy as np
import pytest

from paper_2204_12834_amd import synth
from gpu_common import log, np_, observations, rel
from oracle import camera, lm, schur

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=None)
def batch():
    # uneven sizes; one with a heavy landmark count so tiles and ranges cross problems
    scenes = [synth.ring_scene(nc, nl, (2, 8), seed=100 + k, name=f"b{k}")
              for k, (nc, nl) in enumerate([(5, 200), (23, 3000), (12, 40), (60, 9000), (8, 700)])]
    cat, co, lo = synth.concat_scenes(scenes)
    obs = [observations(s) for s in scenes]
    return scenes, cat, co, lo, np.concatenate(obs)


def _problem(precision="f64", lm_ranges=0, piece_size=0, records="jacobian"):
    from paper_2204_12834_amd.solver import Problem
    scenes, cat, co, lo, obs = batch()
    return Problem(cat.obs_cam, cat.obs_lm, obs, cat.n_cams, cat.n_lms, precision=precision, device="cuda",
                   prob_cam_off=co, prob_lm_off=lo, lm_ranges=lm_ranges, piece_size=piece_size, records=records)


def _state():
    scenes, cat, co, lo, obs = batch()
    return (torch.tensor(cat.cams0, device="cuda"), torch.tensor(cat.lms0, device="cuda"))


@pytest.mark.parametrize("precision,tol,ranges,piece,records", [("f64", 1e-10, 0, 0, "jacobian"),
                                                               ("f64", 1e-10, 8, 64, "jacobian"),
                                                               ("f32", 1e-4, 0, 0, "jacobian"),
                                                               ("f64", 1e-10, 8, 64, "point"),
                                                               ("f32", 1e-4, 0, 0, "point")])
def test_batched_solve_matches_each_problem(precision, tol, ranges, piece, records):
    scenes, cat, co, lo, obs = batch()
    prob = _problem(precision, ranges, piece, records)
    cams, lms = _state()
    cost = np_(prob.linearize(cams, lms))
    lam, m = 1e-2, 20
    dxp, dxl, info = prob.power_solve(lam, m, 0.0)
    dxp, dxl = np_(dxp), np_(dxl)
    for k, s in enumerate(scenes):
        o = obs[sum(x.n_obs for x in scenes[:k]):][:s.n_obs]
        F, r, Jp, Jl = lm.linearize(s.cams0, s.lms0, s.obs_cam, s.obs_lm, o)
        assert abs(cost[k] - F) <= 1e-12 * F, k
        ref = schur.solve(Jp, Jl, r, s.obs_cam, s.obs_lm, s.n_cams, s.n_lms, lam, m)
        ep = rel(dxp[co[k]:co[k + 1]], ref.dxp)
        el = rel(dxl[lo[k]:lo[k + 1]], ref.dxl)
        log(f"batch {precision} problem {k}: dx_p {ep:.2e} dx_l {el:.2e}")
        assert ep <= tol and el <= tol, (k, ep, el)


def test_batched_stop_rule_is_per_problem():
    from paper_2204_12834_amd.solver import read_solve_info
    scenes, cat, co, lo, obs = batch()
    prob = _problem("f64")
    cams, lms = _state()
    prob.linearize(cams, lms)
    lam, m, eps = 1.0, 60, 0.02
    dxp, dxl, info = prob.power_solve(lam, m, eps)
    dxp = np_(dxp)
    for k, s in enumerate(scenes):
        o = obs[sum(x.n_obs for x in scenes[:k]):][:s.n_obs]
        F, r, Jp, Jl = lm.linearize(s.cams0, s.lms0, s.obs_cam, s.obs_lm, o)
        ref = schur.solve(Jp, Jl, r, s.obs_cam, s.obs_lm, s.n_cams, s.n_lms, lam, m, eps)
        it = ref.series.iterates
        crit = [(i + 1) * np.linalg.norm(it[i] - it[i - 1]) / np.linalg.norm(it[i]) for i in range(1, len(it))]
        if min(abs(c - eps) for c in crit) < 1e-9 * eps:
            continue
        inf = read_solve_info(info, k)
        assert inf["stop_order"] == ref.series.stop_order, (k, inf, ref.series.stop_order)
        assert rel(dxp[co[k]:co[k + 1]], ref.dxp) <= 1e-10


def test_observation_across_problems_is_rejected():
    from paper_2204_12834_amd._lib import PobaError
    from paper_2204_12834_amd.solver import Problem
    # problems: cameras {0, 1} / {2, 3}, landmarks {0, 1, 2} / {3, 4, 5}
    oc = np.array([0, 1, 2, 3], np.int32)
    ol = np.array([5, 1, 4, 3], np.int32)  # camera 0 with landmark 5 crosses problems
    with pytest.raises(PobaError) as e:
        Problem(oc, ol, np.zeros((4, 2)), 4, 6, device="cuda", prob_cam_off=[0, 2, 4], prob_lm_off=[0, 3, 6])
    assert e.value.code == 2


def _lm_run(prob, cams, lms, iters, opts):
    from paper_2204_12834_amd.solver import read_lm_states
    st = prob.lm_init(opts)
    hist = []
    for _ in range(iters):
        prob.lm_step(cams, lms, st, opts)
        hist.append(read_lm_states(st))
    return hist


def test_batched_lm_matches_solo_handles():
    """Six LM iterations of the batch against each problem on a handle of its
    own: same accept decisions and costs within float64 rounding."""
    from paper_2204_12834_amd.solver import LMOptions, Problem
    scenes, cat, co, lo, obs = batch()
    opts = LMOptions(m=10, eps=0.0, max_iters=50)
    prob = _problem("f64")
    cams, lms = _state()
    hb = _lm_run(prob, cams, lms, 6, opts)
    cams_b, lms_b = np_(cams), np_(lms)
    off = 0
    for k, s in enumerate(scenes):
        o = obs[off:off + s.n_obs]
        off += s.n_obs
        solo = Problem(s.obs_cam, s.obs_lm, o, s.n_cams, s.n_lms, precision="f64", device="cuda")
        c1 = torch.tensor(s.cams0, device="cuda")
        l1 = torch.tensor(s.lms0, device="cuda")
        hs = _lm_run(solo, c1, l1, 6, opts)
        for it in range(6):
            a, b = hb[it][k], hs[it][0]
            assert a["accepted"] == b["accepted"] and a["iteration"] == b["iteration"], (k, it, a, b)
            assert abs(a["cost"] - b["cost"]) <= 1e-9 * b["cost"], (k, it, a["cost"], b["cost"])
            assert abs(a["lambda"] - b["lambda"]) <= 1e-9 * b["lambda"]
        assert rel(cams_b[co[k]:co[k + 1]], np_(c1)) <= 1e-8
        assert rel(lms_b[lo[k]:lo[k + 1]], np_(l1)) <= 1e-8


def test_lm_graph_replays_eager_steps():
    """A graph of 4 LM steps equals 4 eager steps (bitwise: the same kernels
    on the same data), replayed several times with eager work in between;
    a graph of max_iters steps runs every problem to its end."""
    from paper_2204_12834_amd.solver import LMOptions, read_lm_states
    opts = LMOptions(m=8, eps=0.01, max_iters=12)
    prob = _problem("f32")
    cams, lms = _state()
    st = prob.lm_init(opts)
    for _ in range(4):
        prob.lm_step(cams, lms, st, opts)
    ref = (np_(cams).copy(), np_(lms).copy(), read_lm_states(st))
    cams0, lms0 = _state()
    gc, gl = cams0.clone(), lms0.clone()
    gst = prob.lm_init(opts)
    graph = prob.lm_graph(gc, gl, gst, 4, opts)
    for rep in range(3):
        gc.copy_(cams0)
        gl.copy_(lms0)
        prob.lm_init(opts, gst)
        graph.launch()
        torch.cuda.synchronize()
        assert np.array_equal(np_(gc), ref[0]) and np.array_equal(np_(gl), ref[1]), rep
        assert read_lm_states(gst) == ref[2], rep
        # eager work on the same handle between replays
        prob.linearize(cams0, lms0)
        prob.power_solve(1e-2, 3, 0.0)
    full = prob.lm_graph(gc, gl, gst, opts.max_iters, opts)
    gc.copy_(cams0)
    gl.copy_(lms0)
    prob.lm_init(opts, gst)
    full.launch()
    torch.cuda.synchronize()
    states = read_lm_states(gst)
    assert all(s["done"] == 1 for s in states), states
    # the full run passes through the same first four steps; accepted costs only decrease
    assert all(s["cost"] <= s0["cost"] for s, s0 in zip(states, ref[2])), (states, ref[2])
    graph.close()
    full.close()
