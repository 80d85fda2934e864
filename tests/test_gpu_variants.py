"""Parity of every landmark-pass variant of the series with the oracle.

The landmark pass of each series order (W^T v gathered per landmark, then
V^-1, Sec. 4.3 eqs. S_approx, x_approx) has two forms per record kind:

  camera vector staged in LDS    k_lm_pass_lds         stored blocks, n_c * 9 * s <= 64 KB
                                 k_lm_pass_pt_lds      point records, n_c * f * s <= the LDS budget
                                 k_lm_pass_pt_compact  float64 point records, otherwise where
                                                       n_c * 144 <= the LDS budget (R rebuilt
                                                       per observation)
  camera vector gathered from L2 k_lm_pass             stored blocks, otherwise (or lds_camera = 0)
                                 k_lm_pass_pt          point records, otherwise (or lds_camera = 0)

(s: bytes per vector scalar; f: the folded camera's padded stride, 28
scalars in float32 and 26 in float64; the LDS budget is the device's
per-workgroup limit, 160 KB on gfx950).  The L2 forms give each wavefront tiles_per_wave
64-observation landmark tiles.  These tests reach the L2 forms three ways:
forced through the tuning call, automatically on a ring of 2,048 cameras
(147 KB / 74 KB of float64 / float32 camera vector, 393 KB / 197 KB folded),
and automatically on a batch of 2,100 cameras; and they run the automatic
choice once on the full city workload against the oracle.

Tolerances as the other parity tests: float64 <= 1e-10 relative, float32
<= 1e-4 (2-norm, camera and landmark steps separately, fixed order, eps = 0).
"""
import functools

import numpy as np
import pytest

from paper_2204_12834_amd import synth
from gpu_common import Case, log, np_, observations, rel, round_bf16
from oracle import lm, schur

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-4}


@functools.lru_cache(maxsize=None)
def city_small():
    return Case(synth.city_scene(n_cams=60, n_lms=3000, seed=5, name="city_small"), delta=3.0)


@functools.lru_cache(maxsize=None)
def ladybug_small():
    return Case(synth.ladybug_scene(n_cams=120, n_lms=4000, seed=2, name="ladybug_small"))


@functools.lru_cache(maxsize=None)
def ring_2k():
    # 2,048 cameras: every record kind and precision gathers the camera vector from L2
    return Case(synth.ring_scene(2048, 12000, (2, 6), seed=11, name="ring_2k"))


SMALL = {"city_small": city_small, "ladybug_small": ladybug_small}


def _lm_pass_in_lds(n_cams, precision, records):
    s = 8 if precision == "f64" else 4
    if records == "jacobian":
        return n_cams * 9 * s <= 64 * 1024
    if precision == "f64":
        return n_cams * 144 <= 160 * 1024
    return n_cams * 28 * s <= 160 * 1024


@functools.lru_cache(maxsize=None)
def ring_1k():
    # 1,000 cameras: the float64 fold (208 KB) does not fit LDS, its compact
    # form (144 KB) does
    return Case(synth.ring_scene(1000, 8000, (2, 6), seed=13, name="ring_1k"))


def _check_step(prob, case, lam, m, tol, what):
    dxp, dxl, info = prob.power_solve(lam, m, 0.0)
    ref = case.solve(lam, m)
    ep, el = rel(np_(dxp), ref.dxp), rel(np_(dxl), ref.dxl)
    log(f"{what} lam={lam} m={m}: dx_p {ep:.2e} dx_l {el:.2e}")
    assert ep <= tol and el <= tol, (what, lam, ep, el)
    from paper_2204_12834_amd.solver import read_solve_info
    inf = read_solve_info(info)
    assert inf["stop_order"] == m and inf["status"] == 0


@pytest.mark.parametrize("name", list(SMALL))
@pytest.mark.parametrize("tpw", [1, 4, 8])
@pytest.mark.parametrize("precision,records", [("f64", "jacobian"), ("f32", "jacobian"), ("f64", "point"),
                                               ("f32", "point")])
def test_l2_landmark_pass_forced(name, tpw, precision, records):
    """lds_camera = 0: the L2 gather form at 1, 4 and 8 tiles per wavefront."""
    case = SMALL[name]()
    prob = case.problem(precision, records=records)
    prob.set_tuning("lds_camera", 0)
    prob.set_tuning("tiles_per_wave", tpw)
    assert prob.get_tuning("lds_camera") == 0 and prob.get_tuning("tiles_per_wave") == tpw
    cams, lms = case.state()
    prob.linearize(cams, lms)
    for lam, m in [(1e-4, 20), (1e-2, 1), (1.0, 20)]:
        _check_step(prob, case, lam, m, TOL[precision], f"l2 {name} tpw={tpw} {precision} {records}")


@pytest.mark.parametrize("name", list(SMALL))
@pytest.mark.parametrize("tpw", [1, 8])
def test_l2_landmark_pass_bf16_on_rounded_blocks(name, tpw):
    """bfloat16 Jacobian storage through the L2 form, against the oracle on
    its blocks rounded to bfloat16 (the float32 series arithmetic remains)."""
    case = SMALL[name]()
    s = case.scene
    prob = case.problem("bf16")
    prob.set_tuning("lds_camera", 0)
    prob.set_tuning("tiles_per_wave", tpw)
    cams, lms = case.state()
    prob.linearize(cams, lms)
    Jp, Jl = round_bf16(case.Jp), round_bf16(case.Jl)
    for lam in [1e-4, 1e-2]:
        dxp, dxl, _ = prob.power_solve(lam, 20, 0.0)
        ref = schur.solve(Jp, Jl, case.r, s.obs_cam, s.obs_lm, s.n_cams, s.n_lms, lam, 20)
        ep, el = rel(np_(dxp), ref.dxp), rel(np_(dxl), ref.dxl)
        log(f"bf16 l2 {name} tpw={tpw} lam={lam}: dx_p {ep:.2e} dx_l {el:.2e}")
        assert ep <= 1e-4 and el <= 1e-4


@pytest.mark.parametrize("name", list(SMALL))
@pytest.mark.parametrize("precision,records", [("f64", "jacobian"), ("f32", "point")])
def test_lds_and_l2_forms_agree(name, precision, records):
    """The two forms differ only in summation order."""
    case = SMALL[name]()
    cams, lms = case.state()
    out = []
    for lds in [1, 0]:
        prob = case.problem(precision, records=records)
        prob.set_tuning("lds_camera", lds)
        prob.linearize(cams, lms)
        dxp, dxl, _ = prob.power_solve(1e-3, 16, 0.0)
        out.append((np_(dxp).copy(), np_(dxl).copy()))
    tol = 1e-12 if precision == "f64" else 1e-5
    assert rel(out[1][0], out[0][0]) <= tol and rel(out[1][1], out[0][1]) <= tol


@pytest.mark.parametrize("precision,records", [("f64", "jacobian"), ("f32", "jacobian"), ("f64", "point"),
                                               ("f32", "point")])
def test_many_cameras_switch_to_l2(precision, records):
    """2,048 cameras: the automatic choice is the L2 form for every mode."""
    case = ring_2k()
    assert not _lm_pass_in_lds(case.scene.n_cams, precision, records)
    prob = case.problem(precision, records=records)
    assert prob.get_tuning("lds_camera") == 1  # the default; the size rules it out
    cams, lms = case.state()
    prob.linearize(cams, lms)
    for lam, m in [(1e-4, 20), (1.0, 8)]:
        _check_step(prob, case, lam, m, TOL[precision], f"ring_2k {precision} {records}")


def test_f64_point_compact_fold():
    """1,000 cameras in float64 over point records: the landmark pass and the
    back-substitution stage the compact fold and rebuild R per observation;
    against the oracle, and against the L2 form (lds_camera = 0), which
    differs only in summation order."""
    case = ring_1k()
    n = case.scene.n_cams
    assert n * 26 * 8 > 160 * 1024 and _lm_pass_in_lds(n, "f64", "point")
    cams, lms = case.state()
    out = []
    for lds in [1, 0]:
        prob = case.problem("f64", records="point")
        prob.set_tuning("lds_camera", lds)
        prob.linearize(cams, lms)
        for lam, m in [(1e-4, 20), (1.0, 8)]:
            _check_step(prob, case, lam, m, TOL["f64"], f"ring_1k f64 point lds_camera={lds}")
        dxp, dxl, _ = prob.power_solve(1e-3, 16, 0.0)
        out.append((np_(dxp).copy(), np_(dxl).copy()))
    assert rel(out[1][0], out[0][0]) <= 1e-12 and rel(out[1][1], out[0][1]) <= 1e-12


@pytest.mark.parametrize("tpw", [1, 8])
def test_many_cameras_ragged_piece_ranges(tpw):
    """2,048 cameras with split camera pieces and landmark ranges, through
    the L2 landmark pass at two wavefront loads."""
    case = ring_2k()
    for precision, records in [("f64", "jacobian"), ("f32", "point")]:
        prob = case.problem(precision, piece_size=64, lm_ranges=8, records=records)
        prob.set_tuning("tiles_per_wave", tpw)
        cams, lms = case.state()
        prob.linearize(cams, lms)
        _check_step(prob, case, 1e-2, 12, TOL[precision], f"ring_2k ragged tpw={tpw} {precision} {records}")


@functools.lru_cache(maxsize=None)
def big_batch():
    # 12 problems of 150..200 cameras: 2,100 cameras in all, so the batch's
    # camera vector (76 KB in float32) leaves LDS for L2
    rng = np.random.default_rng(21)
    sizes = [(int(nc), int(nl)) for nc, nl in zip(rng.integers(150, 201, 12), rng.integers(300, 2500, 12))]
    sizes[0] = (200, 2500)
    scenes = [synth.ring_scene(nc, nl, (2, 8), seed=300 + k, name=f"bb{k}") for k, (nc, nl) in enumerate(sizes)]
    cat, co, lo = synth.concat_scenes(scenes)
    obs = [observations(s) for s in scenes]
    return scenes, cat, co, lo, np.concatenate(obs)


@pytest.mark.parametrize("precision,records", [("f64", "jacobian"), ("f32", "jacobian"), ("f32", "point")])
def test_batch_over_1820_cameras(precision, records):
    from paper_2204_12834_amd.solver import Problem
    scenes, cat, co, lo, obs = big_batch()
    assert cat.n_cams > 1820 and not _lm_pass_in_lds(cat.n_cams, precision, records)
    prob = Problem(cat.obs_cam, cat.obs_lm, obs, cat.n_cams, cat.n_lms, precision=precision, device="cuda",
                   prob_cam_off=co, prob_lm_off=lo, records=records)
    cams = torch.tensor(cat.cams0, device="cuda")
    lms = torch.tensor(cat.lms0, device="cuda")
    cost = np_(prob.linearize(cams, lms))
    lam, m = 1e-3, 16
    dxp, dxl, _ = prob.power_solve(lam, m, 0.0)
    dxp, dxl = np_(dxp), np_(dxl)
    tol = TOL[precision]
    start = 0
    for k, s in enumerate(scenes):
        o = obs[start:start + s.n_obs]
        start += s.n_obs
        F, r, Jp, Jl = lm.linearize(s.cams0, s.lms0, s.obs_cam, s.obs_lm, o)
        assert abs(cost[k] - F) <= 1e-12 * F, k
        ref = schur.solve(Jp, Jl, r, s.obs_cam, s.obs_lm, s.n_cams, s.n_lms, lam, m)
        ep, el = rel(dxp[co[k]:co[k + 1]], ref.dxp), rel(dxl[lo[k]:lo[k + 1]], ref.dxl)
        log(f"big batch {precision} {records} problem {k}: dx_p {ep:.2e} dx_l {el:.2e}")
        assert ep <= tol and el <= tol, (k, ep, el)


@functools.lru_cache(maxsize=None)
def city_full():
    # the full city workload: 1,100 cameras, 780,000 landmarks, 4.94M
    # observations, Huber delta 3 px; the oracle's solve at m = 3 takes about
    # a minute on one core
    log("building the city workload and its oracle linearisation")
    return Case(synth.config("c3"), delta=3.0)


@functools.lru_cache(maxsize=None)
def city_full_ref(lam, m):
    return city_full().solve(lam, m)


@pytest.mark.slow
@pytest.mark.timeout(1200)
@pytest.mark.parametrize("precision,records", [("f64", "jacobian"), ("f32", "jacobian"), ("f64", "point"),
                                               ("f32", "point")])
def test_city_full_size(precision, records):
    """The city workload at full size, automatic pieces, ranges and pass
    forms (float64 stored blocks: the L2 landmark pass; float64 point records:
    the compact fold in LDS; float32: the LDS pass), against the oracle at
    m = 3, eps = 0."""
    case = city_full()
    s = case.scene
    prob = case.problem(precision, records=records)
    cams, lms = case.state()
    cost = prob.linearize(cams, lms).item()
    assert abs(cost - case.F) <= 1e-12 * case.F
    lam, m = 1e-2, 3
    dxp, dxl, info = prob.power_solve(lam, m, 0.0)
    ref = city_full_ref(lam, m)
    ep, el = rel(np_(dxp), ref.dxp), rel(np_(dxl), ref.dxl)
    log(f"city full {precision} {records} (lm pass in LDS: {_lm_pass_in_lds(s.n_cams, precision, records)}, "
        f"ranges {prob.get_tuning('lm_ranges')}): dx_p {ep:.2e} dx_l {el:.2e}")
    assert ep <= TOL[precision] and el <= TOL[precision], (ep, el)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_autotuned_handle_matches_oracle(tmp_path, precision):
    """The autotuner's handle (whatever shape it picks, and again from its
    cache) gives the oracle's step."""
    from paper_2204_12834_amd import autotune
    case = city_small()
    s = case.scene
    cams, lms = case.state()
    cache = str(tmp_path / "tune.json")
    for _ in range(2):
        cfg, prob = autotune.tune(lambda ps: case.problem(precision, piece_size=ps), precision, s.n_obs, s.n_lms,
                                  cams, lms, piece_sizes=(256, 1024), tiles=(1, 8), cache=cache)
        log(f"tuned {precision}: {cfg.get('piece_size')}/{cfg.get('tiles_per_wave')}/{cfg.get('lds_camera')} "
            f"cached={cfg['cached']}")
        _check_step(prob, case, 1e-2, 16, TOL[precision], f"autotuned {precision}")
