"""The range-staged camera pass over point records (landmark vector slices in
LDS, per (camera, landmark range) group sums) against the oracle and against
the per-piece pass that gathers from L2.

Tolerances as the other parity tests: float64 <= 1e-10 relative to the
oracle, float32 <= 1e-4; the two passes differ only in summation order
(float64 <= 1e-12 relative to each other)."""
import functools

import numpy as np
import pytest

from paper_2204_12834_amd import synth
from gpu_common import Case, log, np_, rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=None)
def ladybug_small():
    return Case(synth.ladybug_scene(n_cams=120, n_lms=4000, seed=2, name="ladybug_small"))


@functools.lru_cache(maxsize=None)
def city_small():
    return Case(synth.city_scene(n_cams=60, n_lms=3000, seed=5, name="city_small"), delta=3.0)


@functools.lru_cache(maxsize=None)
def many_cameras():
    # 600 cameras over about 3,000 observations: eight wavefronts per range,
    # each walking more than one window of 64 cameras, many groups empty
    return Case(synth.ring_scene(600, 1000, (2, 4), seed=4, name="many_cameras"))


@functools.lru_cache(maxsize=None)
def wide():
    # 8,000 landmarks: 192 KB of float64 landmark vector, more than one slice
    return Case(synth.ring_scene(16, 8000, (2, 4), seed=6, name="wide"))


CASES = {"ladybug_small": ladybug_small, "city_small": city_small, "many_cameras": many_cameras, "wide": wide}


def _solve(prob, cams, lms, lam, m):
    prob.linearize(cams, lms)
    dxp, dxl, _ = prob.power_solve(lam, m, 0.0)
    return np_(dxp).copy(), np_(dxl).copy()


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision,tol", [("f64", 1e-10), ("f32", 1e-4)])
@pytest.mark.parametrize("ranges", [0, 8, 16])
def test_range_pass_matches_oracle_and_piece_pass(name, precision, tol, ranges):
    case = CASES[name]()
    log(f"range pass {name} {precision} ranges={ranges}")
    prob = case.problem(precision, lm_ranges=ranges, records="point")
    assert prob.get_tuning("range_lds") == 1
    R = prob.get_tuning("lm_ranges")
    assert R == ranges or ranges == 0
    cams, lms = case.state()
    for lam in [1e-2, 1.0]:
        ref = case.solve(lam, 20)
        prob.set_tuning("range_lds", 1)
        a = _solve(prob, cams, lms, lam, 20)
        prob.set_tuning("range_lds", 0)
        b = _solve(prob, cams, lms, lam, 20)
        for got in (a, b):
            assert rel(got[0], ref.dxp) <= tol and rel(got[1], ref.dxl) <= tol
        if precision == "f64":
            assert rel(a[0], b[0]) <= 1e-12 and rel(a[1], b[1]) <= 1e-12


def test_automatic_ranges_fit_lds():
    """Automatic ranges for point records keep each slice within the LDS
    target of 144 KB: one range for 8,000 float32 landmarks (96 KB), eight for
    float64 (192 KB)."""
    case = wide()
    assert case.problem("f32", records="point").get_tuning("lm_ranges") == 1
    assert case.problem("f64", records="point").get_tuning("lm_ranges") == 8
    # Jacobian records keep their own rule and never use the range pass
    pj = case.problem("f32")
    assert pj.get_tuning("range_lds") == 0


def test_ranges_too_large_fall_back():
    """A single range of 8,000 float64 landmarks (192 KB) exceeds the LDS
    bound: the handle uses the per-piece pass, refuses to switch, and still
    solves."""
    from paper_2204_12834_amd._lib import PobaError
    case = wide()
    prob = case.problem("f64", lm_ranges=1, records="point")
    assert prob.get_tuning("range_lds") == 0
    with pytest.raises(PobaError):
        prob.set_tuning("range_lds", 1)
    cams, lms = case.state()
    dxp, dxl = _solve(prob, cams, lms, 1e-2, 12)
    ref = case.solve(1e-2, 12)
    assert rel(dxp, ref.dxp) <= 1e-10 and rel(dxl, ref.dxl) <= 1e-10


def test_range_pass_is_deterministic():
    case = city_small()
    prob = case.problem("f32", lm_ranges=8, records="point")
    cams, lms = case.state()
    a = _solve(prob, cams, lms, 1e-3, 16)
    b = _solve(prob, cams, lms, 1e-3, 16)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
