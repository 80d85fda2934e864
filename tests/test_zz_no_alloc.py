"""poba_create_static (the set-up call that allocates nothing: its workspace is
a device array the library holds) against poba_create on the same problems.

Two calls in a row, the second with a smaller problem, so that the second
handle is built over the array the first one left behind.  The observation
orders must be bit-identical to those of poba_create, and cost and step
equal to summation order (float64 <= 1e-12 relative; the kernels and launch
shapes are the same, so in practice they are bit-identical), and both within
the oracle tolerance (1e-10)."""
import ctypes

import numpy as np
import pytest

from paper_2204_12834_amd import synth
from gpu_common import Case, log, np_, rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _pair(case, precision, records):
    from paper_2204_12834_amd.solver import Problem
    s = case.scene
    common = dict(precision=precision, records=records, device="cuda")
    loss = dict(loss="huber", huber_delta=case.delta) if case.delta else {}
    ref = Problem(s.obs_cam, s.obs_lm, case.obs, s.n_cams, s.n_lms, **common, **loss)
    st = Problem(s.obs_cam, s.obs_lm, case.obs, s.n_cams, s.n_lms, **common, **loss, static_workspace=True)
    assert st.workspace is None and st.handle
    return ref, st


def _run(prob, case, lam, m):
    cams, lms = case.state()
    cost = prob.linearize(cams, lms).item()
    dxp, dxl, info = prob.power_solve(lam, m, 0.0)
    orders = [np_(t).copy() for t in prob.get_orders()]
    return cost, np_(dxp).copy(), np_(dxl).copy(), orders


def _check(case, precision, records, lam=1e-2, m=12):
    ref, st = _pair(case, precision, records)
    a = _run(ref, case, lam, m)
    b = _run(st, case, lam, m)
    for x, y in zip(a[3], b[3]):
        np.testing.assert_array_equal(x, y)
    assert abs(a[0] - b[0]) <= 1e-12 * abs(a[0])
    tol = 1e-12 if precision == "f64" else 1e-6
    assert rel(b[1], a[1]) <= tol and rel(b[2], a[2]) <= tol
    o = case.solve(lam, m)
    otol = 1e-10 if precision == "f64" else 1e-4
    ep, el = rel(b[1], o.dxp), rel(b[2], o.dxl)
    log(f"static {case.scene.name} {precision} {records}: vs create {rel(b[1], a[1]):.1e}, "
        f"vs oracle dx_p {ep:.2e} dx_l {el:.2e}")
    assert ep <= otol and el <= otol
    ref.close()
    st.close()


@pytest.mark.parametrize("precision,records", [("f64", "jacobian"), ("f32", "point")])
def test_static_create_matches_create_twice_in_a_row(precision, records):
    big = Case(synth.city_scene(n_cams=60, n_lms=3000, seed=5, name="city_small"), delta=3.0)
    small = Case(synth.ring_scene(8, 300, (2, 5), seed=7, name="ring_small"))
    _check(big, precision, records)
    _check(small, precision, records)


def test_static_create_rejects_a_problem_that_does_not_fit():
    from paper_2204_12834_amd import _lib
    lib = _lib.load()
    # a real (small) problem's device inputs, described as 20M observations:
    # the size check comes before any device work, so nothing reads past them
    oc = torch.zeros(4, dtype=torch.int32, device="cuda")
    xy = torch.zeros(4, 2, dtype=torch.float64, device="cuda")
    d = _lib.PobaDesc(16, 1000, 20_000_000, 1, 0, 0, 0, 0, 0, 0.0)
    h = ctypes.c_void_p()
    rc = lib.poba_create_static(ctypes.byref(d), ctypes.c_void_p(oc.data_ptr()), ctypes.c_void_p(oc.data_ptr()),
                                ctypes.c_void_p(xy.data_ptr()), None, ctypes.byref(h))
    assert rc == _lib.POBA_ERR_WORKSPACE and not h.value
