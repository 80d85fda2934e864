"""The adjoint of the damped step on the GPU (poba_step_adjoint, and the
torch.autograd.Function over it) against the oracle's implicit-differentiation
reference and against central differences of the GPU forward.

Tolerances: float64 against the oracle <= 1e-9 relative (same truncated
operator) and <= 1e-8 against the dense exact inverse at lambda = 1;
float32 <= 1e-3 relative per coordinate with a floor of 1e-6 |gbar|_inf
times the gradient scale."""
import functools

import numpy as np
import pytest

from paper_2204_12834_amd import synth
from gpu_common import log, np_, observations, rel
from oracle import adjoint

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

LAM = 1.0
M = 32


@functools.lru_cache(maxsize=None)
def c1_adjoint():
    s = synth.config("c1")
    obs = observations(s)
    rng = np.random.default_rng(1)
    gp, gl = rng.normal(size=(s.n_cams, 9)), rng.normal(size=(s.n_lms, 3))
    D = adjoint.damping_diagonals(s.cams0, s.lms0, s.obs_cam, s.obs_lm, obs)
    dense = adjoint.adjoint(s.cams0, s.lms0, s.obs_cam, s.obs_lm, obs, LAM, gp, gl, m=None, diagonals=D)
    series = adjoint.adjoint(s.cams0, s.lms0, s.obs_cam, s.obs_lm, obs, LAM, gp, gl, m=M, diagonals=D)
    return s, obs, gp, gl, dense, series


def _gpu_adjoint(s, obs, gp, gl, precision, lam=LAM, m=M, records="jacobian"):
    from paper_2204_12834_amd.solver import Problem
    prob = Problem(s.obs_cam, s.obs_lm, obs, s.n_cams, s.n_lms, precision=precision, device="cuda",
                   records=records)
    cams = torch.tensor(s.cams0, dtype=torch.float64, device="cuda")
    lms = torch.tensor(s.lms0, dtype=torch.float64, device="cuda")
    prob.linearize(cams, lms)
    dxc, dxl, _ = prob.power_solve(lam, m, 0.0)
    go, gi, zc, zl = prob.step_adjoint(lam, m, cams, lms, dxc, dxl, torch.tensor(gp, device="cuda"),
                                       torch.tensor(gl, device="cuda"))
    return prob, dxc, dxl, go, gi, zc, zl


@pytest.mark.parametrize("records", ["jacobian", "point"])
def test_adjoint_f64_matches_oracle(records):
    s, obs, gp, gl, dense, series = c1_adjoint()
    log(f"adjoint f64 c1 {records}")
    _, dxc, dxl, go, gi, zc, zl = _gpu_adjoint(s, obs, gp, gl, "f64", records=records)
    assert rel(np_(dxc), series.dxp) <= 1e-10 and rel(np_(dxl), series.dxl) <= 1e-10
    assert rel(np_(zc), series.zp) <= 1e-10 and rel(np_(zl), series.zl) <= 1e-10
    assert rel(np_(go), series.grad_obs) <= 1e-9
    assert rel(np_(gi), series.grad_intr) <= 1e-9
    # the dense implicit reference (exact inverse): truncation at lambda = 1 is far below 1e-8
    assert rel(np_(go), dense.grad_obs) <= 1e-8
    assert rel(np_(gi), dense.grad_intr) <= 1e-8


@pytest.mark.parametrize("precision,records", [("f32", "jacobian"), ("bf16", "jacobian"), ("f32", "point")])
def test_adjoint_reduced_precision(precision, records):
    s, obs, gp, gl, dense, series = c1_adjoint()
    _, _, _, go, gi, _, _ = _gpu_adjoint(s, obs, gp, gl, precision, records=records)
    eo = rel(np_(go), dense.grad_obs)
    ei = rel(np_(gi), dense.grad_intr)
    log(f"adjoint {precision}: obs {eo:.2e} intrinsics {ei:.2e}")
    if precision == "f32":
        floor = 1e-6 * max(np.abs(gp).max(), np.abs(gl).max())
        for got, ref in [(np_(go), dense.grad_obs), (np_(gi), dense.grad_intr)]:
            err = np.abs(got - ref)
            assert np.all(err <= 1e-3 * np.abs(ref) + floor * np.abs(ref).max()), err.max()
    else:  # bfloat16 Jacobian storage is an experiment: loose bound only
        assert eo <= 0.1 and ei <= 0.1


def test_adjoint_rejects_huber():
    from paper_2204_12834_amd._lib import PobaError
    from paper_2204_12834_amd.solver import Problem
    s = synth.ring_scene(4, 50, (2, 3), seed=1, name="huber_adj")
    obs = observations(s)
    prob = Problem(s.obs_cam, s.obs_lm, obs, s.n_cams, s.n_lms, loss="huber", huber_delta=3.0, device="cuda")
    cams = torch.tensor(s.cams0, device="cuda")
    lms = torch.tensor(s.lms0, device="cuda")
    prob.linearize(cams, lms)
    dxc, dxl, _ = prob.power_solve(1.0, 4)
    with pytest.raises(PobaError):
        prob.step_adjoint(1.0, 4, cams, lms, dxc, dxl, torch.zeros_like(dxc), torch.zeros_like(dxl))


def test_frozen_damping_and_new_observations():
    """With the damping frozen, a solve at another state and other
    observations equals the oracle step with the first state's D."""
    s, obs, gp, gl, dense, series = c1_adjoint()
    from paper_2204_12834_amd.solver import Problem
    prob = Problem(s.obs_cam, s.obs_lm, obs, s.n_cams, s.n_lms, precision="f64", device="cuda")
    cams = torch.tensor(s.cams0, device="cuda")
    lms = torch.tensor(s.lms0, device="cuda")
    prob.linearize(cams, lms)
    prob.power_solve(LAM, 2)  # records D at the first state
    prob.freeze_damping(True)
    D = adjoint.damping_diagonals(s.cams0, s.lms0, s.obs_cam, s.obs_lm, obs)
    cams2 = s.cams0.copy()
    cams2[:, 6] *= 1.01
    obs2 = obs + np.random.default_rng(9).normal(size=obs.shape)
    prob.set_observations(torch.tensor(obs2, device="cuda"))
    prob.linearize(torch.tensor(cams2, device="cuda"), lms)
    dxc, dxl, _ = prob.power_solve(LAM, M)
    rp, rl = adjoint.step(cams2, s.lms0, s.obs_cam, s.obs_lm, obs2, LAM, m=M, diagonals=D)
    assert rel(np_(dxc), rp) <= 1e-10 and rel(np_(dxl), rl) <= 1e-10
    prob.freeze_damping(False)
    prob.power_solve(LAM, M)
    rp2, rl2 = adjoint.step(cams2, s.lms0, s.obs_cam, s.obs_lm, obs2, LAM, m=M)
    dxc2, dxl2, _ = prob.power_solve(LAM, M)
    assert rel(np_(dxc2), rp2) <= 1e-10 and rel(np_(dxl2), rl2) <= 1e-10


@functools.lru_cache(maxsize=None)
def c5_case():
    s = synth.config("c5")
    obs = observations(s)
    rng = np.random.default_rng(1)
    gp, gl = rng.normal(size=(s.n_cams, 9)), rng.normal(size=(s.n_lms, 3))
    return s, obs, gp, gl


def test_adjoint_c5_against_central_differences():
    """200 cameras, 50,000 landmarks: the float32 adjoint on 25 observation
    and 25 intrinsic coordinates (seed 2) against central differences
    (h = 1e-3) of <gbar, dx> with the float64 GPU step at frozen damping."""
    from paper_2204_12834_amd.solver import Problem
    s, obs, gp, gl = c5_case()
    log(f"c5: {s.n_cams} cams, {s.n_lms} lms, {s.n_obs} obs")
    _, _, _, go32, gi32, _, _ = _gpu_adjoint(s, obs, gp, gl, "f32")
    _, _, _, go64, gi64, _, _ = _gpu_adjoint(s, obs, gp, gl, "f64")
    go32, gi32, go64, gi64 = np_(go32), np_(gi32), np_(go64), np_(gi64)
    fwd = Problem(s.obs_cam, s.obs_lm, obs, s.n_cams, s.n_lms, precision="f64", device="cuda")
    lms = torch.tensor(s.lms0, device="cuda")
    gpt, glt = torch.tensor(gp, device="cuda"), torch.tensor(gl, device="cuda")

    def L(cams_np, obs_np):
        fwd.set_observations(torch.tensor(obs_np, device="cuda"))
        fwd.linearize(torch.tensor(cams_np, device="cuda"), lms)
        dxc, dxl, _ = fwd.power_solve(LAM, M)
        return float((dxc * gpt).sum() + (dxl * glt).sum())

    L(s.cams0, obs)  # D at the base state
    fwd.freeze_damping(True)
    rng = np.random.default_rng(2)
    h = 1e-3
    gscale = max(np.abs(gp).max(), np.abs(gl).max())
    checks = []
    for i in rng.choice(s.n_obs, 25, replace=False):
        k = int(rng.integers(2))
        op, om = obs.copy(), obs.copy()
        op[i, k] += h
        om[i, k] -= h
        checks.append(("obs", (int(i), k), (L(s.cams0, op) - L(s.cams0, om)) / (2 * h), go32[i, k], go64[i, k]))
    for _ in range(25):
        c, col = int(rng.integers(s.n_cams)), int(rng.integers(3))
        k = 6 + col
        cp, cm = s.cams0.copy(), s.cams0.copy()
        cp[c, k] += h
        cm[c, k] -= h
        checks.append(("intr", (c, k), (L(cp, obs) - L(cm, obs)) / (2 * h), gi32[c, col], gi64[c, col]))
    scale_o, scale_i = np.abs(go64).max(), np.abs(gi64).max()
    for kind, idx, fd, g32, g64 in checks:
        scale = scale_o if kind == "obs" else scale_i
        floor = 1e-6 * gscale * scale
        assert abs(g32 - fd) <= 1e-3 * abs(fd) + floor, (kind, idx, fd, g32)
        assert abs(g64 - fd) <= 1e-4 * abs(fd) + floor, (kind, idx, fd, g64)


@functools.lru_cache(maxsize=None)
def c5_series_reference():
    s, obs, gp, gl = c5_case()
    return adjoint.adjoint(s.cams0, s.lms0, s.obs_cam, s.obs_lm, obs, LAM, gp, gl, m=M)


@pytest.mark.slow
@pytest.mark.timeout(900)
@pytest.mark.parametrize("records", ["jacobian", "point"])
def test_adjoint_c5_matches_oracle_series_adjoint(records):
    """200 cameras, 50,000 landmarks: the GPU adjoint against the oracle's
    matrix-free one (the same truncated operator, m = 32, lambda = 1, D at
    the state), float64 <= 1e-9 relative, float32 per coordinate <= 1e-3
    with the floor of 1e-6 |gbar|_inf times the gradient scale."""
    s, obs, gp, gl = c5_case()
    ref = c5_series_reference()
    _, dxc, dxl, go, gi, zc, zl = _gpu_adjoint(s, obs, gp, gl, "f64", records=records)
    e = [rel(np_(dxc), ref.dxp), rel(np_(dxl), ref.dxl), rel(np_(zc), ref.zp), rel(np_(zl), ref.zl),
         rel(np_(go), ref.grad_obs), rel(np_(gi), ref.grad_intr)]
    log(f"c5 adjoint f64 {records}: dx {e[0]:.1e}/{e[1]:.1e} z {e[2]:.1e}/{e[3]:.1e} "
        f"grad obs {e[4]:.1e} intrinsics {e[5]:.1e}")
    assert max(e[:4]) <= 1e-10 and e[4] <= 1e-9 and e[5] <= 1e-9
    _, _, _, go32, gi32, _, _ = _gpu_adjoint(s, obs, gp, gl, "f32", records=records)
    floor = 1e-6 * max(np.abs(gp).max(), np.abs(gl).max())
    for what, got, want in [("obs", np_(go32), ref.grad_obs), ("intrinsics", np_(gi32), ref.grad_intr)]:
        err = np.abs(got - want)
        bound = 1e-3 * np.abs(want) + floor * np.abs(want).max()
        log(f"c5 adjoint f32 {records} {what}: rel {rel(got, want):.2e}, worst err/bound {np.max(err / bound):.2f}")
        assert np.all(err <= bound), what


def test_autograd_function():
    from paper_2204_12834_amd.autograd import damped_step
    from paper_2204_12834_amd.solver import Problem
    s, obs, gp, gl, dense, series = c1_adjoint()
    prob = Problem(s.obs_cam, s.obs_lm, obs, s.n_cams, s.n_lms, precision="f64", device="cuda")
    o = torch.tensor(obs, device="cuda", requires_grad=True)
    intr = torch.tensor(s.cams0[:, 6:9].copy(), device="cuda", requires_grad=True)
    extr = torch.tensor(s.cams0[:, :6].copy(), device="cuda")
    lms = torch.tensor(s.lms0, device="cuda")
    dxc, dxl = damped_step(prob, o, intr, extr, lms, LAM, M)
    assert rel(np_(dxc), series.dxp) <= 1e-10
    loss = (dxc * torch.tensor(gp, device="cuda")).sum() + (dxl * torch.tensor(gl, device="cuda")).sum()
    g_o, g_i = torch.autograd.grad(loss, [o, intr])
    assert rel(np_(g_o), series.grad_obs) <= 1e-9
    assert rel(np_(g_i), series.grad_intr) <= 1e-9
    with pytest.raises(ValueError):
        damped_step(prob, o, intr, extr.requires_grad_(True), lms, LAM, M)
