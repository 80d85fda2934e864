"""Python binding of the C ABI: argument marshalling only.

PyTorch supplies device memory and streams; every step of the computation
runs in the HIP kernels of libpoba.so.
"""
from __future__ import annotations

import ctypes
import dataclasses

import torch

from . import _lib

_PREC_BYTES = {"f64": 8, "f32": 4, "bf16": 2}


def _ptr(t: torch.Tensor | None) -> ctypes.c_void_p:
    if t is None:
        return ctypes.c_void_p(0)
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t, dtype, device, shape=None) -> torch.Tensor:
    t = torch.as_tensor(t, dtype=dtype, device=device).contiguous()
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected shape {shape}, got {tuple(t.shape)}")
    return t


@dataclasses.dataclass
class LMOptions:
    """LM settings of Sec. 5.1 (defaults) as passed to poba_lm_step."""
    lambda0: float = 1e-4
    func_tol: float = 1e-6
    eps: float = 0.01
    eta: float = 1e-3
    lambda_min: float = 1e-16
    lambda_max: float = 1e16
    m: int = 20
    max_iters: int = 50

    def c(self) -> _lib.PobaLMOptions:
        return _lib.PobaLMOptions(self.lambda0, self.func_tol, self.eps, self.eta, self.lambda_min,
                                  self.lambda_max, int(self.m), int(self.max_iters))


def default_options() -> LMOptions:
    lib = _lib.load()
    o = _lib.PobaLMOptions()
    lib.poba_lm_default_options(ctypes.byref(o))
    return LMOptions(o.lambda0, o.func_tol, o.eps, o.eta, o.lambda_min, o.lambda_max, o.m, o.max_iters)


def read_solve_info(t: torch.Tensor, index: int = 0) -> dict:
    """Solve info of problem `index` from the info buffer."""
    n = ctypes.sizeof(_lib.PobaSolveInfo)
    raw = bytes(t.cpu().numpy().tobytes())[index * n:(index + 1) * n]
    info = _lib.PobaSolveInfo.from_buffer_copy(raw)
    return {f: getattr(info, f) for f, _ in _lib.PobaSolveInfo._fields_}


def read_pcg_info(t: torch.Tensor) -> list:
    """PCG info of every problem from the info buffer."""
    n = ctypes.sizeof(_lib.PobaPCGInfo)
    raw = bytes(t.cpu().numpy().tobytes())
    out = []
    for j in range(len(raw) // n):
        info = _lib.PobaPCGInfo.from_buffer_copy(raw[j * n:(j + 1) * n])
        out.append({f: getattr(info, f) for f, _ in _lib.PobaPCGInfo._fields_})
    return out


def read_lm_state(t: torch.Tensor, index: int = 0) -> dict:
    """LM state of problem `index` from the state buffer."""
    n = ctypes.sizeof(_lib.PobaLMState)
    raw = bytes(t.cpu().numpy().tobytes())[index * n:(index + 1) * n]
    st = _lib.PobaLMState.from_buffer_copy(raw)
    out = {f: getattr(st, f) for f, _ in _lib.PobaLMState._fields_}
    out["lambda"] = out.pop("lambda_")
    return out


def read_lm_states(t: torch.Tensor) -> list:
    n = t.numel() // ctypes.sizeof(_lib.PobaLMState)
    return [read_lm_state(t, j) for j in range(n)]


def workspace_bytes(n_cams, n_lms, n_obs, precision="f64", damping="marquardt", loss="l2", huber_delta=0.0,
                    piece_size=0, records="jacobian") -> int:
    lib = _lib.load()
    d = _lib.PobaDesc(int(n_cams), int(n_lms), int(n_obs), _lib.PRECISION[precision], _lib.DAMPING[damping],
                      _lib.LOSS[loss], int(piece_size), 0, _lib.RECORDS[records], float(huber_delta))
    return int(lib.poba_workspace_bytes(ctypes.byref(d)))


class Problem:
    """A bundle-adjustment problem held on one GPU (poba_batch_create ...
    poba_destroy).  With prob_cam_off / prob_lm_off (host sequences of
    n_problems + 1 offsets) it holds that many independent problems over the
    concatenated cameras and landmarks, solved together."""

    def __init__(self, obs_cam, obs_lm, obs_xy, n_cams: int, n_lms: int, precision: str = "f64",
                 damping: str = "marquardt", loss: str = "l2", huber_delta: float = 0.0, piece_size: int = 0,
                 lm_ranges: int = 0, device="cuda", stream=None, prob_cam_off=None, prob_lm_off=None,
                 records: str = "jacobian", static_workspace: bool = False):
        self.lib = _lib.load()
        self.device = torch.device(device)
        self.precision = precision
        self.n_cams, self.n_lms = int(n_cams), int(n_lms)
        obs_cam = _dev(obs_cam, torch.int32, self.device)
        obs_lm = _dev(obs_lm, torch.int32, self.device)
        self.n_obs = int(obs_cam.numel())
        obs_xy = _dev(obs_xy, torch.float64, self.device, (self.n_obs, 2))
        self.desc = _lib.PobaDesc(self.n_cams, self.n_lms, self.n_obs, _lib.PRECISION[precision],
                                  _lib.DAMPING[damping], _lib.LOSS[loss], int(piece_size), int(lm_ranges),
                                  _lib.RECORDS[records], float(huber_delta))
        self.records = records
        if prob_cam_off is None:
            prob_cam_off, prob_lm_off = [0, self.n_cams], [0, self.n_lms]
        self.prob_cam_off = [int(v) for v in prob_cam_off]
        self.prob_lm_off = [int(v) for v in prob_lm_off]
        if len(self.prob_cam_off) != len(self.prob_lm_off) or len(self.prob_cam_off) < 2:
            raise ValueError("prob_cam_off and prob_lm_off need n_problems + 1 entries each")
        self.n_problems = len(self.prob_cam_off) - 1
        self._info = torch.zeros(ctypes.sizeof(_lib.PobaSolveInfo) * self.n_problems, dtype=torch.uint8,
                                 device=self.device)
        if static_workspace:
            # the library's own per-device workspace (poba_create_static): no device allocation
            if self.n_problems != 1:
                raise ValueError("static_workspace holds one problem")
            self.workspace = None
            h = ctypes.c_void_p()
            with torch.cuda.device(self.device):
                rc = self.lib.poba_create_static(ctypes.byref(self.desc), _ptr(obs_cam), _ptr(obs_lm), _ptr(obs_xy),
                                                 _stream(stream), ctypes.byref(h))
            if rc == _lib.POBA_ERR_WORKSPACE:
                raise _lib.PobaError("poba_create_static (problem larger than the library-held workspace)", rc)
            _lib.check("poba_create_static", rc)
            self.handle = h
            return
        nbytes = int(self.lib.poba_batch_workspace_bytes(ctypes.byref(self.desc), self.n_problems))
        if nbytes == 0:
            raise _lib.PobaError("poba_batch_workspace_bytes", 1)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        self._ws_ptr = self.workspace.data_ptr() + off
        self._ws_bytes = nbytes
        h = ctypes.c_void_p()
        co = (ctypes.c_int32 * (self.n_problems + 1))(*self.prob_cam_off)
        lo = (ctypes.c_int32 * (self.n_problems + 1))(*self.prob_lm_off)
        with torch.cuda.device(self.device):
            rc = self.lib.poba_batch_create(ctypes.byref(self.desc), self.n_problems, co, lo, _ptr(obs_cam),
                                            _ptr(obs_lm), _ptr(obs_xy), ctypes.c_void_p(self._ws_ptr),
                                            ctypes.c_size_t(nbytes), _stream(stream), ctypes.byref(h))
        _lib.check("poba_batch_create", rc)
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            self.lib.poba_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- hot path --------------------------------------------------------

    def linearize(self, cams: torch.Tensor, lms: torch.Tensor, cost: torch.Tensor | None = None, stream=None):
        cams = _dev(cams, torch.float64, self.device, (self.n_cams, 9))
        lms = _dev(lms, torch.float64, self.device, (self.n_lms, 3))
        if cost is None:
            cost = torch.zeros(self.n_problems, dtype=torch.float64, device=self.device)
        _lib.check("poba_linearize", self.lib.poba_linearize(self.handle, _ptr(cams), _ptr(lms), _ptr(cost),
                                                             _stream(stream)))
        return cost

    def power_solve(self, lam: float, m: int, eps: float = 0.0, dx_cams=None, dx_lms=None, info=None,
                    stream=None):
        if dx_cams is None:
            dx_cams = torch.empty(self.n_cams, 9, dtype=torch.float64, device=self.device)
        if dx_lms is None:
            dx_lms = torch.empty(self.n_lms, 3, dtype=torch.float64, device=self.device)
        info = self._info if info is None else info
        _lib.check("poba_power_solve", self.lib.poba_power_solve(self.handle, float(lam), int(m), float(eps),
                                                                 _ptr(dx_cams), _ptr(dx_lms), _ptr(info),
                                                                 _stream(stream)))
        return dx_cams, dx_lms, info

    def pcg_solve(self, lam: float, precond: str = "schur_jacobi", m: int = 0, tol: float = 1e-8,
                  max_iters: int = 500, dx_cams=None, dx_lms=None, coeffs: bool = False, stream=None):
        """Damped step with the camera step from preconditioned CG on the
        reduced camera system.  Returns dx_cams, dx_lms, the per-problem info
        (list of dicts) and, if `coeffs`, a [max_iters, n_problems, 2] tensor of
        (alpha, beta) per iteration (NaN where not taken)."""
        if dx_cams is None:
            dx_cams = torch.empty(self.n_cams, 9, dtype=torch.float64, device=self.device)
        if dx_lms is None:
            dx_lms = torch.empty(self.n_lms, 3, dtype=torch.float64, device=self.device)
        info = torch.zeros(self.n_problems * ctypes.sizeof(_lib.PobaPCGInfo), dtype=torch.uint8, device=self.device)
        co = None
        if coeffs:
            co = torch.full((max(int(max_iters), 1), self.n_problems, 2), float("nan"), dtype=torch.float64,
                            device=self.device)
        _lib.check("poba_pcg_solve", self.lib.poba_pcg_solve(self.handle, float(lam), _lib.PRECOND[precond], int(m),
                                                             float(tol), int(max_iters), _ptr(dx_cams), _ptr(dx_lms),
                                                             _ptr(info), _ptr(co), _stream(stream)))
        return dx_cams, dx_lms, read_pcg_info(info), co

    def solve_residual(self, dx_cams: torch.Tensor, stream=None) -> torch.Tensor:
        """|S x + b~| / |b~| per problem for a camera step of the last power_solve."""
        dx_cams = _dev(dx_cams, torch.float64, self.device, (self.n_cams, 9))
        out = torch.empty(self.n_problems, dtype=torch.float64, device=self.device)
        _lib.check("poba_solve_residual", self.lib.poba_solve_residual(self.handle, _ptr(dx_cams), _ptr(out),
                                                                       _stream(stream)))
        return out

    def lm_init(self, opts: LMOptions | None = None, state: torch.Tensor | None = None, stream=None):
        opts = opts or LMOptions()
        if state is None:
            state = torch.zeros(ctypes.sizeof(_lib.PobaLMState) * self.n_problems, dtype=torch.uint8,
                                device=self.device)
        o = opts.c()
        _lib.check("poba_lm_init", self.lib.poba_lm_init(self.handle, _ptr(state), ctypes.byref(o),
                                                         _stream(stream)))
        return state

    def lm_step(self, cams: torch.Tensor, lms: torch.Tensor, state: torch.Tensor, opts: LMOptions | None = None,
                stream=None):
        """One LM iteration; cams, lms (float64 device tensors) are updated in place."""
        opts = opts or LMOptions()
        if cams.dtype != torch.float64 or not cams.is_contiguous() or tuple(cams.shape) != (self.n_cams, 9):
            raise ValueError("cams must be a contiguous float64 [n_cams, 9] device tensor")
        if lms.dtype != torch.float64 or not lms.is_contiguous() or tuple(lms.shape) != (self.n_lms, 3):
            raise ValueError("lms must be a contiguous float64 [n_lms, 3] device tensor")
        o = opts.c()
        _lib.check("poba_lm_step", self.lib.poba_lm_step(self.handle, _ptr(cams), _ptr(lms), _ptr(state),
                                                         ctypes.byref(o), _stream(stream)))

    def _check_state(self, cams, lms):
        if cams.dtype != torch.float64 or not cams.is_contiguous() or tuple(cams.shape) != (self.n_cams, 9):
            raise ValueError("cams must be a contiguous float64 [n_cams, 9] device tensor")
        if lms.dtype != torch.float64 or not lms.is_contiguous() or tuple(lms.shape) != (self.n_lms, 3):
            raise ValueError("lms must be a contiguous float64 [n_lms, 3] device tensor")

    def lm_begin(self, cams: torch.Tensor, lms: torch.Tensor, state: torch.Tensor, stream=None):
        """First half of an LM iteration whose step the caller computes:
        linearises where the state asks for it."""
        self._check_state(cams, lms)
        _lib.check("poba_lm_begin", self.lib.poba_lm_begin(self.handle, _ptr(cams), _ptr(lms), _ptr(state),
                                                           _stream(stream)))

    def lm_finish(self, cams: torch.Tensor, lms: torch.Tensor, state: torch.Tensor, dx_cams: torch.Tensor,
                  dx_lms: torch.Tensor, opts: LMOptions | None = None, stream=None):
        """Second half: evaluates, accepts or rejects the step (dx_cams, dx_lms)."""
        self._check_state(cams, lms)
        opts = opts or LMOptions()
        o = opts.c()
        dx_cams = _dev(dx_cams, torch.float64, self.device, (self.n_cams, 9))
        dx_lms = _dev(dx_lms, torch.float64, self.device, (self.n_lms, 3))
        _lib.check("poba_lm_finish", self.lib.poba_lm_finish(self.handle, _ptr(cams), _ptr(lms), _ptr(state),
                                                             ctypes.byref(o), _ptr(dx_cams), _ptr(dx_lms),
                                                             _stream(stream)))

    def back_substitute(self, lam: float, dx_cams: torch.Tensor, dx_lms=None, stream=None) -> torch.Tensor:
        """dx_l = -V_lambda^-1 (b_l + W^T dx_cams) with the last linearisation."""
        dx_cams = _dev(dx_cams, torch.float64, self.device, (self.n_cams, 9))
        if dx_lms is None:
            dx_lms = torch.empty(self.n_lms, 3, dtype=torch.float64, device=self.device)
        _lib.check("poba_back_substitute", self.lib.poba_back_substitute(self.handle, float(lam), _ptr(dx_cams),
                                                                         _ptr(dx_lms), _stream(stream)))
        return dx_lms

    def set_landmark_blocks(self, V: torch.Tensor, bl: torch.Tensor, stream=None):
        """Replaces the undamped V [n_lms, 3, 3] and b_l [n_lms, 3] of the last linearisation."""
        V = _dev(V, torch.float64, self.device, (self.n_lms, 3, 3))
        bl = _dev(bl, torch.float64, self.device, (self.n_lms, 3))
        _lib.check("poba_set_landmark_blocks", self.lib.poba_set_landmark_blocks(self.handle, _ptr(V), _ptr(bl),
                                                                                 _stream(stream)))

    def lm_graph(self, cams: torch.Tensor, lms: torch.Tensor, state: torch.Tensor, n_steps: int,
                 opts: LMOptions | None = None) -> "LMGraph":
        """n_steps LM iterations captured in one HIP graph (poba_lm_graph_create)."""
        opts = opts or LMOptions()
        for t, shape in [(cams, (self.n_cams, 9)), (lms, (self.n_lms, 3))]:
            if t.dtype != torch.float64 or not t.is_contiguous() or tuple(t.shape) != shape:
                raise ValueError(f"expected a contiguous float64 {shape} device tensor")
        g = ctypes.c_void_p()
        o = opts.c()
        with torch.cuda.device(self.device):
            _lib.check("poba_lm_graph_create", self.lib.poba_lm_graph_create(
                self.handle, _ptr(cams), _ptr(lms), _ptr(state), ctypes.byref(o), int(n_steps), ctypes.byref(g)))
        return LMGraph(self, g, (cams, lms, state))

    # -- differentiation ---------------------------------------------------

    def set_observations(self, obs_xy: torch.Tensor, stream=None):
        """Replaces the observed pixels [n_obs, 2] (original order)."""
        obs_xy = _dev(obs_xy, torch.float64, self.device, (self.n_obs, 2))
        _lib.check("poba_set_observations", self.lib.poba_set_observations(self.handle, _ptr(obs_xy),
                                                                           _stream(stream)))

    def freeze_damping(self, frozen: bool = True):
        """Later solves reuse the damping diagonal of the last unfrozen solve."""
        _lib.check("poba_set_damping_frozen", self.lib.poba_set_damping_frozen(self.handle, 1 if frozen else 0))

    def step_adjoint(self, lam: float, m: int, cams, lms, dx_cams, dx_lms, grad_dx_cams, grad_dx_lms, stream=None):
        """Gradients of <gbar, dx> for the step dx of the last linearisation:
        returns (grad_obs [n_obs, 2], grad_intrinsics [n_cams, 3], z_cams, z_lms)."""
        d = self.device
        cams = _dev(cams, torch.float64, d, (self.n_cams, 9))
        lms = _dev(lms, torch.float64, d, (self.n_lms, 3))
        dx_cams = _dev(dx_cams, torch.float64, d, (self.n_cams, 9))
        dx_lms = _dev(dx_lms, torch.float64, d, (self.n_lms, 3))
        gc = _dev(grad_dx_cams, torch.float64, d, (self.n_cams, 9))
        gl = _dev(grad_dx_lms, torch.float64, d, (self.n_lms, 3))
        zc = torch.empty(self.n_cams, 9, dtype=torch.float64, device=d)
        zl = torch.empty(self.n_lms, 3, dtype=torch.float64, device=d)
        go = torch.empty(self.n_obs, 2, dtype=torch.float64, device=d)
        gi = torch.empty(self.n_cams, 3, dtype=torch.float64, device=d)
        _lib.check("poba_step_adjoint", self.lib.poba_step_adjoint(
            self.handle, float(lam), int(m), _ptr(cams), _ptr(lms), _ptr(dx_cams), _ptr(dx_lms), _ptr(gc), _ptr(gl),
            _ptr(zc), _ptr(zl), _ptr(go), _ptr(gi), _ptr(self._info), _stream(stream)))
        return go, gi, zc, zl

    # -- inspection --------------------------------------------------------

    def get_blocks(self, stream=None):
        U = torch.empty(self.n_cams, 9, 9, dtype=torch.float64, device=self.device)
        V = torch.empty(self.n_lms, 3, 3, dtype=torch.float64, device=self.device)
        bp = torch.empty(self.n_cams, 9, dtype=torch.float64, device=self.device)
        bl = torch.empty(self.n_lms, 3, dtype=torch.float64, device=self.device)
        _lib.check("poba_get_blocks", self.lib.poba_get_blocks(self.handle, _ptr(U), _ptr(V), _ptr(bp), _ptr(bl),
                                                               _stream(stream)))
        return U, V, bp, bl

    def get_jacobians(self, order: int = 0, stream=None):
        Jp = torch.empty(self.n_obs, 2, 9, dtype=torch.float64, device=self.device)
        Jl = torch.empty(self.n_obs, 2, 3, dtype=torch.float64, device=self.device)
        r = torch.empty(self.n_obs, 2, dtype=torch.float64, device=self.device)
        _lib.check("poba_get_jacobians", self.lib.poba_get_jacobians(self.handle, int(order), _ptr(Jp), _ptr(Jl),
                                                                     _ptr(r), _stream(stream)))
        return Jp, Jl, r

    def get_orders(self, stream=None):
        pl = torch.empty(self.n_obs, dtype=torch.int32, device=self.device)
        pc = torch.empty(self.n_obs, dtype=torch.int32, device=self.device)
        lo = torch.empty(self.n_lms + 1, dtype=torch.int32, device=self.device)
        co = torch.empty(self.n_cams + 1, dtype=torch.int32, device=self.device)
        _lib.check("poba_get_orders", self.lib.poba_get_orders(self.handle, _ptr(pl), _ptr(pc), _ptr(lo), _ptr(co),
                                                               _stream(stream)))
        return pl, pc, lo, co

    def apply_P(self, v: torch.Tensor, stream=None):
        v = _dev(v, torch.float64, self.device, (self.n_cams, 9))
        out = torch.empty_like(v)
        _lib.check("poba_apply_P", self.lib.poba_apply_P(self.handle, _ptr(v), _ptr(out), _stream(stream)))
        return out

    # -- tuning ------------------------------------------------------------

    def set_tuning(self, key: str, value: int):
        _lib.check("poba_set_tuning", self.lib.poba_set_tuning(self.handle, _lib.TUNING[key], int(value)))

    def get_tuning(self, key: str) -> int:
        v = ctypes.c_int32()
        _lib.check("poba_get_tuning", self.lib.poba_get_tuning(self.handle, _lib.TUNING[key], ctypes.byref(v)))
        return int(v.value)

    # -- timing ------------------------------------------------------------

    def profile(self, enable: bool = True):
        _lib.check("poba_profile_enable", self.lib.poba_profile_enable(self.handle, 1 if enable else 0))

    def profile_read(self) -> dict:
        ms = (ctypes.c_double * 8)()
        n = (ctypes.c_int64 * 8)()
        _lib.check("poba_profile_read", self.lib.poba_profile_read(self.handle, ms, n))
        return {k: (ms[i], n[i]) for i, k in enumerate(_lib.KERNEL_CLASSES)}


class LMGraph:
    """A captured run of LM iterations; launch() replays it on a stream."""

    def __init__(self, problem: Problem, handle: ctypes.c_void_p, keep):
        self.problem, self.handle, self._keep = problem, handle, keep

    def launch(self, stream=None):
        _lib.check("poba_lm_graph_launch", self.problem.lib.poba_lm_graph_launch(self.handle, _stream(stream)))

    def close(self):
        if getattr(self, "handle", None):
            self.problem.lib.poba_lm_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def project(obs_cam, obs_lm, cams, lms, device="cuda", stream=None) -> torch.Tensor:
    """Model pixel positions [n_obs, 2] (poba_project)."""
    lib = _lib.load()
    obs_cam = _dev(obs_cam, torch.int32, device)
    obs_lm = _dev(obs_lm, torch.int32, device)
    cams = _dev(cams, torch.float64, device)
    lms = _dev(lms, torch.float64, device)
    n = int(obs_cam.numel())
    if n and (int(obs_cam.min()) < 0 or int(obs_cam.max()) >= cams.shape[0] or int(obs_lm.min()) < 0
              or int(obs_lm.max()) >= lms.shape[0]):
        raise ValueError("observation index out of range")
    out = torch.empty(n, 2, dtype=torch.float64, device=device)
    _lib.check("poba_project", lib.poba_project(n, _ptr(obs_cam), _ptr(obs_lm), _ptr(cams), _ptr(lms), _ptr(out),
                                                _stream(stream)))
    return out
