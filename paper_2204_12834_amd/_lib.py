"""ctypes view of libpoba.so (the C ABI declared in include/poba.h).

Loading fails loudly: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpoba.so")

POBA_OK = 0
POBA_ERR_WORKSPACE = 32
STATIC_WORKSPACE_BYTES = 64 << 20  # POBA_STATIC_WORKSPACE_BYTES
STATUS_BITS = {
    1: "invalid argument",
    2: "observation index out of range",
    4: "damped block not positive definite",
    8: "non-finite value",
    16: "HIP runtime error",
    32: "workspace missing or too small",
    64: "invalid state",
}
PRECISION = {"f64": 0, "f32": 1, "bf16": 2}
DAMPING = {"marquardt": 0, "identity": 1}
RECORDS = {"jacobian": 0, "point": 1}
LOSS = {"l2": 0, "huber": 1}
TUNING = {"tiles_per_wave": 0, "lm_ranges": 1, "lds_camera": 2, "range_lds": 3}
PRECOND = {"none": 0, "schur_jacobi": 1, "power": 2}
KERNEL_CLASSES = ["linearize", "inverse", "landmark_pass", "camera_pass", "camera_finish", "backsub", "eval", "other"]


class PobaDesc(ctypes.Structure):
    _fields_ = [
        ("n_cams", ctypes.c_int32),
        ("n_lms", ctypes.c_int32),
        ("n_obs", ctypes.c_int64),
        ("precision", ctypes.c_int32),
        ("damping", ctypes.c_int32),
        ("loss", ctypes.c_int32),
        ("piece_size", ctypes.c_int32),
        ("lm_ranges", ctypes.c_int32),
        ("records", ctypes.c_int32),
        ("huber_delta", ctypes.c_double),
    ]


class PobaSolveInfo(ctypes.Structure):
    _fields_ = [
        ("stop_order", ctypes.c_int32),
        ("stopped", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("norm_x", ctypes.c_double),
        ("norm_v", ctypes.c_double),
    ]


class PobaPCGInfo(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int32),
        ("converged", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("rel_residual", ctypes.c_double),
        ("rz", ctypes.c_double),
    ]


class PobaLMState(ctypes.Structure):
    _fields_ = [
        ("lambda_", ctypes.c_double),
        ("nu", ctypes.c_double),
        ("cost", ctypes.c_double),
        ("cost_new", ctypes.c_double),
        ("model_decrease", ctypes.c_double),
        ("gain", ctypes.c_double),
        ("iteration", ctypes.c_int32),
        ("accepted", ctypes.c_int32),
        ("done", ctypes.c_int32),
        ("need_linearize", ctypes.c_int32),
        ("stop_order", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("n_accepted", ctypes.c_int32),
        ("converged", ctypes.c_int32),
    ]


class PobaLMOptions(ctypes.Structure):
    _fields_ = [
        ("lambda0", ctypes.c_double),
        ("func_tol", ctypes.c_double),
        ("eps", ctypes.c_double),
        ("eta", ctypes.c_double),
        ("lambda_min", ctypes.c_double),
        ("lambda_max", ctypes.c_double),
        ("m", ctypes.c_int32),
        ("max_iters", ctypes.c_int32),
    ]


P = ctypes.c_void_p
I32 = ctypes.c_int32
I64 = ctypes.c_int64
F64 = ctypes.c_double

# name -> (restype, argtypes)
SIGNATURES = {
    "poba_version": (I32, []),
    "poba_status_string": (ctypes.c_char_p, [I32]),
    "poba_lm_default_options": (None, [ctypes.POINTER(PobaLMOptions)]),
    "poba_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(PobaDesc)]),
    "poba_create": (I32, [ctypes.POINTER(PobaDesc), P, P, P, P, ctypes.c_size_t, P, ctypes.POINTER(P)]),
    "poba_create_static": (I32, [ctypes.POINTER(PobaDesc), P, P, P, P, ctypes.POINTER(P)]),
    "poba_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(PobaDesc), I32]),
    "poba_batch_create": (I32, [ctypes.POINTER(PobaDesc), I32, ctypes.POINTER(I32), ctypes.POINTER(I32), P, P, P, P,
                                ctypes.c_size_t, P, ctypes.POINTER(P)]),
    "poba_lm_graph_create": (I32, [P, P, P, P, ctypes.POINTER(PobaLMOptions), I32, ctypes.POINTER(P)]),
    "poba_lm_graph_launch": (I32, [P, P]),
    "poba_lm_graph_destroy": (I32, [P]),
    "poba_destroy": (I32, [P]),
    "poba_linearize": (I32, [P, P, P, P, P]),
    "poba_power_solve": (I32, [P, F64, I32, F64, P, P, P, P]),
    "poba_pcg_solve": (I32, [P, F64, I32, I32, F64, I32, P, P, P, P, P]),
    "poba_lm_begin": (I32, [P, P, P, P, P]),
    "poba_lm_finish": (I32, [P, P, P, P, ctypes.POINTER(PobaLMOptions), P, P, P]),
    "poba_back_substitute": (I32, [P, F64, P, P, P]),
    "poba_set_landmark_blocks": (I32, [P, P, P, P]),
    "poba_camera_graph_create": (I32, [I64, P, P, I32, I32, ctypes.POINTER(P)]),
    "poba_camera_graph_destroy": (I32, [P]),
    "poba_camera_graph_edges": (I32, [P, ctypes.POINTER(I64), P, P, P]),
    "poba_camera_graph_cluster": (I32, [P, I32, I64, P, ctypes.POINTER(I32)]),
    "poba_camera_graph_layout": (I32, [P, P, I32, P, P, P, ctypes.POINTER(I32), P, P]),
    "poba_camera_graph_order": (I32, [P, P]),
    "poba_lm_init": (I32, [P, P, ctypes.POINTER(PobaLMOptions), P]),
    "poba_lm_step": (I32, [P, P, P, P, ctypes.POINTER(PobaLMOptions), P]),
    "poba_project": (I32, [I64, P, P, P, P, P, P]),
    "poba_get_blocks": (I32, [P, P, P, P, P, P]),
    "poba_get_jacobians": (I32, [P, I32, P, P, P, P]),
    "poba_get_orders": (I32, [P, P, P, P, P, P]),
    "poba_apply_P": (I32, [P, P, P, P]),
    "poba_solve_residual": (I32, [P, P, P, P]),
    "poba_set_observations": (I32, [P, P, P]),
    "poba_set_damping_frozen": (I32, [P, I32]),
    "poba_step_adjoint": (I32, [P, F64, I32, P, P, P, P, P, P, P, P, P, P, P, P]),
    "poba_set_tuning": (I32, [P, I32, I32]),
    "poba_get_tuning": (I32, [P, I32, ctypes.POINTER(I32)]),
    "poba_probe": (I32, [I32, P, P, ctypes.c_size_t, I32, P]),
    "poba_profile_enable": (I32, [P, I32]),
    "poba_profile_read": (I32, [P, ctypes.POINTER(F64), ctypes.POINTER(I64)]),
}

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Loads libpoba.so; raises RuntimeError if it is missing or incomplete."""
    global _lib
    if _lib is not None:
        return _lib
    # PyTorch supplies device memory and streams; importing it first makes the
    # library bind to the HIP runtime torch already loaded (two runtimes in one
    # process do not share devices).
    import torch  # noqa: F401
    if not os.path.exists(path):
        raise RuntimeError(f"libpoba.so not found at {path}: build it with paper_2204_12834_amd/build.py "
                           "(there is no fallback implementation)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)  # AttributeError if a symbol is missing
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def status_text(code: int) -> str:
    if code == 0:
        return "ok"
    return ", ".join(t for b, t in STATUS_BITS.items() if code & b) or f"status {code}"


class PobaError(RuntimeError):
    def __init__(self, where: str, code: int):
        super().__init__(f"{where} failed: {status_text(code)} (status {code})")
        self.code = code


def check(where: str, code: int) -> None:
    if code != POBA_OK:
        raise PobaError(where, code)
