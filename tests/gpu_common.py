"""Helpers for the GPU parity tests: build a problem on the device from a
synthetic scene with observations made by the oracle's projection."""
from __future__ import annotations

import functools
import sys

import numpy as np

from oracle import camera, lm, schur


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def observations(scene):
    return camera.project(scene.cams_gt, scene.lms_gt, scene.obs_cam, scene.obs_lm) + scene.noise


class Case:
    """A scene, its observations and the oracle's linearisation at the initial state."""

    def __init__(self, scene, delta=None):
        self.scene = scene
        self.obs = observations(scene)
        self.delta = delta
        self.F, self.r, self.Jp, self.Jl = lm.linearize(scene.cams0, scene.lms0, scene.obs_cam, scene.obs_lm,
                                                        self.obs, delta)

    def solve(self, lam, m, eps=0.0, damping="marquardt"):
        s = self.scene
        return schur.solve(self.Jp, self.Jl, self.r, s.obs_cam, s.obs_lm, s.n_cams, s.n_lms, lam, m, eps, damping)

    def problem(self, precision="f64", damping="marquardt", piece_size=0, lm_ranges=0, records="jacobian"):
        import torch
        from paper_2204_12834_amd.solver import Problem
        s = self.scene
        loss = "huber" if self.delta else "l2"
        return Problem(s.obs_cam, s.obs_lm, self.obs, s.n_cams, s.n_lms, precision=precision, damping=damping,
                       loss=loss, huber_delta=self.delta or 0.0, piece_size=piece_size, lm_ranges=lm_ranges,
                       device="cuda", records=records)

    def state(self):
        import torch
        s = self.scene
        return (torch.tensor(s.cams0, dtype=torch.float64, device="cuda"),
                torch.tensor(s.lms0, dtype=torch.float64, device="cuda"))


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def np_(t):
    return t.detach().cpu().numpy()


def round_bf16(a):
    """float64 -> float32 -> bfloat16 (round to nearest even) -> float64: the
    values a bfloat16 record holds."""
    f = np.asarray(a, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return (u.astype(np.uint32)).view(np.float32).astype(np.float64)

