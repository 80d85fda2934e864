"""Shared small problems for the oracle tests (CPU only)."""
from __future__ import annotations

import functools

import numpy as np

from paper_2204_12834_amd import synth
from oracle import camera, lm


class Problem:
    def __init__(self, scene, state="init", delta=None):
        self.scene = scene
        self.obs_cam = scene.obs_cam
        self.obs_lm = scene.obs_lm
        self.n_cams = scene.n_cams
        self.n_lms = scene.n_lms
        self.obs = camera.project(scene.cams_gt, scene.lms_gt, scene.obs_cam, scene.obs_lm) + scene.noise
        self.cams = scene.cams0 if state == "init" else scene.cams_gt
        self.lms = scene.lms0 if state == "init" else scene.lms_gt
        self.F, self.r, self.Jp, self.Jl = lm.linearize(self.cams, self.lms, self.obs_cam, self.obs_lm,
                                                        self.obs, delta)


@functools.lru_cache(maxsize=None)
def tiny(seed=3):
    """4 cameras, 12 landmarks: small enough for a finite-difference Jacobian of
    the whole residual vector."""
    return Problem(synth.ring_scene(4, 12, (2, 4), seed=seed, name="tiny"))


@functools.lru_cache(maxsize=None)
def c1():
    return Problem(synth.config("c1"))


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
