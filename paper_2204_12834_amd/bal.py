"""Reader and writer for the text format of the Bundle Adjustment in the Large
(BAL) problems, so that a user-supplied problem file runs through the same
handles and LM steps as the synthetic workloads.

The format, whitespace separated:

    <n_cameras> <n_points> <n_observations>
    <camera> <point> <x> <y>                  (n_observations lines)
    9 values per camera: Rodrigues rotation (3), translation (3), f, k1, k2
    3 values per point

The camera model of the format is the one the library implements: P = R(w) X + t,
p = -P_xy / P_z, pixel = f (1 + k1 |p|^2 + k2 |p|^4) p, with the pixel origin
at the image centre.  Files ending in .bz2 are read and written through the
bz2 module.
"""
from __future__ import annotations

import bz2
import dataclasses
import os

import numpy as np


@dataclasses.dataclass
class BALProblem:
    """obs_cam, obs_lm [n_obs] int32; obs_xy [n_obs, 2] float64;
    cams [n_cams, 9] float64 (w_xyz, t_xyz, f, k1, k2); lms [n_lms, 3] float64."""

    name: str
    obs_cam: np.ndarray
    obs_lm: np.ndarray
    obs_xy: np.ndarray
    cams: np.ndarray
    lms: np.ndarray

    @property
    def n_cams(self) -> int:
        return int(self.cams.shape[0])

    @property
    def n_lms(self) -> int:
        return int(self.lms.shape[0])

    @property
    def n_obs(self) -> int:
        return int(self.obs_cam.shape[0])


def _open(path: str, mode: str):
    return bz2.open(path, mode) if path.endswith(".bz2") else open(path, mode)


def read(path: str) -> BALProblem:
    """Parses a BAL file; raises ValueError for a malformed one (counts that do
    not match the values present, non-integral or out-of-range indices)."""
    with _open(path, "rb") as f:
        tokens = f.read().split()
    if len(tokens) < 3:
        raise ValueError(f"{path}: missing header")
    try:
        nc, nl, no = (int(t) for t in tokens[:3])
    except ValueError as e:
        raise ValueError(f"{path}: header is not three integers") from e
    if nc < 1 or nl < 1 or no < 0:
        raise ValueError(f"{path}: bad counts {nc} {nl} {no}")
    need = 3 + 4 * no + 9 * nc + 3 * nl
    if len(tokens) != need:
        raise ValueError(f"{path}: expected {need} values for {nc} cameras, {nl} points, {no} observations, "
                         f"found {len(tokens)}")
    vals = np.array(tokens[3:], dtype=np.float64)
    obs = vals[:4 * no].reshape(no, 4)
    idx = obs[:, :2]
    if not np.all(np.isfinite(idx)) or np.any(idx != np.round(idx)):
        raise ValueError(f"{path}: observation indices are not integers")
    obs_cam = obs[:, 0].astype(np.int64)
    obs_lm = obs[:, 1].astype(np.int64)
    if no and (obs_cam.min() < 0 or obs_cam.max() >= nc or obs_lm.min() < 0 or obs_lm.max() >= nl):
        raise ValueError(f"{path}: observation index out of range")
    cams = vals[4 * no:4 * no + 9 * nc].reshape(nc, 9).copy()
    lms = vals[4 * no + 9 * nc:].reshape(nl, 3).copy()
    name = os.path.basename(path).split(".")[0]
    return BALProblem(name, obs_cam.astype(np.int32), obs_lm.astype(np.int32), obs[:, 2:4].copy(), cams, lms)


def write(path: str, p: BALProblem) -> None:
    """Writes p in the BAL format (17 significant digits, so a read returns the
    same doubles)."""
    out = [f"{p.n_cams} {p.n_lms} {p.n_obs}\n"]
    out.extend(f"{int(c)} {int(l)} {x!r} {y!r}\n"
               for c, l, (x, y) in zip(p.obs_cam, p.obs_lm, p.obs_xy.tolist()))
    out.extend(f"{v!r}\n" for v in p.cams.ravel().tolist())
    out.extend(f"{v!r}\n" for v in p.lms.ravel().tolist())
    with _open(path, "wb") as f:
        f.write("".join(out).encode())


def from_scene(scene, obs_xy: np.ndarray) -> BALProblem:
    """A BAL problem from a synthetic scene (its initial state) and observations."""
    return BALProblem(scene.name, np.asarray(scene.obs_cam, np.int32), np.asarray(scene.obs_lm, np.int32),
                      np.asarray(obs_xy, np.float64), np.asarray(scene.cams0, np.float64).copy(),
                      np.asarray(scene.lms0, np.float64).copy())
