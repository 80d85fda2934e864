"""Seeded synthetic bundle-adjustment scenes.

This module only builds scenes: it places cameras (look-at frames), samples
landmarks, decides visibility with a viewing-cone test, draws track lengths,
pixel noise, outliers and the perturbation of the initial state.  It does not
evaluate the camera projection model or any step of the solver.  A caller turns
ground truth into pixel observations with its own projection:

    obs = project(cams_gt, lms_gt)[obs_cam, obs_lm] + noise

Cameras follow the 9-parameter layout used by the public BAL files
(angle-axis rotation, translation, focal length, two radial coefficients); the
camera looks down its own -z axis.  Rotations are built as matrices from a
look-at frame and converted to angle-axis with the SO(3) logarithm; the
initial state turns each camera about its own centre and moves the centre
(App. B perturbs camera positions), so it also uses the SO(3) exponential.

The workloads stand in for the BAL problems the paper evaluates on (Sec. 5.1
"Dataset", Appendix D); none of the dataset's own content is reproduced.
Seeds, sizes and distributions are listed with each generator.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Scene",
    "ring_scene",
    "ladybug_scene",
    "city_scene",
    "batched_scenes",
    "concat_scenes",
    "config",
]


@dataclasses.dataclass
class Scene:
    """One synthetic problem.

    cams_gt, cams0 : [n_cams, 9] float64  (omega_xyz, t_xyz, f, k1, k2)
    lms_gt, lms0   : [n_lms, 3] float64
    obs_cam, obs_lm: [n_obs] int32, in a shuffled (unsorted) order
    noise          : [n_obs, 2] float64 pixel displacement added to the projection
    outlier        : [n_obs] bool, True where noise is an outlier displacement
    """

    name: str
    cams_gt: np.ndarray
    lms_gt: np.ndarray
    obs_cam: np.ndarray
    obs_lm: np.ndarray
    noise: np.ndarray
    outlier: np.ndarray
    cams0: np.ndarray
    lms0: np.ndarray

    @property
    def n_cams(self) -> int:
        return int(self.cams_gt.shape[0])

    @property
    def n_lms(self) -> int:
        return int(self.lms_gt.shape[0])

    @property
    def n_obs(self) -> int:
        return int(self.obs_cam.shape[0])


# ----------------------------------------------------------------------------
# frames
# ----------------------------------------------------------------------------

def _look_at(centers: np.ndarray, forwards: np.ndarray, up=(0.0, 0.0, 1.0)) -> np.ndarray:
    """World-to-camera rotation matrices [n,3,3] whose -z axis is `forwards`."""
    fwd = forwards / np.linalg.norm(forwards, axis=1, keepdims=True)
    zc = -fwd
    upv = np.broadcast_to(np.asarray(up, dtype=np.float64), zc.shape)
    yc = upv - np.sum(upv * zc, axis=1, keepdims=True) * zc
    yc /= np.linalg.norm(yc, axis=1, keepdims=True)
    xc = np.cross(yc, zc)
    return np.stack([xc, yc, zc], axis=1)


def _so3_log(R: np.ndarray) -> np.ndarray:
    """Angle-axis vectors [n,3] of rotation matrices [n,3,3]."""
    n = R.shape[0]
    out = np.zeros((n, 3))
    tr = np.trace(R, axis1=1, axis2=2)
    cos_t = np.clip((tr - 1.0) * 0.5, -1.0, 1.0)
    theta = np.arccos(cos_t)
    skew = np.stack([R[:, 2, 1] - R[:, 1, 2], R[:, 0, 2] - R[:, 2, 0], R[:, 1, 0] - R[:, 0, 1]], axis=1)
    small = theta < 1e-8
    near_pi = theta > math.pi - 1e-4
    gen = ~(small | near_pi)
    out[small] = 0.5 * skew[small]
    out[gen] = (theta[gen] / (2.0 * np.sin(theta[gen])))[:, None] * skew[gen]
    for i in np.nonzero(near_pi)[0]:
        B = 0.5 * (R[i] + np.eye(3))
        j = int(np.argmax(np.diag(B)))
        axis = B[:, j] / math.sqrt(max(B[j, j], 1e-300))
        if np.dot(axis, skew[i]) < 0:
            axis = -axis
        out[i] = theta[i] * axis
    return out


def _cameras(rng, centers, forwards, f_range=(450.0, 550.0), k_sigma=1e-3):
    R = _look_at(centers, forwards)
    omega = _so3_log(R)
    t = -np.einsum("nij,nj->ni", R, centers)
    n = centers.shape[0]
    f = rng.uniform(f_range[0], f_range[1], n)
    k = rng.normal(0.0, k_sigma, (n, 2))
    cams = np.concatenate([omega, t, f[:, None], k], axis=1)
    return cams, R


def _so3_exp(w: np.ndarray) -> np.ndarray:
    """Rotation matrices [n,3,3] of angle-axis vectors [n,3] (Rodrigues)."""
    th = np.linalg.norm(w, axis=1)
    k = w / np.where(th > 0.0, th, 1.0)[:, None]
    K = np.zeros((w.shape[0], 3, 3))
    K[:, 0, 1], K[:, 0, 2], K[:, 1, 2] = -k[:, 2], k[:, 1], -k[:, 0]
    K[:, 1, 0], K[:, 2, 0], K[:, 2, 1] = k[:, 2], -k[:, 1], k[:, 0]
    s, c = np.sin(th)[:, None, None], np.cos(th)[:, None, None]
    return np.eye(3)[None] + s * K + (1.0 - c) * (K @ K)


def _perturb(rng, cams, lms, rot_sigma=1e-2, pos_sigma=0.1, x0="centre"):
    """Initial state: every camera turned about its own centre by a rotation
    of angle-axis N(0, rot_sigma^2 I), its centre moved by N(0, pos_sigma^2 I)
    in world units, and every landmark moved by N(0, pos_sigma^2 I).  The
    translation follows from the moved centre, t0 = -R0 c0, so a camera far
    from the world origin moves no further than one near it.

    x0 = "angle-axis" instead adds the rotation noise to the angle-axis
    vector and the position noise to t, both at the other fixed (the earlier
    initial state, kept to reproduce measurements made with it; it moves a
    camera's centre by about rot_sigma |t|).  Both draw the same numbers in
    the same order."""
    rot = rng.normal(0.0, rot_sigma, (cams.shape[0], 3))
    pos = rng.normal(0.0, pos_sigma, (cams.shape[0], 3))
    cams0 = cams.copy()
    if x0 == "angle-axis":
        cams0[:, 0:3] += rot
        cams0[:, 3:6] += pos
    elif x0 == "centre":
        R = _so3_exp(cams[:, 0:3])
        centers = -np.einsum("nji,nj->ni", R, cams[:, 3:6])
        R0 = _so3_exp(rot) @ R
        c0 = centers + pos
        cams0[:, 0:3] = _so3_log(R0)
        cams0[:, 3:6] = -np.einsum("nij,nj->ni", R0, c0)
    else:
        raise ValueError(x0)
    lms0 = lms + rng.normal(0.0, pos_sigma, lms.shape)
    return cams0, lms0


def _finish(name, rng, cams, lms, cam_lists, noise_sigma=1.0, outlier_frac=0.0, outlier_px=20.0):
    """Flatten per-landmark camera lists into a shuffled observation list."""
    counts = np.array([len(c) for c in cam_lists], dtype=np.int64)
    obs_lm = np.repeat(np.arange(len(cam_lists), dtype=np.int32), counts)
    obs_cam = (np.concatenate(cam_lists).astype(np.int32) if len(cam_lists)
               else np.zeros(0, np.int32))
    return _finish_arrays(name, rng, cams, lms, obs_cam, obs_lm, noise_sigma, outlier_frac, outlier_px)


def _finish_arrays(name, rng, cams, lms, obs_cam, obs_lm, noise_sigma=1.0, outlier_frac=0.0,
                   outlier_px=20.0, x0="centre"):
    n = obs_cam.shape[0]
    perm = rng.permutation(n)
    obs_cam = np.ascontiguousarray(obs_cam[perm], dtype=np.int32)
    obs_lm = np.ascontiguousarray(obs_lm[perm], dtype=np.int32)
    noise = rng.normal(0.0, noise_sigma, (n, 2))
    outlier = np.zeros(n, dtype=bool)
    if outlier_frac > 0:
        outlier = rng.random(n) < outlier_frac
        phi = rng.uniform(0.0, 2.0 * math.pi, int(outlier.sum()))
        noise[outlier] = outlier_px * np.stack([np.cos(phi), np.sin(phi)], axis=1)
    cams0, lms0 = _perturb(rng, cams, lms, x0=x0)
    return Scene(name, cams, lms, obs_cam, obs_lm, noise, outlier, cams0, lms0)


# ----------------------------------------------------------------------------
# ring: cameras on a circle looking at the origin
# ----------------------------------------------------------------------------

def ring_scene(n_cams: int = 16, n_lms: int = 1000, track=(2, 6), seed: int = 0,
               radius: float = 10.0, box: float = 5.0, lm_sigma: float = 2.0,
               name: str = "ring") -> Scene:
    """Cameras at angles 2*pi*k/n on a circle of `radius` in z=0, facing the
    origin with +z up.  Landmarks ~ N(0, lm_sigma^2 I), rejection-sampled into
    [-box, box]^3 (every landmark is then in front of every camera).  Each
    landmark is seen by U{track[0]..track[1]} distinct cameras drawn uniformly.
    Noise N(0, 1 px) per coordinate."""
    rng = np.random.default_rng(seed)
    ang = 2.0 * math.pi * np.arange(n_cams) / n_cams
    centers = np.stack([radius * np.cos(ang), radius * np.sin(ang), np.zeros(n_cams)], axis=1)
    cams, _ = _cameras(rng, centers, -centers)
    lms = np.zeros((0, 3))
    while lms.shape[0] < n_lms:
        cand = rng.normal(0.0, lm_sigma, (2 * (n_lms - lms.shape[0]) + 16, 3))
        cand = cand[np.all(np.abs(cand) <= box, axis=1)]
        lms = np.concatenate([lms, cand], axis=0)
    lms = np.ascontiguousarray(lms[:n_lms])
    lo, hi = track
    k = rng.integers(lo, hi + 1, n_lms)
    k = np.minimum(k, n_cams)
    if n_lms:
        order = np.argsort(rng.random((n_lms, n_cams)), axis=1)
        cam_lists = [order[i, :k[i]] for i in range(n_lms)]
    else:
        cam_lists = []
    return _finish(name, rng, cams, lms, cam_lists)


# ----------------------------------------------------------------------------
# ladybug: a vehicle-mounted 5-direction rig driving along a path
# ----------------------------------------------------------------------------

def _trunc_geometric(rng, p, lo, hi, size):
    ks = np.arange(lo, hi + 1)
    w = (1.0 - p) ** (ks - lo)
    return rng.choice(ks, size=size, p=w / w.sum())


def ladybug_scene(n_cams: int = 1200, n_lms: int = 150_000, seed: int = 0,
                  geo_p: float = 0.4347, track=(2, 20), window: int = 60,
                  name: str = "ladybug") -> Scene:
    """Frame s (s = 0..n-1) sits at (s, 20 sin(s/150), 2) and looks
    horizontally at heading offset {0, +72, -72, +144, -144} deg (cycling per
    frame) from the direction of travel.  Landmarks are uniform in a corridor:
    arc position U(0, n-1), lateral offset +-U(3, 25), height U(0, 12).
    A landmark's track is k consecutive valid frames (depth > 0.5, normalised
    image radius < 1.2) around the frame nearest to it, k truncated-geometric
    (p = 0.4347 on {2..20}, mean 3.3); a landmark with fewer than k valid frames
    in +-`window` frames is redrawn."""
    rng = np.random.default_rng(seed)
    s = np.arange(n_cams, dtype=np.float64)

    def path(u):
        return np.stack([u, 20.0 * np.sin(u / 150.0), np.full_like(u, 2.0)], axis=-1)

    def tangent(u):
        d = np.stack([np.ones_like(u), (20.0 / 150.0) * np.cos(u / 150.0), np.zeros_like(u)], axis=-1)
        return d / np.linalg.norm(d, axis=-1, keepdims=True)

    centers = path(s)
    tan = tangent(s)
    offs = np.deg2rad(np.array([0.0, 72.0, -72.0, 144.0, -144.0]))[np.arange(n_cams) % 5]
    c, sn = np.cos(offs), np.sin(offs)
    fwd = np.stack([c * tan[:, 0] - sn * tan[:, 1], sn * tan[:, 0] + c * tan[:, 1], np.zeros(n_cams)], axis=1)
    cams, _ = _cameras(rng, centers, fwd)
    fwd_n = fwd / np.linalg.norm(fwd, axis=1, keepdims=True)

    lms = np.zeros((n_lms, 3))
    cam_lists: list = [None] * n_lms
    todo = np.arange(n_lms)
    ks = _trunc_geometric(rng, geo_p, track[0], track[1], n_lms)
    offsets = np.arange(-window, window + 1)
    while todo.size:
        m = todo.size
        u = rng.uniform(0.0, n_cams - 1, m)
        side = np.where(rng.random(m) < 0.5, -1.0, 1.0)
        lat = side * rng.uniform(3.0, 25.0, m)
        h = rng.uniform(0.0, 12.0, m)
        tg = tangent(u)
        nrm = np.stack([-tg[:, 1], tg[:, 0], np.zeros(m)], axis=1)
        X = path(u) + lat[:, None] * nrm
        X[:, 2] = h
        near = np.clip(np.rint(u).astype(np.int64), 0, n_cams - 1)
        frames = near[:, None] + offsets[None, :]
        inside = (frames >= 0) & (frames < n_cams)
        fr = np.clip(frames, 0, n_cams - 1)
        d = X[:, None, :] - centers[fr]
        depth = np.einsum("mwk,mwk->mw", d, fwd_n[fr])
        lat2 = np.einsum("mwk,mwk->mw", d, d) - depth ** 2
        valid = inside & (depth > 0.5) & (lat2 < (1.2 ** 2) * depth ** 2)
        redo = []
        for j in range(m):
            i = todo[j]
            vf = fr[j][valid[j]]
            k = ks[i]
            if vf.size < k:
                redo.append(i)
                continue
            pos = int(np.searchsorted(vf, near[j]))
            start = min(max(pos - k // 2, 0), vf.size - k)
            cam_lists[i] = vf[start:start + k]
            lms[i] = X[j]
        todo = np.asarray(redo, dtype=np.int64)
    return _finish(name, rng, cams, lms, cam_lists)


# ----------------------------------------------------------------------------
# city: cameras on an annulus looking into a central cylinder of landmarks
# ----------------------------------------------------------------------------

def _trunc_power(rng, alpha, lo, hi, size):
    ks = np.arange(lo, hi + 1, dtype=np.float64)
    w = ks ** (-alpha)
    return rng.choice(np.arange(lo, hi + 1), size=size, p=w / w.sum())


def city_scene(n_cams: int = 1100, n_lms: int = 780_000, seed: int = 0,
               alpha: float = 2.1397, track=(2, 200), outlier_frac: float = 0.02,
               outlier_px: float = 20.0, chunk: int = 8192, n_cand: int = 64,
               name: str = "city", x0: str = "centre") -> Scene:
    """Cameras uniform (by area) on the annulus 40 <= r <= 80, height
    U(1.5, 30), each looking at a target uniform in the disc of radius 20 at
    height U(0, 40).  Landmarks uniform in the cylinder r <= 25, z in [0, 40].
    Track length k ~ P(k) ∝ k^-2.1397 on {2..200} (mean 6.3); the k cameras
    are drawn uniformly among those with depth > 1 and normalised image radius
    < 1.5, and a landmark with fewer valid cameras is redrawn.  Noise N(0, 1 px);
    a fraction `outlier_frac` of observations is replaced by a displacement of
    `outlier_px` in a uniform random direction."""
    rng = np.random.default_rng(seed)
    rc = np.sqrt(rng.uniform(40.0 ** 2, 80.0 ** 2, n_cams))
    ac = rng.uniform(0.0, 2.0 * math.pi, n_cams)
    centers = np.stack([rc * np.cos(ac), rc * np.sin(ac), rng.uniform(1.5, 30.0, n_cams)], axis=1)
    rt = 20.0 * np.sqrt(rng.random(n_cams))
    at = rng.uniform(0.0, 2.0 * math.pi, n_cams)
    targets = np.stack([rt * np.cos(at), rt * np.sin(at), rng.uniform(0.0, 40.0, n_cams)], axis=1)
    fwd = targets - centers
    cams, _ = _cameras(rng, centers, fwd)
    fwd_n = fwd / np.linalg.norm(fwd, axis=1, keepdims=True)
    c_dot_f = np.sum(centers * fwd_n, axis=1)
    c_sq = np.sum(centers * centers, axis=1)

    ks = _trunc_power(rng, alpha, track[0], track[1], n_lms)
    ks = np.minimum(ks, n_cams)
    lms = np.zeros((n_lms, 3))
    sel_lm, sel_cam = [], []
    fwd32 = fwd_n.T.astype(np.float32)
    cen32 = centers.T.astype(np.float32)
    cdf32 = c_dot_f.astype(np.float32)[None, :]
    csq32 = c_sq.astype(np.float32)[None, :]
    todo = np.arange(n_lms)
    while todo.size:
        redo = []
        for a in range(0, todo.size, chunk):
            idx = todo[a:a + chunk]
            m = idx.size
            rl = 25.0 * np.sqrt(rng.random(m))
            al = rng.uniform(0.0, 2.0 * math.pi, m)
            X = np.stack([rl * np.cos(al), rl * np.sin(al), rng.uniform(0.0, 40.0, m)], axis=1)
            X32 = X.astype(np.float32)
            depth = X32 @ fwd32
            depth -= cdf32
            lat2 = X32 @ cen32
            lat2 *= -2.0
            lat2 += np.sum(X32 * X32, axis=1)[:, None]
            lat2 += csq32
            d2 = depth * depth
            lat2 -= d2
            valid = (depth > 1.0) & (lat2 < np.float32(1.5 ** 2) * d2)
            k = ks[idx]
            ok = valid.sum(axis=1) >= k
            kmax = int(k.max())
            # k cameras uniformly among the valid ones: draw candidates with
            # replacement and keep the first k distinct valid ones (a uniform
            # random k-subset); rows left short fall back to ranking every camera.
            cand = rng.integers(0, n_cams, (m, n_cand))
            good = np.take_along_axis(valid, cand, axis=1)
            srt = np.argsort(cand, axis=1, kind="stable")
            cs = np.take_along_axis(cand, srt, axis=1)
            dup = np.zeros_like(good)
            np.put_along_axis(dup, srt[:, 1:], cs[:, 1:] == cs[:, :-1], axis=1)
            good &= ~dup
            cum = np.cumsum(good, axis=1)
            fast = ok & (cum[:, -1] >= k)
            pick = good & (cum <= k[:, None]) & fast[:, None]
            order = np.zeros((m, kmax), dtype=np.int64)
            keep = np.zeros((m, kmax), dtype=bool)
            rows_f = np.nonzero(fast)[0]
            if rows_f.size:
                slot = cum - 1
                rr, cc = np.nonzero(pick)
                order[rr, slot[rr, cc]] = cand[rr, cc]
                keep[rows_f] = np.arange(kmax)[None, :] < k[rows_f, None]
            slow = np.nonzero(ok & ~fast)[0]
            if slow.size:
                score = rng.random((slow.size, n_cams), dtype=np.float32)
                score[~valid[slow]] = 2.0
                ks_s = k[slow]
                kk = int(ks_s.max())
                if kk < n_cams:
                    part = np.argpartition(score, kk - 1, axis=1)[:, :kk]
                else:
                    part = np.broadcast_to(np.arange(n_cams), (slow.size, n_cams))
                ps = np.take_along_axis(score, part, axis=1)
                od = np.take_along_axis(part, np.argsort(ps, axis=1, kind="stable"), axis=1)
                order[slow, :kk] = od
                keep[slow] = np.arange(kmax)[None, :] < ks_s[:, None]
            sel_lm.append(np.broadcast_to(idx[:, None], keep.shape)[keep])
            sel_cam.append(order[keep])
            lms[idx[ok]] = X[ok]
            redo.append(idx[~ok])
        todo = np.concatenate(redo) if redo else np.zeros(0, np.int64)
    obs_lm = np.concatenate(sel_lm).astype(np.int32) if sel_lm else np.zeros(0, np.int32)
    obs_cam = np.concatenate(sel_cam).astype(np.int32) if sel_cam else np.zeros(0, np.int32)
    return _finish_arrays(name, rng, cams, lms, obs_cam, obs_lm, 1.0, outlier_frac, outlier_px, x0)


# ----------------------------------------------------------------------------
# batched sub-problems
# ----------------------------------------------------------------------------

def batched_scenes(n_problems: int = 256, base_seed: int = 1000, cams_range=(20, 200),
                   lms_range=(2000, 40000), track=(2, 8)) -> list:
    """Independent ring problems; problem b uses seed base_seed + b and draws
    n_cams ~ round(logU(cams_range)), n_lms ~ round(logU(lms_range))."""
    out = []
    for b in range(n_problems):
        rng = np.random.default_rng(base_seed + b)
        nc = int(round(math.exp(rng.uniform(math.log(cams_range[0]), math.log(cams_range[1])))))
        nl = int(round(math.exp(rng.uniform(math.log(lms_range[0]), math.log(lms_range[1])))))
        out.append(ring_scene(nc, nl, track=track, seed=base_seed + b, name=f"batch{b}"))
    return out


def concat_scenes(scenes: list, name: str = "batch"):
    """Independent scenes as one scene over concatenated cameras and landmarks
    (observation indices shifted), plus the per-problem camera and landmark
    offsets [n + 1] each."""
    cam_off = np.cumsum([0] + [s.n_cams for s in scenes])
    lm_off = np.cumsum([0] + [s.n_lms for s in scenes])
    cat = lambda f: np.concatenate([getattr(s, f) for s in scenes])
    obs_cam = np.concatenate([s.obs_cam + cam_off[k] for k, s in enumerate(scenes)]).astype(np.int32)
    obs_lm = np.concatenate([s.obs_lm + lm_off[k] for k, s in enumerate(scenes)]).astype(np.int32)
    scene = Scene(name, cat("cams_gt"), cat("lms_gt"), obs_cam, obs_lm, cat("noise"), cat("outlier"), cat("cams0"),
                  cat("lms0"))
    return scene, cam_off.astype(np.int32), lm_off.astype(np.int32)


def config(name: str, **kw):
    """Named workloads.

    c1    : 16 cameras, 1,000 landmarks, tracks 2-6 (about 4,000 observations)
    c2    : 1,200 cameras, 150,000 landmarks, ~500k observations (vehicle rig)
    c3    : 1,100 cameras, 780,000 landmarks, ~4.9M observations, 2% outliers
    c4    : 256 uneven ring problems (list of scenes)
    c5    : 200 cameras, 50,000 landmarks, tracks 2-8 (~250k observations)
    """
    if name == "c1":
        return ring_scene(16, 1000, (2, 6), seed=kw.get("seed", 0), name="c1")
    if name == "c2":
        return ladybug_scene(seed=kw.get("seed", 0), name="c2")
    if name == "c3":
        return city_scene(seed=kw.get("seed", 0), name="c3", x0=kw.get("x0", "centre"))
    if name == "c4":
        return batched_scenes(kw.get("n_problems", 256))
    if name == "c5":
        return ring_scene(200, 50_000, (2, 8), seed=kw.get("seed", 0), name="c5")
    raise KeyError(name)
