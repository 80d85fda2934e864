"""Power Stochastic Bundle Adjustment (Sec. 5.3, PoST) on one GPU.

Inside every LM iteration the cameras are split into clusters of at most
`max_cluster` (100 in the paper) by the library's greedy clustering of the
camera graph, with a new seeded draw of random edge weights per iteration
(the stochastic part); the reduced camera system keeps only its diagonal
blocks over the clusters, S_KK dx_K = -b~_K, and all of them are solved at
once by the batched power series: a batched handle whose problems are the
clusters and whose landmarks are the (cluster, landmark) pairs, with the V
and b_l of the whole problem written over its own.  The combined camera step
is back-substituted on the whole problem, whose handle also evaluates and
accepts or rejects the step.

This module only marshals: the clustering and the relabelling are host C++
of the library, every step of the solve runs in its kernels.
"""
from __future__ import annotations

import ctypes
import dataclasses

import numpy as np
import torch

from . import _lib
from .solver import LMOptions, Problem, _ptr, read_lm_state


class CameraGraph:
    """The camera graph of a problem (host, built once)."""

    def __init__(self, obs_cam, obs_lm, n_cams: int, n_lms: int):
        self.lib = _lib.load()
        self.obs_cam = np.ascontiguousarray(obs_cam, dtype=np.int32)
        self.obs_lm = np.ascontiguousarray(obs_lm, dtype=np.int32)
        self.n_cams, self.n_lms = int(n_cams), int(n_lms)
        h = ctypes.c_void_p()
        _lib.check("poba_camera_graph_create", self.lib.poba_camera_graph_create(
            self.obs_cam.size, self.obs_cam.ctypes.data, self.obs_lm.ctypes.data, self.n_cams, self.n_lms,
            ctypes.byref(h)))
        self.handle = h
        self.order = np.empty(self.obs_cam.size, np.int32)
        _lib.check("poba_camera_graph_order", self.lib.poba_camera_graph_order(self.handle, self.order.ctypes.data))

    def edges(self):
        n = ctypes.c_int64()
        _lib.check("poba_camera_graph_edges", self.lib.poba_camera_graph_edges(self.handle, ctypes.byref(n),
                                                                               None, None, None))
        a, b, w = (np.empty(n.value, np.int32) for _ in range(3))
        _lib.check("poba_camera_graph_edges", self.lib.poba_camera_graph_edges(
            self.handle, ctypes.byref(n), a.ctypes.data, b.ctypes.data, w.ctypes.data))
        return a, b, w

    def cluster(self, max_size: int, seed: int = -1):
        """Cluster index per camera and the number of clusters (seed < 0: the
        plain weights)."""
        out = np.empty(self.n_cams, np.int32)
        k = ctypes.c_int32()
        _lib.check("poba_camera_graph_cluster", self.lib.poba_camera_graph_cluster(
            self.handle, int(max_size), int(seed), out.ctypes.data, ctypes.byref(k)))
        return out, int(k.value)

    def layout(self, cluster: np.ndarray, n_clusters: int):
        """Batched layout of the clustered problem (see poba_camera_graph_layout);
        obs_vlm follows the observations in the order `self.order`."""
        cluster = np.ascontiguousarray(cluster, dtype=np.int32)
        n = self.obs_cam.size
        cam_pos = np.empty(self.n_cams, np.int32)
        obs_vlm = np.empty(n, np.int32)
        vlm_src = np.empty(n + n_clusters, np.int32)
        pco = np.empty(n_clusters + 1, np.int32)
        plo = np.empty(n_clusters + 1, np.int32)
        nv = ctypes.c_int32()
        _lib.check("poba_camera_graph_layout", self.lib.poba_camera_graph_layout(
            self.handle, cluster.ctypes.data, int(n_clusters), cam_pos.ctypes.data, obs_vlm.ctypes.data,
            vlm_src.ctypes.data, ctypes.byref(nv), pco.ctypes.data, plo.ctypes.data))
        return cam_pos, obs_vlm, vlm_src[:nv.value].copy(), pco, plo

    def close(self):
        if getattr(self, "handle", None):
            self.lib.poba_camera_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclasses.dataclass
class Clustered:
    """One draw of clusters and its batched handle."""
    cluster: np.ndarray
    n_clusters: int
    problem: Problem
    cam_pos: torch.Tensor    # clustered index of each camera
    cam_order: torch.Tensor  # camera at each clustered index
    vlm_src: torch.Tensor    # landmark of each (cluster, landmark) pair


class PoST:
    """PoST for one problem.  draws = 0 draws new clusters every LM
    iteration; draws = D > 0 draws D clusterings once and uses them in turn
    (their handles are kept)."""

    def __init__(self, obs_cam, obs_lm, obs_xy, n_cams: int, n_lms: int, max_cluster: int = 100, seed: int = 0,
                 draws: int = 0, precision: str = "f64", damping: str = "marquardt", loss: str = "l2",
                 huber_delta: float = 0.0, records: str = "jacobian", device="cuda"):
        self.device = torch.device(device)
        kw = dict(precision=precision, damping=damping, loss=loss, huber_delta=huber_delta, records=records,
                  device=self.device)
        self.kw = kw
        self.whole = Problem(obs_cam, obs_lm, obs_xy, n_cams, n_lms, **kw)
        self.graph = CameraGraph(obs_cam, obs_lm, n_cams, n_lms)
        # the clustered handles take the observations in the graph's (landmark) order
        order = torch.as_tensor(self.graph.order, device=self.device).long()
        self.obs_xy = torch.as_tensor(obs_xy, dtype=torch.float64, device=self.device)[order].contiguous()
        self.obs_cam_ordered = torch.as_tensor(self.graph.obs_cam, device=self.device).long()[order]
        self.n_cams, self.n_lms = int(n_cams), int(n_lms)
        self.max_cluster, self.seed, self.draws = int(max_cluster), int(seed), int(draws)
        self._pool = {}

    def clustered(self, iteration: int) -> Clustered:
        key = iteration % self.draws if self.draws else iteration
        if key in self._pool:
            return self._pool[key]
        cluster, k = self.graph.cluster(self.max_cluster, self.seed + key)
        cam_pos, obs_vlm, vlm_src, pco, plo = self.graph.layout(cluster, k)
        obs_cam = torch.as_tensor(cam_pos, device=self.device)[self.obs_cam_ordered]
        prob = Problem(obs_cam, obs_vlm, self.obs_xy, self.n_cams, int(vlm_src.size), prob_cam_off=pco,
                       prob_lm_off=plo, **self.kw)
        pos = torch.as_tensor(cam_pos, device=self.device).long()
        order = torch.empty_like(pos)
        order[pos] = torch.arange(self.n_cams, device=self.device)
        c = Clustered(cluster, k, prob, pos, order, torch.as_tensor(vlm_src, device=self.device).long())
        if self.draws:
            self._pool[key] = c
        return c

    def step(self, cams: torch.Tensor, lms: torch.Tensor, lam: float, m: int, eps: float, iteration: int = 0):
        """The clustered damped step at the whole handle's last linearisation
        (taken at cams, lms): camera step, landmark step, per-cluster info."""
        c = self.clustered(iteration)
        c.problem.linearize(cams[c.cam_order].contiguous(), lms[c.vlm_src].contiguous())
        _, V, _, bl = self.whole.get_blocks()
        c.problem.set_landmark_blocks(V[c.vlm_src].contiguous(), bl[c.vlm_src].contiguous())
        dxp_c, _, info = c.problem.power_solve(lam, m, eps)
        dxp = dxp_c[c.cam_pos].contiguous()
        dxl = self.whole.back_substitute(lam, dxp)
        return dxp, dxl, info, c

    def lm(self, cams: torch.Tensor, lms: torch.Tensor, opts: LMOptions | None = None, callback=None):
        """LM with the clustered step until the whole problem is done; cams,
        lms are updated in place.  callback(iteration, state dict) after every
        iteration.  Returns the list of LM states."""
        opts = opts or LMOptions()
        st = self.whole.lm_init(opts)
        out = []
        for it in range(opts.max_iters):
            self.whole.lm_begin(cams, lms, st)
            s = read_lm_state(st)
            if s["done"]:
                break
            dxp, dxl, _, _ = self.step(cams, lms, s["lambda"], opts.m, opts.eps, it)
            self.whole.lm_finish(cams, lms, st, dxp, dxl, opts)
            s = read_lm_state(st)
            out.append(s)
            if callback is not None:
                callback(it, s)
            if s["done"]:
                break
        return out

    def close(self):
        self.graph.close()
        for c in self._pool.values():
            c.problem.close()
        self._pool.clear()
        self.whole.close()
