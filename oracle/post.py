"""Clustered reduced camera system of Power Stochastic Bundle Adjustment
(Sec. 5.3, PoST) (oracle; test infrastructure: only tests/, smoke() and the
benchmark's CPU leg use it).

The paper summarises STBA as splitting the reduced camera system into camera
clusters of at most 100 cameras inside every LM iteration and solving the
per-cluster linear sub-problems in parallel; PoST solves each sub-problem with
the power series of Sec. 4.3 at the settings of Sec. 5.1.  The paper gives no
further detail, so these readings are taken:

  clustering  the camera graph has an edge between two cameras that observe a
              common landmark, weighted by the number of such landmarks;
              greedy agglomeration visits the edges by decreasing weight (ties:
              the smaller camera pair first) and merges the clusters of an edge
              when the merged cluster stays within the size cap; the stochastic
              part is a new clustering per LM iteration, drawn by multiplying
              every edge weight by a uniform number of its own;
  sub-problem the diagonal block of eq. (Sx) over cluster K,
              S_KK dx_K = -b~_K with S_KK = U_K - (W V^-1 W^T)_KK: the
              couplings between clusters are dropped, V and b~ are those of the
              whole problem;
  its solve   the power series of eq. (x_approx) with P_KK = U_K^-1 (W V^-1 W^T)_KK
              and the stop rule of eq. (qcriterion) per cluster;
  landmarks   dx_l = -V^-1 (b_l + W^T dx_p) with the combined camera step.
"""
from __future__ import annotations

import collections
import dataclasses

import numpy as np

from . import normal, schur


def camera_graph(obs_cam, obs_lm):
    """{(a, b): number of landmarks observed by both cameras a < b}."""
    cams_of = collections.defaultdict(set)
    for c, l in zip(obs_cam.tolist(), obs_lm.tolist()):
        cams_of[l].add(c)
    w = collections.Counter()
    for cs in cams_of.values():
        cs = sorted(cs)
        for i in range(len(cs)):
            for j in range(i + 1, len(cs)):
                w[(cs[i], cs[j])] += 1
    return w


_M64 = (1 << 64) - 1


def edge_uniform(seed, a, b):
    """Uniform number in [0, 1) for edge (a, b): the SplitMix64 finaliser
    (Steele, Lea and Flood, 2014) of seed ^ (a << 32 | b), top 53 bits."""
    z = (seed ^ ((a << 32) | b)) & _M64
    z = (z + 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    z ^= z >> 31
    return (z >> 11) / float(1 << 53)


def cluster_cameras(obs_cam, obs_lm, n_cams, max_size, seed=None):
    """Cluster index of every camera (clusters numbered in the order of their
    smallest camera).  With a seed, each edge weight is multiplied by its
    edge_uniform draw before the greedy pass (a new clustering per seed)."""
    w = camera_graph(np.asarray(obs_cam), np.asarray(obs_lm))
    if seed is not None:
        w = {e: float(c) * edge_uniform(seed, e[0], e[1]) for e, c in w.items()}
    edges = sorted(w.items(), key=lambda e: (-e[1], e[0][0], e[0][1]))
    root = list(range(n_cams))
    size = [1] * n_cams

    def find(a):
        while root[a] != a:
            a = root[a]
        return a

    for (a, b), _ in edges:
        ra, rb = find(a), find(b)
        if ra != rb and size[ra] + size[rb] <= max_size:
            lo, hi = min(ra, rb), max(ra, rb)
            root[hi] = lo
            size[lo] += size[hi]
    label = {}
    out = np.empty(n_cams, dtype=np.int64)
    for c in range(n_cams):
        r = find(c)
        if r not in label:
            label[r] = len(label)
        out[c] = label[r]
    return out


@dataclasses.dataclass
class ClusteredSolve:
    dxp: np.ndarray
    dxl: np.ndarray
    btilde: np.ndarray
    stop_orders: list     # per cluster: the highest power of P_KK summed
    n_clusters: int


def solve_clustered(Jp, Jl, r, obs_cam, obs_lm, n_cams, n_lms, lam, m, eps, cluster, damping="marquardt"):
    """One damped step with the camera step from the per-cluster power series."""
    U, V, bp, bl = normal.assemble(Jp, Jl, r, obs_cam, obs_lm, n_cams, n_lms)
    dp, dl = normal.damping_diagonals(U, V, damping)
    Ul, Vl = normal.damp(U, V, lam, dp, dl)
    Uinv, _ = normal.damped_inverse(Ul, lam * dp)
    Vinv, _ = normal.damped_inverse(Vl, lam * dl)
    bt = schur.reduced_rhs(Jp, Jl, obs_cam, obs_lm, bp, bl, Vinv)
    cluster = np.asarray(cluster)
    dxp = np.zeros((n_cams, 9))
    orders = []
    for k in range(int(cluster.max()) + 1 if n_cams else 0):
        mask = cluster == k

        def apply_PK(v):
            full = np.zeros((n_cams, 9))
            full[mask] = v
            return schur.apply_P(Jp, Jl, obs_cam, obs_lm, Uinv, Vinv, full)[mask]

        v = -schur.block_matvec(Uinv[mask], bt[mask])
        x = v.copy()
        order = 0
        for i in range(1, m + 1):
            v = apply_PK(v)
            x = x + v
            order = i
            if eps > 0.0:
                nx, nv = np.linalg.norm(x.ravel()), np.linalg.norm(v.ravel())
                if nx == 0.0 or (i + 1) * nv < eps * nx:
                    break
        dxp[mask] = x
        orders.append(order)
    dxl = schur.back_substitute(Jp, Jl, obs_cam, obs_lm, bl, Vinv, dxp)
    return ClusteredSolve(dxp, dxl, bt, orders, len(orders))
