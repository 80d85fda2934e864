"""Pins of the oracle's clustered reduced camera system (Sec. 5.3, PoST), on
the CPU: the greedy camera clustering on a hand-worked graph, and the
per-cluster power series against the dense diagonal blocks of the reduced
camera system, the unclustered series and the block-diagonal special cases."""
import numpy as np
import pytest
import scipy.linalg

from oracle import dense, lm, normal, post, schur
from oracle_fixtures import c1, rel, tiny

# Hand-worked camera graph: landmarks and the cameras that observe them.
#   w(0,1) = 3, w(3,4) = 3, w(1,2) = 2, w(4,5) = 2, w(0,5) = 1, w(2,3) = 1
GRAPH = [(0, 1), (0, 1), (0, 1), (1, 2), (1, 2), (3, 4), (3, 4), (3, 4), (2, 3), (4, 5), (4, 5), (0, 5)]


def _graph_obs(extra=()):
    cams, lms = [], []
    for l, pair in enumerate(GRAPH):
        for c in pair:
            cams.append(c)
            lms.append(l)
    for c, l in extra:
        cams.append(c)
        lms.append(l)
    return np.array(cams), np.array(lms)


@pytest.mark.parametrize("cap,want", [
    # edges in order (0,1) (3,4) (1,2) (4,5) (0,5) (2,3)
    (1, [0, 1, 2, 3, 4, 5]),
    (2, [0, 0, 1, 2, 2, 3]),       # (1,2) would make 3
    (3, [0, 0, 0, 1, 1, 1]),       # (0,5) would make 6
    (6, [0, 0, 0, 0, 0, 0]),
])
def test_clustering_hand_worked(cap, want):
    oc, ol = _graph_obs()
    assert post.camera_graph(oc, ol) == {(0, 1): 3, (1, 2): 2, (3, 4): 3, (2, 3): 1, (4, 5): 2, (0, 5): 1}
    assert post.cluster_cameras(oc, ol, 6, cap).tolist() == want


def test_clustering_counts_a_landmark_once_per_camera_pair():
    # camera 0 observes landmark 11 (shared with camera 5) three times
    oc, ol = _graph_obs(extra=[(0, 11), (0, 11)])
    assert post.camera_graph(oc, ol)[(0, 5)] == 1
    assert post.cluster_cameras(oc, ol, 6, 3).tolist() == [0, 0, 0, 1, 1, 1]


def test_clustering_cap_and_partition_on_c1():
    P = c1()
    for cap in [1, 3, 5, 16]:
        cl = post.cluster_cameras(P.obs_cam, P.obs_lm, P.n_cams, cap)
        sizes = np.bincount(cl)
        assert sizes.max() <= cap and sizes.sum() == P.n_cams
        # labels in the order of each cluster's smallest camera
        first = [int(np.flatnonzero(cl == k)[0]) for k in range(len(sizes))]
        assert first == sorted(first)


def _parts(P, lam):
    J = dense.dense_jacobian(P.Jp, P.Jl, P.obs_cam, P.obs_lm, P.n_cams, P.n_lms)
    return dense.schur_parts(J, P.r, lam, P.n_cams)


@pytest.mark.parametrize("eps", [0.0, 0.05])
def test_one_cluster_is_the_power_series(eps):
    P = c1()
    cl = np.zeros(P.n_cams, dtype=np.int64)
    got = post.solve_clustered(P.Jp, P.Jl, P.r, P.obs_cam, P.obs_lm, P.n_cams, P.n_lms, 1e-2, 12, eps, cl)
    ref = schur.solve(P.Jp, P.Jl, P.r, P.obs_cam, P.obs_lm, P.n_cams, P.n_lms, 1e-2, 12, eps)
    assert got.stop_orders == [ref.series.stop_order]
    assert rel(got.dxp, ref.dxp) <= 1e-12 and rel(got.dxl, ref.dxl) <= 1e-12


def test_order_zero_does_not_depend_on_the_clusters():
    P = c1()
    a = post.solve_clustered(P.Jp, P.Jl, P.r, P.obs_cam, P.obs_lm, P.n_cams, P.n_lms, 1e-2, 0, 0.0,
                             np.arange(P.n_cams))
    b = post.solve_clustered(P.Jp, P.Jl, P.r, P.obs_cam, P.obs_lm, P.n_cams, P.n_lms, 1e-2, 0, 0.0,
                             np.zeros(P.n_cams, dtype=np.int64))
    assert rel(a.dxp, b.dxp) <= 1e-15


@pytest.mark.parametrize("cap", [1, 4, 7])
def test_each_cluster_converges_to_its_dense_block(cap):
    """m -> infinity: dx_K = -S_KK^-1 b~_K with the dense diagonal block of S
    (couplings between clusters dropped), and dx_l the dense back-substitution."""
    P = c1()
    lam = 1.0
    cl = post.cluster_cameras(P.obs_cam, P.obs_lm, P.n_cams, cap)
    U, W, V, S, bt, bp, bl = _parts(P, lam)
    got = post.solve_clustered(P.Jp, P.Jl, P.r, P.obs_cam, P.obs_lm, P.n_cams, P.n_lms, lam, 400, 0.0, cl)
    want = np.zeros(9 * P.n_cams)
    for k in range(int(cl.max()) + 1):
        idx = np.concatenate([np.arange(9 * c, 9 * c + 9) for c in np.flatnonzero(cl == k)])
        SKK = S[np.ix_(idx, idx)]
        want[idx] = -scipy.linalg.cho_solve(scipy.linalg.cho_factor(SKK), bt[idx])
    assert rel(got.dxp.ravel(), want) <= 1e-9
    dxl = -np.linalg.solve(V, bl + W.T @ got.dxp.ravel())
    assert rel(got.dxl.ravel(), dxl) <= 1e-10
    if cl.max() > 0:  # dropped couplings: not the solution of the whole system
        full = -scipy.linalg.cho_solve(scipy.linalg.cho_factor(S), bt)
        assert rel(got.dxp.ravel(), full) > 1e-6


def test_clustered_lm_descends_and_converges():
    """LM with the clustered step and a new draw of clusters per iteration
    (the stochastic clustering) on the tiny ring: accepted costs fall
    monotonically and come within 1e-3 (f0 - f*) of the optimum f* of the LM
    with dense solves (the performance-profile tolerance of Sec. 5); with the
    same two clusters in every iteration it stalls above 1e-2 (f0 - f*): the
    dropped couplings are never seen."""
    P = tiny()
    opts = lm.LMOptions(m=20, eps=0.0, max_iters=200, func_tol=1e-10)
    ref = lm.lm(P.scene.cams0, P.scene.lms0, P.obs_cam, P.obs_lm, P.obs, opts, solver="dense")
    best = min(it.cost_new for it in ref.iterations if it.accepted)
    f0 = ref.iterations[0].cost

    def draw(it):
        return post.cluster_cameras(P.obs_cam, P.obs_lm, P.n_cams, 2, seed=it)

    res = lm.lm(P.scene.cams0, P.scene.lms0, P.obs_cam, P.obs_lm, P.obs, opts, solver="clustered", cluster=draw)
    acc = [it.cost_new for it in res.iterations if it.accepted]
    assert all(b < a for a, b in zip(acc, acc[1:]))
    assert acc[-1] <= lm.cost_threshold(f0, best, 1e-3)
    fixed = post.cluster_cameras(P.obs_cam, P.obs_lm, P.n_cams, 2)
    res_fixed = lm.lm(P.scene.cams0, P.scene.lms0, P.obs_cam, P.obs_lm, P.obs, opts, solver="clustered",
                      cluster=fixed)
    assert min(it.cost_new for it in res_fixed.iterations if it.accepted) > lm.cost_threshold(f0, best, 1e-2)
