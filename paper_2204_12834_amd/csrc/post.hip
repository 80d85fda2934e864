// Power Stochastic Bundle Adjustment (Sec. 5.3, PoST): the reduced camera
// system split into camera clusters of bounded size inside each LM iteration,
// every cluster's diagonal block S_KK dx_K = -b~_K solved by the power series.
//
// On the GPU the clusters become the problems of a batched handle whose
// landmarks are the (landmark, cluster) pairs that have observations (a
// landmark seen from two clusters is one landmark of each).  Its V and b_l are
// overwritten with those of the whole problem, so that its reduced system is
// exactly the block diagonal of the whole one: b~_c and U_c involve only the
// camera's own observations, and the landmark pass of a pair sums only the
// observations of its cluster.  The camera steps are then combined and the
// landmark step is back-substituted on the whole problem.
//
// Host side: the camera graph (edge weight: landmarks two cameras both
// observe), its greedy clustering under a size cap with seeded random edge
// weights, and the relabelling of a problem into cluster order.
#include <algorithm>
#include <cstring>
#include <memory>
#include <new>
#include <numeric>
#include <vector>

#include "device_ops.hpp"
#include "kernels.hpp"

struct poba_camera_graph_s {
    int32_t n_cams = 0, n_lms = 0;
    std::vector<int32_t> a, b, w;  // edges a < b with their weights, ordered by (a, b)
    // the observations in landmark order (stable): original index, camera, landmark
    std::vector<int32_t> lm_order, lm_order_cam, lm_order_lm;
};

namespace poba {

namespace {

// SplitMix64 finaliser (Steele, Lea and Flood, 2014) of seed ^ (a << 32 | b),
// as a uniform double in [0, 1) from its top 53 bits.
double edge_uniform(uint64_t seed, uint32_t a, uint32_t b) {
    uint64_t z = seed ^ ((uint64_t(a) << 32) | uint64_t(b));
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return double(z >> 11) * (1.0 / 9007199254740992.0);
}

// CSR of the distinct values of `val` grouped by `key` (keys in [0, nk)).
void group_distinct(int64_t n, const int32_t* key, const int32_t* val, int32_t nk, std::vector<int32_t>& off,
                    std::vector<int32_t>& out) {
    off.assign(size_t(nk) + 1, 0);
    for (int64_t i = 0; i < n; ++i) ++off[size_t(key[i]) + 1];
    for (int32_t k = 0; k < nk; ++k) off[k + 1] += off[k];
    std::vector<int32_t> fill(off.begin(), off.end() - 1);
    out.resize(size_t(n));
    for (int64_t i = 0; i < n; ++i) out[size_t(fill[key[i]]++)] = val[i];
    int32_t w = 0;
    for (int32_t k = 0; k < nk; ++k) {
        const int32_t a = off[k], e = off[k + 1];
        std::sort(out.begin() + a, out.begin() + e);
        const int32_t start = w;
        for (int32_t i = a; i < e; ++i)
            if (i == a || out[i] != out[i - 1]) out[size_t(w++)] = out[i];
        off[k] = start;
    }
    off[nk] = w;
    out.resize(size_t(w));
}

// The caller's camera step into the series sum, which the back-substitution
// dx_l = -V^-1 (b_l + W^T x) reads.
__global__ __launch_bounds__(kBlock) void k_copy_x(Buffers b, Sizes z, const double* __restrict__ x) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i < int64_t(z.nc) * 9) b.x[i] = x[i];
}

// V [nl][3][3] (symmetric; the upper triangle is read) and b_l [nl][3] into
// the handle's packed V and b_l.
__global__ __launch_bounds__(kBlock) void k_set_lm_blocks(Buffers b, Sizes z, const double* __restrict__ V,
                                                          const double* __restrict__ bl) {
    const int64_t l = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (l >= z.nl) return;
    const double* s = V + 9 * l;
    double* o = b.V + 6 * l;
    o[0] = s[0];
    o[1] = s[1];
    o[2] = s[2];
    o[3] = s[4];
    o[4] = s[5];
    o[5] = s[8];
    b.bl[3 * l] = bl[3 * l];
    b.bl[3 * l + 1] = bl[3 * l + 1];
    b.bl[3 * l + 2] = bl[3 * l + 2];
}

}  // namespace

}  // namespace poba

using namespace poba;

extern "C" {

poba_status poba_camera_graph_create(int64_t n_obs, const int32_t* obs_cam, const int32_t* obs_lm, int32_t n_cams,
                                     int32_t n_lms, poba_camera_graph* out) {
    try {
        if (!out || n_obs < 0 || n_cams < 1 || n_lms < 1 || (n_obs > 0 && (!obs_cam || !obs_lm)))
            return POBA_ERR_INVALID_ARG;
        for (int64_t i = 0; i < n_obs; ++i)
            if (obs_cam[i] < 0 || obs_cam[i] >= n_cams || obs_lm[i] < 0 || obs_lm[i] >= n_lms)
                return POBA_ERR_INDEX_RANGE;
        std::vector<int32_t> lm_off, lm_cams, cam_off, cam_lms;
        group_distinct(n_obs, obs_lm, obs_cam, n_lms, lm_off, lm_cams);
        group_distinct(n_obs, obs_cam, obs_lm, n_cams, cam_off, cam_lms);
        std::unique_ptr<poba_camera_graph_s> g(new poba_camera_graph_s);
        g->n_cams = n_cams;
        g->n_lms = n_lms;
        {
            std::vector<int64_t> off(static_cast<size_t>(n_lms) + 1, 0);
            for (int64_t i = 0; i < n_obs; ++i) ++off[size_t(obs_lm[i]) + 1];
            for (int32_t l = 0; l < n_lms; ++l) off[l + 1] += off[l];
            g->lm_order.resize(size_t(n_obs));
            for (int64_t i = 0; i < n_obs; ++i) g->lm_order[size_t(off[obs_lm[i]]++)] = int32_t(i);
            g->lm_order_cam.resize(size_t(n_obs));
            g->lm_order_lm.resize(size_t(n_obs));
            for (int64_t j = 0; j < n_obs; ++j) {
                g->lm_order_cam[size_t(j)] = obs_cam[g->lm_order[size_t(j)]];
                g->lm_order_lm[size_t(j)] = obs_lm[g->lm_order[size_t(j)]];
            }
        }
        std::vector<int32_t> cnt(size_t(n_cams), 0), touched;
        for (int32_t a = 0; a < n_cams; ++a) {
            touched.clear();
            for (int32_t k = cam_off[a]; k < cam_off[a + 1]; ++k) {
                const int32_t l = cam_lms[k];
                for (int32_t j = lm_off[l]; j < lm_off[l + 1]; ++j) {
                    const int32_t b = lm_cams[j];
                    if (b <= a) continue;
                    if (cnt[b]++ == 0) touched.push_back(b);
                }
            }
            std::sort(touched.begin(), touched.end());
            for (int32_t b : touched) {
                g->a.push_back(a);
                g->b.push_back(b);
                g->w.push_back(cnt[b]);
                cnt[b] = 0;
            }
        }
        *out = g.release();
        return POBA_OK;
    } catch (const std::bad_alloc&) {
        return POBA_ERR_WORKSPACE;  // host memory
    }
}

poba_status poba_camera_graph_edges(poba_camera_graph g, int64_t* n_edges, int32_t* a, int32_t* b, int32_t* w) {
    if (!g || !n_edges) return POBA_ERR_INVALID_ARG;
    const size_t n = g->a.size();
    if (a && b && w && n > 0) {
        std::memcpy(a, g->a.data(), n * 4);
        std::memcpy(b, g->b.data(), n * 4);
        std::memcpy(w, g->w.data(), n * 4);
    }
    *n_edges = int64_t(n);
    return POBA_OK;
}

poba_status poba_camera_graph_cluster(poba_camera_graph g, int32_t max_size, int64_t seed, int32_t* cluster,
                                      int32_t* n_clusters) {
    try {
        if (!g || !cluster || max_size < 1) return POBA_ERR_INVALID_ARG;
        const size_t ne = g->a.size();
        // Edges are visited heaviest first, ties in edge order ((a, b) ascending),
        // from a binary heap, until no two clusters fit together any more.
        const int32_t n = g->n_cams;
        std::vector<std::pair<double, int32_t>> heap(ne);
        for (size_t e = 0; e < ne; ++e)
            heap[e] = {seed < 0 ? double(g->w[e]) : double(g->w[e]) * edge_uniform(uint64_t(seed), g->a[e], g->b[e]),
                       int32_t(e)};
        // "less" for the max-heap: lighter, or as heavy and later in edge order
        auto later = [](const std::pair<double, int32_t>& x, const std::pair<double, int32_t>& y) {
            return x.first < y.first || (x.first == y.first && x.second > y.second);
        };
        std::make_heap(heap.begin(), heap.end(), later);
        std::vector<int32_t> root(static_cast<size_t>(n)), size(static_cast<size_t>(n), 1);
        std::iota(root.begin(), root.end(), 0);
        auto find = [&](int32_t x) {
            while (root[x] != x) {
                root[x] = root[root[x]];  // path halving; the roots stay as they are
                x = root[x];
            }
            return x;
        };
        // clusters by size (sizes up to the cap), to see when no merge can happen
        const bool track = max_size <= 4096;
        std::vector<int32_t> n_of_size(track ? size_t(max_size) + 1 : 0, 0);
        if (track) n_of_size[1] = n;
        auto can_merge = [&]() {
            int32_t first = 0;  // smallest size, then the next one (possibly equal)
            for (int32_t s2 = 1; s2 <= max_size; ++s2) {
                if (n_of_size[s2] == 0) continue;
                if (first == 0) {
                    if (n_of_size[s2] >= 2) return 2 * s2 <= max_size;
                    first = s2;
                } else {
                    return first + s2 <= max_size;
                }
            }
            return false;
        };
        size_t left = track && !can_merge() ? 0 : ne;
        while (left > 0) {
            std::pop_heap(heap.begin(), heap.begin() + left, later);
            const int32_t e = heap[--left].second;
            const int32_t ra = find(g->a[e]), rb = find(g->b[e]);
            if (ra != rb && size[ra] + size[rb] <= max_size) {
                const int32_t lo = std::min(ra, rb), hi = std::max(ra, rb);
                if (track) {
                    --n_of_size[size[lo]];
                    --n_of_size[size[hi]];
                    ++n_of_size[size[lo] + size[hi]];
                }
                root[hi] = lo;
                size[lo] += size[hi];
                if (track && !can_merge()) break;
            }
        }
        std::vector<int32_t> label(size_t(n), -1);
        int32_t k = 0;
        for (int32_t c = 0; c < n; ++c) {
            const int32_t r = find(c);
            if (label[r] < 0) label[r] = k++;
            cluster[c] = label[r];
        }
        if (n_clusters) *n_clusters = k;
        return POBA_OK;
    } catch (const std::bad_alloc&) {
        return POBA_ERR_WORKSPACE;  // host memory
    }
}

poba_status poba_camera_graph_order(poba_camera_graph g, int32_t* order) {
    if (!g || (!order && !g->lm_order.empty())) return POBA_ERR_INVALID_ARG;
    if (!g->lm_order.empty()) std::memcpy(order, g->lm_order.data(), g->lm_order.size() * 4);
    return POBA_OK;
}

poba_status poba_camera_graph_destroy(poba_camera_graph g) {
    delete g;
    return POBA_OK;
}

poba_status poba_camera_graph_layout(poba_camera_graph g, const int32_t* cluster, int32_t n_clusters,
                                     int32_t* cam_pos, int32_t* obs_vlm, int32_t* vlm_src, int32_t* n_vlm,
                                     int32_t* prob_cam_off, int32_t* prob_lm_off) {
    try {
        if (!g || n_clusters < 1 || !cluster || !cam_pos || !obs_vlm || !vlm_src || !n_vlm || !prob_cam_off ||
            !prob_lm_off)
            return POBA_ERR_INVALID_ARG;
        const int32_t n_cams = g->n_cams;
        const int64_t n_obs = int64_t(g->lm_order.size());
        for (int32_t c = 0; c < n_cams; ++c)
            if (cluster[c] < 0 || cluster[c] >= n_clusters) return POBA_ERR_INDEX_RANGE;
        // cameras in cluster order, ascending within a cluster
        std::fill(prob_cam_off, prob_cam_off + n_clusters + 1, 0);
        for (int32_t c = 0; c < n_cams; ++c) ++prob_cam_off[cluster[c] + 1];
        for (int32_t k = 0; k < n_clusters; ++k) {
            if (prob_cam_off[k + 1] == 0) return POBA_ERR_INVALID_ARG;  // empty cluster label
            prob_cam_off[k + 1] += prob_cam_off[k];
        }
        {
            std::vector<int32_t> fill(prob_cam_off, prob_cam_off + n_clusters);
            for (int32_t c = 0; c < n_cams; ++c) cam_pos[c] = fill[cluster[c]]++;
        }
        // (cluster, landmark) pairs with observations, numbered cluster-major then
        // by landmark; a cluster without any gets one unobserved pair (landmark 0).
        // The observations come in landmark order, so a pair is new for its
        // cluster exactly when the cluster's last landmark differs: one pass ranks
        // the pairs within their clusters, a second adds the clusters' offsets.
        const int32_t* oc = g->lm_order_cam.data();
        const int32_t* ol = g->lm_order_lm.data();
        std::vector<int32_t> cnt(static_cast<size_t>(n_clusters), 0), last(static_cast<size_t>(n_clusters), -1);
        for (int64_t j = 0; j < n_obs; ++j) {
            const int32_t k = cluster[oc[j]];
            if (last[k] != ol[j]) {
                last[k] = ol[j];
                ++cnt[k];
            }
            obs_vlm[j] = cnt[k] - 1;
        }
        int32_t v = 0;
        std::vector<int32_t> first(static_cast<size_t>(n_clusters));
        prob_lm_off[0] = 0;
        for (int32_t k = 0; k < n_clusters; ++k) {
            first[k] = v;
            if (cnt[k] == 0) vlm_src[v] = 0;
            v += std::max(cnt[k], 1);
            prob_lm_off[k + 1] = v;
        }
        for (int64_t j = 0; j < n_obs; ++j) {
            const int32_t k = cluster[oc[j]];
            obs_vlm[j] += first[k];
            vlm_src[obs_vlm[j]] = ol[j];
        }
        *n_vlm = v;
        return POBA_OK;
    } catch (const std::bad_alloc&) {
        return POBA_ERR_WORKSPACE;  // host memory
    }
}

poba_status poba_set_landmark_blocks(poba_problem p, const double* V, const double* bl, poba_stream stream) {
    (void)hipGetLastError();  // report only this call's launch errors
    if (!p || !V || !bl) return POBA_ERR_INVALID_ARG;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_set_lm_blocks, dim3(unsigned(ceil_div(p->z.nl, kBlock))), dim3(kBlock), 0, s, p->b, p->z, V,
                       bl);
    return hipGetLastError() == hipSuccess ? POBA_OK : POBA_ERR_HIP;
}

poba_status poba_back_substitute(poba_problem p, double lambda, const double* dx_cams, double* dx_lms,
                                 poba_stream stream) {
    (void)hipGetLastError();  // report only this call's launch errors
    if (!p || !dx_cams || !dx_lms || !(lambda > 0.0)) return POBA_ERR_INVALID_ARG;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    poba_status st;
    if ((st = launch_begin_solve(p, lambda, s))) return st;
    if ((st = launch_solve_prepare(p, s))) return st;
    hipLaunchKernelGGL(k_copy_x, dim3(unsigned(ceil_div(int64_t(p->z.nc) * 9, kBlock))), dim3(kBlock), 0, s, p->b,
                       p->z, dx_cams);
    if (hipGetLastError() != hipSuccess) return POBA_ERR_HIP;
    // the camera step is copied back to b.dxp (the LM step buffer), unchanged
    return launch_backsub_from_x(p, p->b.dxp, dx_lms, s);
}

}  // extern "C"
