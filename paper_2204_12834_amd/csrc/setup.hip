// Problem set-up: workspace layout, observation orders and work tiles.
//
// The paper groups Jacobian blocks per landmark (Sec. 5 "Efficient storage").
// Here every observation is kept in two orders: landmark-major (for W^T v,
// the landmark side of the series) and camera-major (for W s, the camera
// side), each a stable sort of the observations by (index, original
// position).  Landmark-major positions are cut into 64-observation tiles; a
// tile owns the landmarks whose first observation falls inside it, so a
// wavefront reduces whole landmark segments without talking to other waves.
// Camera-major positions are cut into pieces of at most `piece` observations
// that never straddle two cameras.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <mutex>

#include "camera_model.hpp"
#include "common.hpp"

namespace poba {

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Landmark ranges whose slices of the landmark vector (three scalars of
// `sbytes` per observed landmark) meet the LDS target of the range-staged
// camera pass; a multiple of the die count above one.
int32_t point_ranges(int64_t nseg, int sbytes) {
    const int64_t bytes = nseg * 3 * sbytes;
    if (bytes <= kRangeLds) return 1;
    return int32_t(std::min<int64_t>(4096, kXcds * ceil_div(bytes, kXcds * kRangeLds)));
}

bool compute_sizes(const poba_desc* d, int32_t n_problems, Sizes* z) {
    if (!d) return false;
    if (n_problems < 1 || n_problems > d->n_cams || n_problems > d->n_lms) return false;
    if (d->n_cams < 1 || d->n_cams >= (1 << 30) || d->n_lms < 1 || d->n_obs < 0 || d->n_obs >= (int64_t(1) << 31))
        return false;
    if (d->precision < POBA_F64 || d->precision > POBA_F32_BF16J) return false;
    if (d->damping != POBA_DAMP_MARQUARDT && d->damping != POBA_DAMP_IDENTITY) return false;
    if (d->loss != POBA_LOSS_L2 && d->loss != POBA_LOSS_HUBER) return false;
    if (d->loss == POBA_LOSS_HUBER && !(d->huber_delta > 0.0)) return false;
    if (d->piece_size < 0) return false;
    if (d->records != POBA_RECORDS_JACOBIAN && d->records != POBA_RECORDS_POINT) return false;
    if (d->records == POBA_RECORDS_POINT && d->precision == POBA_F32_BF16J) return false;
    if (d->lm_ranges < 0 || (d->lm_ranges > 1 && d->lm_ranges % kXcds != 0) || d->lm_ranges > 4096) return false;
    z->nc = d->n_cams;
    z->nl = d->n_lms;
    z->np = n_problems;
    z->N = d->n_obs;
    z->npad = std::max<int64_t>(ceil_div(z->N, kWave) * kWave, kWave);
    z->ntiles = z->N / kWave + 1;
    z->piece = d->piece_size ? d->piece_size : kDefaultPiece;
    z->piece = std::max(64, std::min(z->piece, 1 << 20));
    // automatic choice: one range per die when the landmark vector exceeds the
    // slice size, more when a slice per die would still be larger
    const int64_t s_bytes_max = int64_t(z->nl) * 32;
    int64_t auto_max = s_bytes_max > kRangeBytes ? kXcds * ceil_div(s_bytes_max, kXcds * kRangeBytes) : 1;
    if (d->records == POBA_RECORDS_POINT)
        auto_max = std::max<int64_t>(auto_max, point_ranges(z->nl, d->precision == POBA_F64 ? 8 : 4));
    z->ranges_max = d->lm_ranges ? d->lm_ranges : auto_max;
    z->npieces_max = z->N / z->piece + int64_t(z->nc) * z->ranges_max + 1;
    z->jbytes = d->precision == POBA_F64 ? 8 : (d->precision == POBA_F32 ? 4 : 2);
    z->sbytes = d->precision == POBA_F64 ? 8 : 4;
    z->point = d->records == POBA_RECORDS_POINT ? 1 : 0;
    z->rbytes = z->point ? 4 * z->sbytes : 24 * z->jbytes;
    return true;
}

size_t sort_tmp_upper_bound(int64_t N) {
    // onesweep radix sort scratch: lookback state and histograms, well below
    // this bound for every supported size (checked against the query in
    // poba_create).
    return (size_t(64) << 20) + size_t(N) * 8;
}

size_t layout(const poba_desc* d, const Sizes& z, char* base, Buffers* b, size_t sort_tmp_bytes) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        off = align_up(off, 256);
        char* p = base ? base + off : nullptr;
        off += std::max<size_t>(bytes, 1);
        return p;
    };
    const size_t N = size_t(z.N), nc = size_t(z.nc), nl = size_t(z.nl);
    const size_t jrec = size_t(z.npad) * size_t(z.rbytes);
    Buffers t{};
    t.perm_l = (int32_t*)take(N * 4);
    t.perm_c = (int32_t*)take(N * 4);
    t.lo_cam = (uint32_t*)take(N * 4);
    t.co_lm = (int32_t*)take(N * 4);
    t.co_seg = (int32_t*)take(N * 4);
    t.lm_off = (int32_t*)take((nl + 1) * 4);
    t.cam_off = (int32_t*)take((nc + 1) * 4);
    t.nel = (int32_t*)take(nl * 4);
    t.tile_start = (int32_t*)take(size_t(z.ntiles + 1) * 4);
    t.seg_base = (int32_t*)take(size_t(z.ntiles) * 4);
    t.piece_cam = (int32_t*)take(size_t(z.npieces_max) * 4);
    t.piece_begin = (int32_t*)take(size_t(z.npieces_max) * 4);
    t.piece_end = (int32_t*)take(size_t(z.npieces_max) * 4);
    t.piece_grp = (int32_t*)take(size_t(z.npieces_max) * 4);
    t.cam_piece = (int32_t*)take((nc + 1) * 4);
    t.grp_off = (int32_t*)take((nc * size_t(z.ranges_max) + 1) * 4);
    t.grp_piece = (int32_t*)take((nc * size_t(z.ranges_max) + 1) * 4);
    t.dgrp_off = (int32_t*)take((nc * kXcds + 1) * 4);
    t.sched = (int32_t*)take(size_t(kXcds) * size_t(z.npieces_max) * 4);
    t.sched_rec = (PieceRec*)take(size_t(kXcds) * size_t(z.npieces_max) * sizeof(PieceRec));
    t.cw_rec = (int4*)take(size_t(z.ranges_max) * kMaxRangeBlocks * kMaxCwWaves * sizeof(int4));
    t.cw_list = (int4*)take(z.point ? size_t(z.ranges_max) * nc * sizeof(int4) : 0);
    t.obs_lo = (double*)take(N * 16);
    t.obs_co = (double*)take(N * 16);
    t.J_lo = take(jrec);
    t.J_co = take(jrec);
    t.r_co = (double*)take(N * 16);
    t.U = (double*)take(nc * 81 * 8);
    t.bp = (double*)take(nc * 9 * 8);
    t.V = (double*)take(nl * 6 * 8);
    t.bl = (double*)take(nl * 3 * 8);
    t.Uinv = (double*)take(nc * 81 * 8);
    t.Dp = (double*)take(nc * 9 * 8);
    t.Dl = (double*)take(nl * 3 * 8);
    t.Vinv = take(nl * 6 * z.sbytes);
    t.vinv64 = (double*)take(nl * 6 * 8);
    t.ybl = (double*)take(nl * 4 * 8);
    t.s = take(nl * 4 * 8);  // also holds float64 landmark vectors
    t.v = (double*)take(nc * 9 * 8);
    t.vq = take(nc * 28 * 8);  // camera vector (stride 12), or folded camera records (stride kFoldStride)
    t.x = (double*)take(nc * 9 * 8);
    t.bt = (double*)take(nc * 9 * 8);
    t.part = (double*)take(size_t(z.npieces_max) * 54 * 8);
    t.part_grp = take(z.point ? size_t(z.ranges_max) * nc * 9 * size_t(z.sbytes) : 0);
    t.dxl = (double*)take(nl * 3 * 8);
    t.dxp = (double*)take(nc * 9 * 8);
    t.cam_rec = (double*)take(nc * 24 * 8);
    t.lin_rec = (double*)take(nc * 24 * 8);
    t.cams_new = (double*)take(nc * 9 * 8);
    t.lm_trial = (double*)take(nl * 8 * 8);
    t.piece_red = (double*)take(size_t(z.npieces_max) * 3 * 8);
    t.cam_red = (double*)take(nc * 2 * 8);
    t.xq = (double*)take(nc * 28 * 8);
    t.cg = (double*)take(5 * nc * 9 * 8);
    t.sj = (double*)take(nc * 81 * 8);
    const size_t np1 = size_t(z.np) + 1;
    t.prob_cam_off = (int32_t*)take(np1 * 4);
    t.prob_lm_off = (int32_t*)take(np1 * 4);
    t.prob_piece_off = (int32_t*)take(np1 * 4);
    t.cam_prob = (int32_t*)take(nc * 4);
    t.lm_prob = (int32_t*)take(nl * 4);
    t.pctl = (PCtrl*)take(size_t(z.np) * sizeof(PCtrl));
    t.pcg_ctl = (PcgCtl*)take(size_t(z.np) * sizeof(PcgCtl));

    t.ctrl = (Ctrl*)take(sizeof(Ctrl));
    t.keys_tmp = (int32_t*)take(N * 4);
    t.vals_tmp = (int32_t*)take(N * 4);
    t.keys_out = (int32_t*)take(N * 4);
    t.iota = (int32_t*)take(N * 4);
    t.scratch_i = (int32_t*)take(2 * (std::max(nc, nl) + 2) * 4);
    t.sort_tmp_bytes = sort_tmp_bytes;
    t.sort_tmp = take(sort_tmp_bytes);
    if (b) *b = t;
    return align_up(off, 256);
}

// ------------------------------------------------------------------ kernels --

// Every index in range, and camera and landmark of one observation in the
// same problem.
__global__ void k_check_indices(const int32_t* obs_cam, const int32_t* obs_lm, int64_t N, int32_t nc,
                                int32_t nl, const int32_t* cam_prob, const int32_t* lm_prob, int32_t* err,
                                int32_t* iota) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= N) return;
    iota[i] = int32_t(i);
    const int32_t c = obs_cam[i], l = obs_lm[i];
    if (c < 0 || c >= nc || l < 0 || l >= nl) {
        atomicOr(err, 1);
        return;
    }
    if (cam_prob[c] != lm_prob[l]) atomicOr(err, 2);
}

// prob[i] = the problem j with off[j] <= i < off[j+1] (off ascending).
__global__ void k_fill_prob(const int32_t* off, int32_t np, int32_t n, int32_t* prob) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t lo = 0, hi = np - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (off[mid] <= i) lo = mid; else hi = mid - 1;
    }
    prob[i] = lo;
}

// Piece data of every schedule slot.
__global__ void k_sched_rec(const int32_t* sched, const int32_t* piece_begin, const int32_t* piece_end,
                            const int32_t* piece_cam, const int32_t* cam_prob, int64_t n, PieceRec* out) {
    const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int32_t p = sched[j];
    PieceRec r{-1, 0, 0, 0, 0, 0, 0, 0};
    if (p >= 0) {
        r.p = p;
        r.begin = piece_begin[p];
        r.end = piece_end[p];
        r.cam = piece_cam[p];
        r.prob = cam_prob[r.cam];
    }
    out[j] = r;
}

// First camera piece of every problem (pieces are ordered by camera).
__global__ void k_prob_pieces(const int32_t* prob_cam_off, const int32_t* cam_piece, int32_t np,
                              int32_t* prob_piece_off) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j > np) return;
    prob_piece_off[j] = cam_piece[prob_cam_off[j]];
}

// off[k] = first sorted position whose key is >= k (k = 0..n); keys sorted.
__global__ void k_segment_offsets(const int32_t* keys, int64_t N, int32_t n, int32_t* off) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i > N) return;
    const int32_t prev = i == 0 ? -1 : keys[i - 1];
    const int32_t cur = i == N ? n : keys[i];
    for (int32_t k = prev + 1; k <= cur; ++k) off[k] = int32_t(i);
}

__global__ void k_gather_orders(const int32_t* perm_l, const int32_t* perm_c, const int32_t* obs_cam,
                                const int32_t* obs_lm, const double* obs_xy, const int32_t* lm_off,
                                const int32_t* sorted_lm, const int32_t* rank, int64_t N, uint32_t* lo_cam,
                                int32_t* co_lm, int32_t* co_seg, double* obs_lo, double* obs_co) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int32_t ol = perm_l[i];
    const int32_t l = sorted_lm[i];
    const bool head = lm_off[l] == int32_t(i);
    const bool tail = lm_off[l + 1] == int32_t(i + 1);
    lo_cam[i] = uint32_t(obs_cam[ol]) | (head ? kHeadBit : 0u) | (tail ? kTailBit : 0u);
    obs_lo[2 * i] = obs_xy[2 * ol];
    obs_lo[2 * i + 1] = obs_xy[2 * ol + 1];
    const int32_t oc = perm_c[i];
    const int32_t lc = obs_lm[oc];
    co_lm[i] = lc;
    co_seg[i] = rank[lc];
    obs_co[2 * i] = obs_xy[2 * oc];
    obs_co[2 * i + 1] = obs_xy[2 * oc + 1];
}

// flags[l] = 1 if landmark l has an observation.
__global__ void k_nonempty_flags(const int32_t* lm_off, int32_t nl, int32_t* flags) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nl) return;
    flags[i] = lm_off[i + 1] > lm_off[i] ? 1 : 0;
}

// nel[rank[l]] = l for non-empty l (rank = exclusive scan of the flags).
__global__ void k_compact_nonempty(const int32_t* lm_off, const int32_t* rank, int32_t nl, int32_t* nel) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nl) return;
    if (lm_off[i + 1] > lm_off[i]) nel[rank[i]] = i;
}

// Tile t covers landmark-major positions [tile_start[t], tile_start[t+1]):
// tile_start[t] is the first landmark head at or after 64 t (N if none), and
// seg_base[t] counts the non-empty landmarks whose head precedes it.  An empty
// landmark shares its offset with the next non-empty one, so the lower bound
// over lm_off already lands on a head.
__global__ void k_tiles(const int32_t* lm_off, const int32_t* rank, int32_t nl, int64_t N, int64_t ntiles,
                        int32_t* tile_start, int32_t* seg_base) {
    int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t > ntiles) return;
    if (t == ntiles) {
        tile_start[t] = int32_t(N);
        return;
    }
    const int64_t target = t * kWave;
    int32_t lo = 0, hi = nl;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (int64_t(lm_off[mid]) < target) lo = mid + 1; else hi = mid;
    }
    tile_start[t] = lo >= nl ? int32_t(N) : lm_off[lo];
    seg_base[t] = rank[lo];
}

// Camera-major sort key of each observation: camera * R + landmark range.
__global__ void k_cam_keys(const int32_t* obs_cam, const int32_t* obs_lm, const int32_t* rank, int64_t N,
                           int32_t R, int32_t seg_per_range, int32_t* keys) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= N) return;
    keys[i] = obs_cam[i] * R + rank[obs_lm[i]] / seg_per_range;
}

__global__ void k_piece_counts(const int32_t* grp_off, int32_t ngrp, int32_t piece, int32_t* counts) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g > ngrp) return;
    if (g == ngrp) {
        counts[g] = 0;
        return;
    }
    const int32_t len = grp_off[g + 1] - grp_off[g];
    counts[g] = (len + piece - 1) / piece;
}

__global__ void k_piece_fill(const int32_t* grp_off, const int32_t* grp_piece, int32_t ngrp, int32_t R, int32_t piece,
                             int32_t* piece_cam, int32_t* piece_begin, int32_t* piece_end, int32_t* piece_grp) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ngrp) return;
    const int32_t a = grp_off[g], b = grp_off[g + 1];
    int32_t p = grp_piece[g];
    for (int32_t s = a; s < b; s += piece, ++p) {
        piece_cam[p] = g / R;
        piece_begin[p] = s;
        piece_end[p] = min(s + piece, b);
        piece_grp[p] = g;
    }
}

// First camera-major position of each (camera, die) group: camera c's
// observations in the ranges [g R / 8, (g + 1) R / 8), the ranges whose
// series passes run on die g (R a multiple of 8).
__global__ void k_die_group_off(const int32_t* grp_off, int32_t nc, int32_t R, int32_t* dgrp_off) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t n = int64_t(nc) * kXcds;
    if (i > n) return;
    dgrp_off[i] = i == n ? grp_off[int64_t(nc) * R] : grp_off[(i / kXcds) * R + (i % kXcds) * (R / kXcds)];
}

// cam_piece[c] = first piece of camera c (pieces are ordered by camera, range).
__global__ void k_cam_piece(const int32_t* grp_piece, int32_t nc, int32_t R, int32_t* cam_piece) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c > nc) return;
    cam_piece[c] = grp_piece[int64_t(c) * R];
}

// cam_off[c] = first camera-major position of camera c.
__global__ void k_cam_off(const int32_t* grp_off, int32_t nc, int32_t R, int32_t* cam_off) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c > nc) return;
    cam_off[c] = grp_off[int64_t(c) * R];
}

__global__ void k_init_ctrl(Ctrl* ctrl, PCtrl* pctl, int32_t np) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j == 0) {
        ctrl->active = 0;
        ctrl->lin = 0;
        ctrl->running = 0;
        ctrl->pad = 0;
    }
    if (j < np) {
        PCtrl& q = pctl[j];
        q.lambda = q.cost = q.cost_new = q.model = q.norm_x2 = q.norm_v2 = 0.0;
        q.active = q.stopped = q.stop_order = q.status = q.accepted = q.pad = 0;
    }
}

__global__ void k_zero_f64(double* p, int64_t n) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

__global__ void k_project(int64_t N, const int32_t* obs_cam, const int32_t* obs_lm, const double* cams,
                          const double* lms, double* out) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double cam[9], X[3], px[2];
    const int32_t c = obs_cam[i], l = obs_lm[i];
    for (int k = 0; k < 9; ++k) cam[k] = cams[9 * int64_t(c) + k];
    for (int k = 0; k < 3; ++k) X[k] = lms[3 * int64_t(l) + k];
    project_point(cam, X, px);
    out[2 * i] = px[0];
    out[2 * i + 1] = px[1];
}

static unsigned grid_for(int64_t n, int block = kBlock) { return unsigned(std::max<int64_t>(ceil_div(n, block), 1)); }

static int key_bits(int32_t n) {
    int b = 1;
    while ((int64_t(1) << b) < int64_t(n)) ++b;
    return b;
}

// ------------------------------------------------- library-held workspace --
//
// The workspace of poba_create_static: one array per GPU, held from the load
// of the library until the process ends.  In host code the array's name is
// a stand-in, not a device address: host code takes the address on each
// device from hipGetSymbolAddress and passes only that to kernels and copies.
constexpr size_t kStaticWorkspaceBytes = POBA_STATIC_WORKSPACE_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticWorkspaceBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the array on the current device (looked up once per device).
static poba_status static_workspace(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return POBA_ERR_HIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return POBA_ERR_HIP;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return POBA_OK;
}

// Scratch bytes that set-up's radix sorts and scans need for these sizes
// (size queries only, nothing runs): both sorts at the widest key, the scans
// at their longest input.
static bool sort_tmp_exact(const Sizes& z, size_t* bytes) {
    const int n = int(std::max<int64_t>(z.N, 1));
    size_t sort = 0, scan = 0;
    hipcub::DoubleBuffer<int32_t> kb(nullptr, nullptr), vb(nullptr, nullptr);
    if (hipcub::DeviceRadixSort::SortPairs(nullptr, sort, kb, vb, n, 0, 31, hipStream_t(0)) != hipSuccess)
        return false;
    const int64_t scan_n = std::max<int64_t>(int64_t(z.nl) + 1, int64_t(z.nc) * z.ranges_max + 1);
    if (scan_n >= (int64_t(1) << 31)) return false;
    if (hipcub::DeviceScan::ExclusiveSum(nullptr, scan, static_cast<int32_t*>(nullptr),
                                         static_cast<int32_t*>(nullptr), int(scan_n), hipStream_t(0)) != hipSuccess)
        return false;
    *bytes = std::max(sort, scan) + 256;
    return true;
}

// ------------------------------------------------------------------ profiling --

void prof_begin(Problem* p, int cls, hipStream_t s, ProfileSlot** slot) {
    *slot = nullptr;
    if (!p || !p->profiling) return;
    if (p->slot_used >= p->slots.size()) return;
    ProfileSlot* sl = &p->slots[p->slot_used++];
    sl->cls = cls;
    (void)hipEventRecord(sl->start, s);
    *slot = sl;
}

void prof_end(ProfileSlot* slot, hipStream_t s) {
    if (slot) (void)hipEventRecord(slot->stop, s);
}

}  // namespace poba

using namespace poba;

extern "C" {

int32_t poba_version(void) { return 10000; }

const char* poba_status_string(poba_status s) {
    if (s == POBA_OK) return "ok";
    if (s & POBA_ERR_INVALID_ARG) return "invalid argument";
    if (s & POBA_ERR_INDEX_RANGE) return "observation index out of range";
    if (s & POBA_ERR_NOT_SPD) return "damped block not positive definite";
    if (s & POBA_ERR_NONFINITE) return "non-finite value";
    if (s & POBA_ERR_HIP) return "HIP runtime error";
    if (s & POBA_ERR_WORKSPACE) return "workspace missing or too small";
    if (s & POBA_ERR_STATE) return "invalid state";
    return "unknown status";
}

void poba_lm_default_options(poba_lm_options* o) {
    if (!o) return;
    o->lambda0 = 1e-4;
    o->func_tol = 1e-6;
    o->eps = 0.01;
    o->eta = 1e-3;
    o->lambda_min = 1e-16;
    o->lambda_max = 1e16;
    o->m = 20;
    o->max_iters = 50;
}

size_t poba_batch_workspace_bytes(const poba_desc* d, int32_t n_problems) {
    Sizes z;
    if (!compute_sizes(d, n_problems, &z)) return 0;
    return layout(d, z, nullptr, nullptr, sort_tmp_upper_bound(z.N));
}

size_t poba_workspace_bytes(const poba_desc* d) { return poba_batch_workspace_bytes(d, 1); }

poba_status poba_create(const poba_desc* d, const int32_t* obs_cam, const int32_t* obs_lm, const double* obs_xy,
                        void* workspace, size_t workspace_bytes, poba_stream stream, poba_problem* out) {
    if (!d) return POBA_ERR_INVALID_ARG;
    const int32_t cam_off[2] = {0, d->n_cams}, lm_off[2] = {0, d->n_lms};
    return poba_batch_create(d, 1, cam_off, lm_off, obs_cam, obs_lm, obs_xy, workspace, workspace_bytes, stream, out);
}

// Set-up of poba_batch_create and poba_create_static over a workspace whose
// layout reserves sort_tmp_bytes for the radix sorts and scans.
static poba_status create_impl(const poba_desc* d, int32_t n_problems, const int32_t* prob_cam_off,
                               const int32_t* prob_lm_off, const int32_t* obs_cam, const int32_t* obs_lm,
                               const double* obs_xy, void* workspace, size_t workspace_bytes, size_t sort_tmp_bytes,
                               hipStream_t s, poba_problem* out) {
    (void)hipGetLastError();  // report only this call's launch errors
    if (!out) return POBA_ERR_INVALID_ARG;
    *out = nullptr;
    Sizes z;
    if (!compute_sizes(d, n_problems, &z)) return POBA_ERR_INVALID_ARG;
    if (z.N > 0 && (!obs_cam || !obs_lm || !obs_xy)) return POBA_ERR_INVALID_ARG;
    if (!prob_cam_off || !prob_lm_off) return POBA_ERR_INVALID_ARG;
    if (prob_cam_off[0] != 0 || prob_lm_off[0] != 0 || prob_cam_off[n_problems] != z.nc ||
        prob_lm_off[n_problems] != z.nl)
        return POBA_ERR_INVALID_ARG;
    for (int32_t j = 0; j < n_problems; ++j)
        if (prob_cam_off[j + 1] <= prob_cam_off[j] || prob_lm_off[j + 1] <= prob_lm_off[j]) return POBA_ERR_INVALID_ARG;
    const size_t need = layout(d, z, nullptr, nullptr, sort_tmp_bytes);
    if (!workspace || workspace_bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 255u))
        return POBA_ERR_WORKSPACE;

    Problem* p = new Problem();
    p->d = *d;
    p->z = z;
    layout(d, z, reinterpret_cast<char*>(workspace), &p->b, sort_tmp_bytes);
    Buffers& b = p->b;
    const int64_t N = z.N;
    poba_status st = POBA_OK;

    auto fail = [&](poba_status e) {
        delete p;
        return e;
    };

    {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            p->n_cus = cus;
        int lds = 0;
        if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && lds > 0)
            p->lds_max = lds;
    }
    hipLaunchKernelGGL(k_init_ctrl, dim3(grid_for(z.np)), dim3(kBlock), 0, s, b.ctrl, b.pctl, z.np);
    const size_t np1 = size_t(z.np) + 1;
    if (hipMemcpyAsync(b.prob_cam_off, prob_cam_off, np1 * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(b.prob_lm_off, prob_lm_off, np1 * 4, hipMemcpyHostToDevice, s) != hipSuccess)
        return fail(POBA_ERR_HIP);
    hipLaunchKernelGGL(k_fill_prob, dim3(grid_for(z.nc)), dim3(kBlock), 0, s, b.prob_cam_off, z.np, z.nc, b.cam_prob);
    hipLaunchKernelGGL(k_fill_prob, dim3(grid_for(z.nl)), dim3(kBlock), 0, s, b.prob_lm_off, z.np, z.nl, b.lm_prob);
    int32_t* err = b.scratch_i;  // reuse scratch for the error flag, cleared below
    if (hipMemsetAsync(err, 0, sizeof(int32_t), s) != hipSuccess) return fail(POBA_ERR_HIP);
    if (N > 0) {
        hipLaunchKernelGGL(k_check_indices, dim3(grid_for(N)), dim3(kBlock), 0, s, obs_cam, obs_lm, N, z.nc, z.nl,
                           b.cam_prob, b.lm_prob, err, b.iota);
    }
    int32_t herr = 0;
    if (hipMemcpyAsync(&herr, err, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess) return fail(POBA_ERR_HIP);
    if (hipStreamSynchronize(s) != hipSuccess) return fail(POBA_ERR_HIP);
    if (herr) return fail(POBA_ERR_INDEX_RANGE);  // out of range, or across problems

    if (N > 0) {
        // landmark-major: stable radix sort by landmark
        size_t tmp = 0;
        hipcub::DoubleBuffer<int32_t> kb(b.keys_out, b.keys_tmp), vb(b.perm_l, b.vals_tmp);
        if (hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, kb, vb, int(N), 0, key_bits(z.nl), s) != hipSuccess)
            return fail(POBA_ERR_HIP);
        if (tmp > b.sort_tmp_bytes) return fail(POBA_ERR_WORKSPACE);
        if (hipMemcpyAsync(b.keys_out, obs_lm, N * 4, hipMemcpyDeviceToDevice, s) != hipSuccess) return fail(POBA_ERR_HIP);
        if (hipMemcpyAsync(b.perm_l, b.iota, N * 4, hipMemcpyDeviceToDevice, s) != hipSuccess) return fail(POBA_ERR_HIP);
        tmp = b.sort_tmp_bytes;
        if (hipcub::DeviceRadixSort::SortPairs(b.sort_tmp, tmp, kb, vb, int(N), 0, key_bits(z.nl), s) != hipSuccess)
            return fail(POBA_ERR_HIP);
        if (kb.Current() != b.keys_out)
            if (hipMemcpyAsync(b.keys_out, kb.Current(), N * 4, hipMemcpyDeviceToDevice, s) != hipSuccess) return fail(POBA_ERR_HIP);
        if (vb.Current() != b.perm_l)
            if (hipMemcpyAsync(b.perm_l, vb.Current(), N * 4, hipMemcpyDeviceToDevice, s) != hipSuccess) return fail(POBA_ERR_HIP);
        hipLaunchKernelGGL(k_segment_offsets, dim3(grid_for(N + 1)), dim3(kBlock), 0, s, b.keys_out, N, z.nl, b.lm_off);
        // sorted landmark keys (head and tail flags) wait in co_lm until the gather
        if (hipMemcpyAsync(b.co_lm, b.keys_out, N * 4, hipMemcpyDeviceToDevice, s) != hipSuccess) return fail(POBA_ERR_HIP);
    } else {
        hipLaunchKernelGGL(k_segment_offsets, dim3(1), dim3(kBlock), 0, s, b.keys_out, int64_t(0), z.nl, b.lm_off);
    }

    // non-empty landmark list (segments) and landmark tiles
    const int64_t half = std::max<int64_t>(z.nc, z.nl) + 2;
    int32_t* rank = b.scratch_i + half;
    {
        int32_t* flags = b.scratch_i;
        hipLaunchKernelGGL(k_nonempty_flags, dim3(grid_for(z.nl)), dim3(kBlock), 0, s, b.lm_off, z.nl, flags);
        if (hipMemsetAsync(flags + z.nl, 0, 4, s) != hipSuccess) return fail(POBA_ERR_HIP);
        size_t tmp = 0;
        if (hipcub::DeviceScan::ExclusiveSum(nullptr, tmp, flags, rank, z.nl + 1, s) != hipSuccess) return fail(POBA_ERR_HIP);
        if (tmp > b.sort_tmp_bytes) return fail(POBA_ERR_WORKSPACE);
        tmp = b.sort_tmp_bytes;
        if (hipcub::DeviceScan::ExclusiveSum(b.sort_tmp, tmp, flags, rank, z.nl + 1, s) != hipSuccess) return fail(POBA_ERR_HIP);
        hipLaunchKernelGGL(k_compact_nonempty, dim3(grid_for(z.nl)), dim3(kBlock), 0, s, b.lm_off, rank, z.nl, b.nel);
        hipLaunchKernelGGL(k_tiles, dim3(grid_for(z.ntiles + 1)), dim3(kBlock), 0, s, b.lm_off, rank, z.nl, N, z.ntiles,
                           b.tile_start, b.seg_base);
        int32_t nnel = 0;
        if (hipMemcpyAsync(&nnel, rank + z.nl, 4, hipMemcpyDeviceToHost, s) != hipSuccess) return fail(POBA_ERR_HIP);
        if (hipStreamSynchronize(s) != hipSuccess) return fail(POBA_ERR_HIP);
        p->nnel = nnel;
    }

    // landmark ranges of the camera-major order: each die of the GPU gathers
    // the landmark vector from one slice small enough for its L2
    // (point records: slices that the camera pass stages in LDS)
    int32_t R = d->lm_ranges;
    if (R == 0) {
        if (z.point) {
            R = point_ranges(p->nnel, z.sbytes);
        } else {
            const int64_t s_bytes = p->nnel * (d->precision == POBA_F64 ? 32 : 16);
            R = s_bytes > kRangeBytes ? int32_t(kXcds * ceil_div(s_bytes, kXcds * kRangeBytes)) : 1;
        }
    }
    if (R > z.ranges_max) return fail(POBA_ERR_STATE);
    p->lm_ranges = R;
    const int32_t spr = int32_t(std::max<int64_t>(1, ceil_div(std::max<int64_t>(p->nnel, 1), R)));
    const int64_t ngrp = int64_t(z.nc) * R;
    p->seg_per_range = spr;
    p->range_lds_ok = z.point && N > 0 &&
                      int64_t(spr) * 3 * z.sbytes <= std::min<int64_t>(kRangeLdsMax, p->lds_max) ? 1 : 0;
    p->range_lds = p->range_lds_ok;

    if (N > 0) {
        // camera-major: stable radix sort by (camera, landmark range)
        hipLaunchKernelGGL(k_cam_keys, dim3(grid_for(N)), dim3(kBlock), 0, s, obs_cam, obs_lm, rank, N, R, spr,
                           b.keys_out);
        size_t tmp2 = 0;
        const int bits = key_bits(int32_t(std::min<int64_t>(ngrp, int64_t(1) << 30)));
        hipcub::DoubleBuffer<int32_t> kc(b.keys_out, b.keys_tmp), vc(b.perm_c, b.vals_tmp);
        if (hipcub::DeviceRadixSort::SortPairs(nullptr, tmp2, kc, vc, int(N), 0, bits, s) != hipSuccess)
            return fail(POBA_ERR_HIP);
        if (tmp2 > b.sort_tmp_bytes) return fail(POBA_ERR_WORKSPACE);
        if (hipMemcpyAsync(b.perm_c, b.iota, N * 4, hipMemcpyDeviceToDevice, s) != hipSuccess) return fail(POBA_ERR_HIP);
        tmp2 = b.sort_tmp_bytes;
        if (hipcub::DeviceRadixSort::SortPairs(b.sort_tmp, tmp2, kc, vc, int(N), 0, bits, s) != hipSuccess)
            return fail(POBA_ERR_HIP);
        if (kc.Current() != b.keys_out)
            if (hipMemcpyAsync(b.keys_out, kc.Current(), N * 4, hipMemcpyDeviceToDevice, s) != hipSuccess) return fail(POBA_ERR_HIP);
        if (vc.Current() != b.perm_c)
            if (hipMemcpyAsync(b.perm_c, vc.Current(), N * 4, hipMemcpyDeviceToDevice, s) != hipSuccess) return fail(POBA_ERR_HIP);
        hipLaunchKernelGGL(k_segment_offsets, dim3(grid_for(N + 1)), dim3(kBlock), 0, s, b.keys_out, N, int32_t(ngrp),
                           b.grp_off);
        if (hipMemcpyAsync(b.keys_tmp, b.co_lm, N * 4, hipMemcpyDeviceToDevice, s) != hipSuccess) return fail(POBA_ERR_HIP);
        hipLaunchKernelGGL(k_gather_orders, dim3(grid_for(N)), dim3(kBlock), 0, s, b.perm_l, b.perm_c, obs_cam, obs_lm,
                           obs_xy, b.lm_off, b.keys_tmp, rank, N, b.lo_cam, b.co_lm, b.co_seg, b.obs_lo, b.obs_co);
    } else {
        hipLaunchKernelGGL(k_segment_offsets, dim3(grid_for(ngrp + 1)), dim3(kBlock), 0, s, b.keys_out, int64_t(0),
                           int32_t(ngrp), b.grp_off);
    }
    hipLaunchKernelGGL(k_cam_off, dim3(grid_for(z.nc + 1)), dim3(kBlock), 0, s, b.grp_off, z.nc, R, b.cam_off);

    // camera pieces: at most `piece` observations of one (camera, range)
    // group; with range-staged camera passes (the series passes then walk the
    // groups themselves) of one camera and the ranges of one die, so that the
    // per-piece kernels keep larger pieces and their landmark gathers stay
    // within the die's eighth of the landmarks (or of one camera where R is
    // not a multiple of 8)
    const bool die_groups = p->range_lds_ok && R % kXcds == 0;
    const int32_t Rp = p->range_lds_ok ? (die_groups ? kXcds : 1) : R;
    if (die_groups)
        hipLaunchKernelGGL(k_die_group_off, dim3(grid_for(int64_t(z.nc) * kXcds + 1)), dim3(kBlock), 0, s, b.grp_off,
                           z.nc, R, b.dgrp_off);
    {
        const int32_t* goff = p->range_lds_ok ? (die_groups ? b.dgrp_off : b.cam_off) : b.grp_off;
        const int64_t ngp = int64_t(z.nc) * Rp;
        int32_t* counts = b.sched;  // scratch until the schedule is written
        hipLaunchKernelGGL(k_piece_counts, dim3(grid_for(ngp + 1)), dim3(kBlock), 0, s, goff, int32_t(ngp), z.piece,
                           counts);
        size_t tmp = 0;
        if (hipcub::DeviceScan::ExclusiveSum(nullptr, tmp, counts, b.grp_piece, int(ngp + 1), s) != hipSuccess)
            return fail(POBA_ERR_HIP);
        if (tmp > b.sort_tmp_bytes) return fail(POBA_ERR_WORKSPACE);
        tmp = b.sort_tmp_bytes;
        if (hipcub::DeviceScan::ExclusiveSum(b.sort_tmp, tmp, counts, b.grp_piece, int(ngp + 1), s) != hipSuccess)
            return fail(POBA_ERR_HIP);
        hipLaunchKernelGGL(k_piece_fill, dim3(grid_for(ngp)), dim3(kBlock), 0, s, goff, b.grp_piece, int32_t(ngp), Rp,
                           z.piece, b.piece_cam, b.piece_begin, b.piece_end, b.piece_grp);
        hipLaunchKernelGGL(k_cam_piece, dim3(grid_for(z.nc + 1)), dim3(kBlock), 0, s, b.grp_piece, z.nc, Rp,
                           b.cam_piece);
        hipLaunchKernelGGL(k_prob_pieces, dim3(grid_for(z.np + 1)), dim3(kBlock), 0, s, b.prob_cam_off, b.cam_piece,
                           z.np, b.prob_piece_off);
        int32_t np = 0;
        if (hipMemcpyAsync(&np, b.grp_piece + ngp, 4, hipMemcpyDeviceToHost, s) != hipSuccess) return fail(POBA_ERR_HIP);
        if (hipStreamSynchronize(s) != hipSuccess) return fail(POBA_ERR_HIP);
        if (np > z.npieces_max) return fail(POBA_ERR_STATE);
        p->npieces = np;
    }
    // camera-pass schedule: workgroups are dealt to the dies in turn, so block
    // b runs on die b % 8; with ranges it takes a piece of a range r with
    // r % 8 == b % 8, otherwise piece b
    {
        std::vector<int32_t> sched;
        if (Rp > 1 && p->npieces > 0) {
            std::vector<int32_t> pgrp(size_t(p->npieces));
            if (hipMemcpyAsync(pgrp.data(), b.piece_grp, pgrp.size() * 4, hipMemcpyDeviceToHost, s) != hipSuccess)
                return fail(POBA_ERR_HIP);
            if (hipStreamSynchronize(s) != hipSuccess) return fail(POBA_ERR_HIP);
            std::vector<std::vector<int32_t>> lists(kXcds);
            for (int32_t q = 0; q < int32_t(pgrp.size()); ++q) lists[(pgrp[q] % Rp) % kXcds].push_back(q);
            size_t maxlen = 0;
            for (auto& l : lists) maxlen = std::max(maxlen, l.size());
            sched.assign(maxlen * kXcds, -1);
            for (int x = 0; x < kXcds; ++x)
                for (size_t j = 0; j < lists[x].size(); ++j) sched[j * kXcds + x] = lists[x][j];
        } else {
            sched.resize(size_t(p->npieces));
            for (int32_t q = 0; q < int32_t(sched.size()); ++q) sched[q] = q;
        }
        if (int64_t(sched.size()) > int64_t(kXcds) * z.npieces_max) return fail(POBA_ERR_STATE);
        p->sched_len = int64_t(sched.size());
        if (sched.empty()) sched.push_back(-1);  // a one-block launch over no piece stays idle
        if (!sched.empty() &&
            hipMemcpyAsync(b.sched, sched.data(), sched.size() * 4, hipMemcpyHostToDevice, s) != hipSuccess)
            return fail(POBA_ERR_HIP);
        hipLaunchKernelGGL(k_sched_rec, dim3(grid_for(int64_t(sched.size()))), dim3(kBlock), 0, s, b.sched,
                           b.piece_begin, b.piece_end, b.piece_cam, b.cam_prob, int64_t(sched.size()), b.sched_rec);
        if (hipStreamSynchronize(s) != hipSuccess) return fail(POBA_ERR_HIP);
    }
    // range-staged camera pass: G workgroups per landmark range (one per
    // compute unit in all), each with range_pass_waves wavefronts.  A range's
    // non-empty (camera, range) groups are sorted longest first and dealt to
    // its G workgroups in turn; each workgroup cuts its share, in that order,
    // into batches of kSets groups (a batch takes as many steps as its first,
    // longest group needs) and gives each batch to the wavefront with the
    // fewest steps so far (longest processing time first), so its wavefronts
    // end close together.  A wavefront's list is its batches in the order it
    // got them; only the workgroup's last batch can hold fewer than kSets
    // groups, and it is the last of its wavefront's list.  Neighbouring
    // ranges run on the same die (workgroups are dealt to the dies in turn),
    // so the cache lines that two adjacent groups of one camera share, and
    // the staged slices, are fetched into one L2.  Group sums of empty groups
    // stay zero.
    if (p->range_lds_ok) {
        std::vector<int32_t> go(size_t(ngrp) + 1);
        std::vector<int32_t> cprob(size_t(z.nc));
        if (hipMemcpyAsync(go.data(), b.grp_off, go.size() * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(cprob.data(), b.cam_prob, cprob.size() * 4, hipMemcpyDeviceToHost, s) != hipSuccess)
            return fail(POBA_ERR_HIP);
        if (hipStreamSynchronize(s) != hipSuccess) return fail(POBA_ERR_HIP);
        const int waves = range_pass_waves(z.sbytes);
        int64_t G = std::max<int64_t>(1, (p->n_cus + R / 2) / R);
        G = std::min<int64_t>(G, kMaxRangeBlocks);
        G = std::min<int64_t>(G, std::max<int64_t>(1, N / (int64_t(R) * waves * 256)));
        const int64_t nblk = int64_t(R) * G;
        const int64_t per_die = R % kXcds == 0 ? R / kXcds : 0;  // consecutive ranges per die
        std::vector<int4> rec(size_t(nblk) * waves);
        std::vector<int4> list;
        list.reserve(size_t(ngrp));
        std::vector<std::pair<int32_t, int32_t>> grp;  // (length, camera) of the range's non-empty groups
        std::vector<std::vector<int32_t>> mine(static_cast<size_t>(waves));  // per wavefront: its groups (indices into grp)
        std::vector<int64_t> load(static_cast<size_t>(waves));
        for (int32_t r = 0; r < R; ++r) {
            grp.clear();
            for (int32_t c = 0; c < z.nc; ++c) {
                const int32_t len = go[size_t(c) * R + r + 1] - go[size_t(c) * R + r];
                if (len > 0) grp.emplace_back(len, c);
            }
            std::stable_sort(grp.begin(), grp.end(),
                             [](const std::pair<int32_t, int32_t>& x, const std::pair<int32_t, int32_t>& y) {
                                 return x.first > y.first;
                             });
            for (int64_t j = 0; j < G; ++j) {
                // the workgroup's share: groups j, j + G, j + 2G, ... of the sorted list
                for (auto& m : mine) m.clear();
                std::fill(load.begin(), load.end(), 0);
                for (size_t q0 = size_t(j); q0 < grp.size(); q0 += size_t(G) * kSets) {
                    const int64_t steps = (grp[q0].first + kSetLanes - 1) / kSetLanes;
                    const size_t w = size_t(std::min_element(load.begin(), load.end()) - load.begin());
                    load[w] += steps;
                    for (int k = 0; k < kSets; ++k) {
                        const size_t q = q0 + size_t(k) * size_t(G);
                        if (q < grp.size()) mine[w].push_back(int32_t(q));
                    }
                }
                const int64_t blk = per_die ? ((r % per_die) * G + j) * kXcds + r / per_die : int64_t(r) * G + j;
                for (int w = 0; w < waves; ++w) {
                    const int32_t begin = int32_t(list.size());
                    for (const int32_t q : mine[size_t(w)]) {
                        const int32_t c = grp[size_t(q)].second;
                        list.push_back(make_int4(c, go[size_t(c) * R + r], grp[size_t(q)].first, cprob[size_t(c)]));
                    }
                    rec[size_t(blk) * waves + size_t(w)] = make_int4(r, begin, int32_t(list.size()), 0);
                }
            }
        }
        if (int64_t(list.size()) > ngrp) return fail(POBA_ERR_STATE);
        if (hipMemcpyAsync(b.cw_rec, rec.data(), rec.size() * sizeof(int4), hipMemcpyHostToDevice, s) != hipSuccess)
            return fail(POBA_ERR_HIP);
        if (!list.empty() &&
            hipMemcpyAsync(b.cw_list, list.data(), list.size() * sizeof(int4), hipMemcpyHostToDevice, s) != hipSuccess)
            return fail(POBA_ERR_HIP);
        if (hipMemsetAsync(b.part_grp, 0, size_t(ngrp) * 9 * size_t(z.sbytes), s) != hipSuccess)
            return fail(POBA_ERR_HIP);
        if (hipStreamSynchronize(s) != hipSuccess) return fail(POBA_ERR_HIP);
        p->cw_blocks = nblk;
    }
    // blocks of landmarks without observations are never written by a pass
    hipLaunchKernelGGL(k_zero_f64, dim3(grid_for(int64_t(z.nl) * 6)), dim3(kBlock), 0, s, b.V, int64_t(z.nl) * 6);
    hipLaunchKernelGGL(k_zero_f64, dim3(grid_for(int64_t(z.nl) * 3)), dim3(kBlock), 0, s, b.bl, int64_t(z.nl) * 3);
    hipLaunchKernelGGL(k_zero_f64, dim3(grid_for(int64_t(z.nl) * 4)), dim3(kBlock), 0, s, (double*)b.s, int64_t(z.nl) * 4);
    // camera vectors of cameras without observations stay zero
    hipLaunchKernelGGL(k_zero_f64, dim3(grid_for(int64_t(z.nc) * 9)), dim3(kBlock), 0, s, b.x, int64_t(z.nc) * 9);
    hipLaunchKernelGGL(k_zero_f64, dim3(grid_for(int64_t(z.nc) * 9)), dim3(kBlock), 0, s, b.Dp, int64_t(z.nc) * 9);
    hipLaunchKernelGGL(k_zero_f64, dim3(grid_for(int64_t(z.nl) * 3)), dim3(kBlock), 0, s, b.Dl, int64_t(z.nl) * 3);
    hipLaunchKernelGGL(k_zero_f64, dim3(grid_for(int64_t(z.nc) * 9)), dim3(kBlock), 0, s, b.v, int64_t(z.nc) * 9);
    hipLaunchKernelGGL(k_zero_f64, dim3(grid_for(int64_t(z.nc) * 12)), dim3(kBlock), 0, s, (double*)b.vq, int64_t(z.nc) * 12);

    if (hipStreamSynchronize(s) != hipSuccess) return fail(POBA_ERR_HIP);
    if (hipGetLastError() != hipSuccess) return fail(POBA_ERR_HIP);
    *out = p;
    return st;
}

poba_status poba_batch_create(const poba_desc* d, int32_t n_problems, const int32_t* prob_cam_off,
                              const int32_t* prob_lm_off, const int32_t* obs_cam, const int32_t* obs_lm,
                              const double* obs_xy, void* workspace, size_t workspace_bytes, poba_stream stream,
                              poba_problem* out) {
    Sizes z;
    if (!compute_sizes(d, n_problems, &z)) {
        if (out) *out = nullptr;
        return POBA_ERR_INVALID_ARG;
    }
    return create_impl(d, n_problems, prob_cam_off, prob_lm_off, obs_cam, obs_lm, obs_xy, workspace, workspace_bytes,
                       sort_tmp_upper_bound(z.N), reinterpret_cast<hipStream_t>(stream), out);
}

poba_status poba_create_static(const poba_desc* d, const int32_t* obs_cam, const int32_t* obs_lm,
                               const double* obs_xy, poba_stream stream, poba_problem* out) {
    (void)hipGetLastError();  // report only this call's launch errors
    if (!d || !out) return POBA_ERR_INVALID_ARG;
    *out = nullptr;
    Sizes z;
    if (!compute_sizes(d, 1, &z)) return POBA_ERR_INVALID_ARG;
    size_t tmp = 0;
    if (!sort_tmp_exact(z, &tmp)) return POBA_ERR_HIP;
    const size_t need = layout(d, z, nullptr, nullptr, tmp);
    if (need > kStaticWorkspaceBytes) return POBA_ERR_WORKSPACE;  // before any device work
    void* ws = nullptr;
    poba_status st = static_workspace(&ws);
    if (st) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // the array keeps the previous handle's contents: start from zero
    hipLaunchKernelGGL(k_zero_f64, dim3(grid_for(int64_t(need / 8))), dim3(kBlock), 0, s, static_cast<double*>(ws),
                       int64_t(need / 8));
    if (hipGetLastError() != hipSuccess) return POBA_ERR_HIP;
    const int32_t cam_off[2] = {0, d->n_cams}, lm_off[2] = {0, d->n_lms};
    return create_impl(d, 1, cam_off, lm_off, obs_cam, obs_lm, obs_xy, ws, kStaticWorkspaceBytes, tmp, s, out);
}

poba_status poba_destroy(poba_problem p) {
    if (!p) return POBA_ERR_INVALID_ARG;
    for (auto& sl : p->slots) {
        hipEventDestroy(sl.start);
        hipEventDestroy(sl.stop);
    }
    delete p;
    return POBA_OK;
}

poba_status poba_project(int64_t n_obs, const int32_t* obs_cam, const int32_t* obs_lm, const double* cams,
                         const double* lms, double* out_xy, poba_stream stream) {
    (void)hipGetLastError();  // report only this call's launch errors
    if (n_obs < 0) return POBA_ERR_INVALID_ARG;
    if (n_obs == 0) return POBA_OK;
    if (!obs_cam || !obs_lm || !cams || !lms || !out_xy) return POBA_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_project, dim3(grid_for(n_obs)), dim3(kBlock), 0, reinterpret_cast<hipStream_t>(stream), n_obs,
                       obs_cam, obs_lm, cams, lms, out_xy);
    return hipGetLastError() == hipSuccess ? POBA_OK : POBA_ERR_HIP;
}

poba_status poba_get_orders(poba_problem p, int32_t* perm_lm, int32_t* perm_cam, int32_t* lm_off, int32_t* cam_off,
                            poba_stream stream) {
    if (!p) return POBA_ERR_INVALID_ARG;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const Buffers& b = p->b;
    const int64_t N = p->z.N;
    if (perm_lm && N && hipMemcpyAsync(perm_lm, b.perm_l, N * 4, hipMemcpyDeviceToDevice, s) != hipSuccess) return POBA_ERR_HIP;
    if (perm_cam && N && hipMemcpyAsync(perm_cam, b.perm_c, N * 4, hipMemcpyDeviceToDevice, s) != hipSuccess) return POBA_ERR_HIP;
    if (lm_off && hipMemcpyAsync(lm_off, b.lm_off, (p->z.nl + 1) * 4, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return POBA_ERR_HIP;
    if (cam_off && hipMemcpyAsync(cam_off, b.cam_off, (p->z.nc + 1) * 4, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return POBA_ERR_HIP;
    return POBA_OK;
}

poba_status poba_set_tuning(poba_problem p, int32_t key, int32_t value) {
    if (!p) return POBA_ERR_INVALID_ARG;
    switch (key) {
        case POBA_TUNE_TILES_PER_WAVE:
            if (value < 1 || value > 64) return POBA_ERR_INVALID_ARG;
            p->tiles_per_wave = value;
            return POBA_OK;
        case POBA_TUNE_LDS_CAMERA:
            if (value != 0 && value != 1) return POBA_ERR_INVALID_ARG;
            p->lds_cam = value;
            return POBA_OK;
        case POBA_TUNE_RANGE_LDS:
            if (value != 0 && value != 1) return POBA_ERR_INVALID_ARG;
            if (value == 1 && !p->range_lds_ok) return POBA_ERR_INVALID_ARG;
            p->range_lds = value;
            return POBA_OK;
        default: return POBA_ERR_INVALID_ARG;
    }
}

poba_status poba_get_tuning(poba_problem p, int32_t key, int32_t* value) {
    if (!p || !value) return POBA_ERR_INVALID_ARG;
    switch (key) {
        case POBA_TUNE_TILES_PER_WAVE: *value = p->tiles_per_wave; return POBA_OK;
        case POBA_TUNE_LM_RANGES: *value = p->lm_ranges; return POBA_OK;
        case POBA_TUNE_LDS_CAMERA: *value = p->lds_cam; return POBA_OK;
        case POBA_TUNE_RANGE_LDS: *value = p->range_lds; return POBA_OK;
        default: return POBA_ERR_INVALID_ARG;
    }
}

poba_status poba_profile_enable(poba_problem p, int32_t enable) {
    if (!p) return POBA_ERR_INVALID_ARG;
    if (enable && p->slots.empty()) {
        p->slots.resize(kMaxProfiled);
        for (auto& sl : p->slots) {
            if (hipEventCreate(&sl.start) != hipSuccess || hipEventCreate(&sl.stop) != hipSuccess) return POBA_ERR_HIP;
        }
    }
    p->profiling = enable != 0;
    return POBA_OK;
}

poba_status poba_profile_read(poba_problem p, double* ms, int64_t* n) {
    if (!p) return POBA_ERR_INVALID_ARG;
    for (size_t i = 0; i < p->slot_used; ++i) {
        ProfileSlot& sl = p->slots[i];
        if (hipEventSynchronize(sl.stop) != hipSuccess) return POBA_ERR_HIP;
        float t = 0.f;
        if (hipEventElapsedTime(&t, sl.start, sl.stop) != hipSuccess) return POBA_ERR_HIP;
        p->prof_ms[sl.cls] += t;
        p->prof_n[sl.cls] += 1;
    }
    p->slot_used = 0;
    for (int k = 0; k < POBA_K_COUNT; ++k) {
        if (ms) ms[k] = p->prof_ms[k];
        if (n) n[k] = p->prof_n[k];
        p->prof_ms[k] = 0.0;
        p->prof_n[k] = 0;
    }
    return POBA_OK;
}

}  // extern "C"
