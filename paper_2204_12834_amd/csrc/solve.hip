// The damped step of Sec. 4.2-4.3: block inverses, the reduced right-hand side
// b~ = b_p - W V^-1 b_l (eq. Schur), the power series
// x(m) = -sum_{i=0..m} (U^-1 W V^-1 W^T)^i U^-1 b~ (eqs. S_approx, x_approx)
// with the stop rule of eq. qcriterion, and the back-substitution
// dx_l = -V^-1 (b_l + W^T dx_p).
//
// One application of P = U^-1 W V^-1 W^T is two streaming passes over the
// Jacobian records (the paper counts it as four matrix-vector products,
// Fig. 2):
//   landmark pass (landmark-major):  t_l = sum_i J_l^T (J_p v_c),  s_l = V_l^-1 t_l
//   camera pass   (camera-major):    u_c = sum_i J_p^T (J_l s_l)   per piece
//   camera finish (per camera):      v_c = U_c^-1 u_c,  x_c += v_c,  norms
// Both passes are segmented reductions inside a wavefront or block; camera
// pieces are combined in a fixed order; no floating-point atomics are used.
#include <type_traits>
#include <utility>

#include "device_ops.hpp"
#include "kernels.hpp"

namespace poba {

__device__ __forceinline__ int64_t ceil_div_d(int64_t a, int64_t b) { return (a + b - 1) / b; }

enum FinMode { kFinRhs = 0, kFinSeries = 1, kFinApply = 2 };

// ---------------------------------------------------------------- control --

// Every problem active with damping lam; series flags cleared.
__global__ void k_begin_solve(Ctrl* ctrl, PCtrl* pctl, int32_t np, double lam) {
    for (int32_t j = threadIdx.x; j < np; j += blockDim.x) {
        PCtrl& q = pctl[j];
        q.lambda = lam;
        q.active = 1;
        q.stopped = 0;
        q.stop_order = 0;
        q.status = 0;
    }
    if (threadIdx.x == 0) {
        ctrl->active = np;
        ctrl->running = np;
    }
}

// ---------------------------------------------------------------- inverses --

// U_lambda^-1 per camera by a 9x9 Cholesky factorisation, in float64.  The
// damping diagonal is taken from U and kept in Dp, or, when `frozen`, read
// from Dp as an earlier solve left it.
__global__ __launch_bounds__(kBlock) void k_inv_cam(Buffers b, Sizes z, int damping, int frozen, const Ctrl* ctrl) {
    if (!ctrl->active) return;
    const int32_t c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= z.nc) return;
    PCtrl& q = b.pctl[b.cam_prob[c]];
    if (!q.active) return;
    const double lam = q.lambda;
    const double* U = b.U + 81 * int64_t(c);
    double L[81];
#pragma unroll
    for (int k = 0; k < 81; ++k) L[k] = U[k];
    double dg[9];
#pragma unroll
    for (int j = 0; j < 9; ++j) {
        double dj;
        if (frozen) {
            dj = b.Dp[9 * int64_t(c) + j];
        } else {
            dj = damp_diag(U[10 * j], damping);
            b.Dp[9 * int64_t(c) + j] = dj;
        }
        dg[j] = lam * dj;
        L[10 * j] += dg[j];
    }
    double* out = b.Uinv + 81 * int64_t(c);
    const bool ok = spd_inverse9(L, out);
    if (!ok) {
#pragma unroll
        for (int i = 0; i < 9; ++i)
#pragma unroll
            for (int j = 0; j < 9; ++j) out[9 * i + j] = (i == j && dg[i] > 0.0) ? 1.0 / dg[i] : 0.0;
        atomicOr(&q.status, POBA_ERR_NOT_SPD);
    }
}

// V_lambda^-1 of every non-empty landmark in float64, stored in the landmark
// storage type and in float64 at the landmark's segment index, and
// y = V_lambda^-1 b_l (first half of b~) into the float64 view of s and into
// ybl with a flag 1 (kept there for the back-substitution; flag 0 for the
// landmarks of inactive problems, whose step the back-substitution leaves).
// The damping diagonal goes to (or, when `frozen`, comes from) Dl at the same
// index.
template <typename TS>
__global__ __launch_bounds__(kBlock) void k_inv_lm(Buffers b, int32_t nseg, int damping, int frozen,
                                                   const Ctrl* ctrl) {
    if (!ctrl->active) return;
    const int32_t g = blockIdx.x * kBlock + threadIdx.x;
    if (g >= nseg) return;
    const int64_t l = b.nel[g];
    PCtrl& q = b.pctl[b.lm_prob[l]];
    if (!q.active) {
        b.ybl[4 * int64_t(g) + 3] = 0.0;
        return;
    }
    double Vd[6], inv[6], dd[3], bl[3], y[3];
#pragma unroll
    for (int k = 0; k < 6; ++k) Vd[k] = b.V[6 * l + k];
#pragma unroll
    for (int k = 0; k < 3; ++k) bl[k] = b.bl[3 * l + k];
    if (frozen) {
#pragma unroll
        for (int k = 0; k < 3; ++k) dd[k] = b.Dl[3 * int64_t(g) + k];
    } else {
        damp_diag3(Vd, damping, dd);
#pragma unroll
        for (int k = 0; k < 3; ++k) b.Dl[3 * int64_t(g) + k] = dd[k];
    }
    const bool ok = inv3_damped(Vd, q.lambda, dd, inv);
    TS* o = reinterpret_cast<TS*>(b.Vinv) + 6 * int64_t(g);
#pragma unroll
    for (int k = 0; k < 6; ++k) o[k] = TS(inv[k]);
    double2* o64 = reinterpret_cast<double2*>(b.vinv64 + 6 * int64_t(g));
    o64[0] = make_double2(inv[0], inv[1]);
    o64[1] = make_double2(inv[2], inv[3]);
    o64[2] = make_double2(inv[4], inv[5]);
    if (!ok) atomicOr(&q.status, POBA_ERR_NOT_SPD);
    sym3_apply(inv, bl, y);
    double2* so = reinterpret_cast<double2*>(reinterpret_cast<double*>(b.s) + 4 * int64_t(g));
    so[0] = make_double2(y[0], y[1]);
    so[1] = make_double2(y[2], 0.0);
    double2* yo = reinterpret_cast<double2*>(b.ybl + 4 * int64_t(g));
    yo[0] = make_double2(y[0], y[1]);
    yo[1] = make_double2(y[2], 1.0);
}

// ------------------------------------------------------------ landmark pass --

// Camera vector (stride 12, storage type) for one observation.
__device__ __forceinline__ void load_cam_vec(const float* vq, int64_t cam, float* x) {
    const float4* p = reinterpret_cast<const float4*>(vq + 12 * cam);
    const float4 a = p[0], b = p[1], c = p[2];
    x[0] = a.x; x[1] = a.y; x[2] = a.z; x[3] = a.w;
    x[4] = b.x; x[5] = b.y; x[6] = b.z; x[7] = b.w;
    x[8] = c.x;
}
__device__ __forceinline__ void load_cam_vec(const double* vq, int64_t cam, double* x) {
    const double2* p = reinterpret_cast<const double2*>(vq + 12 * cam);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double2 a = p[k];
        x[2 * k] = a.x;
        x[2 * k + 1] = a.y;
    }
    x[8] = vq[12 * cam + 8];
}

// Packed symmetric V^-1 of one landmark (6 entries, storage type).
__device__ __forceinline__ void load_vinv(const float* V, int64_t l, float* A) {
    const float2* p = reinterpret_cast<const float2*>(V + 6 * l);
    const float2 a = p[0], b = p[1], c = p[2];
    A[0] = a.x; A[1] = a.y; A[2] = b.x; A[3] = b.y; A[4] = c.x; A[5] = c.y;
}
__device__ __forceinline__ void load_vinv(const double* V, int64_t l, double* A) {
    const double2* p = reinterpret_cast<const double2*>(V + 6 * l);
    const double2 a = p[0], b = p[1], c = p[2];
    A[0] = a.x; A[1] = a.y; A[2] = b.x; A[3] = b.y; A[4] = c.x; A[5] = c.y;
}

__device__ __forceinline__ void store_s(float* s, int64_t l, const float* y) {
    reinterpret_cast<float4*>(s)[l] = make_float4(y[0], y[1], y[2], 0.f);
}
__device__ __forceinline__ void store_s(double* s, int64_t l, const double* y) {
    double2* p = reinterpret_cast<double2*>(s + 4 * l);
    p[0] = make_double2(y[0], y[1]);
    p[1] = make_double2(y[2], 0.0);
}

// Landmark pass: s_g = V_g^-1 sum_{i in g} J_l^T (J_p v_c(i)) for every
// non-empty landmark (segment g).  One wavefront walks `tpw` consecutive
// 64-tiles as one range, in chunks of 64 positions, as a two-stage pipeline:
// while chunk k is reduced, the records of chunk k+1 are in flight, and the
// gathers of chunk k+1 (camera vector per observation, V^-1 per landmark end)
// are issued after them, so no wait ever covers a younger load.
// TJ: record storage, TC: arithmetic, TS: landmark storage and camera copy.
template <typename TJ, typename TC, typename TS, bool LDS_CAM, typename Tail>
__device__ __forceinline__ void lm_pass_range(const Buffers& b, const Sizes& z, int64_t t0, int64_t t1,
                                              const TS* __restrict__ vq, const Tail& tail);

// What the landmark stream does at a segment's tail lane.  The series:
// s_g = V_g^-1 t_g in the storage type, with V^-1 requested a chunk ahead.
template <typename TS, typename TC>
struct SeriesTail {
    const TS* __restrict__ Vinv;
    TS* __restrict__ sout;
    struct Slot {
        TS A[6];
    };
    __device__ __forceinline__ static bool skip(const Ctrl* ctrl) { return ctrl->running == 0; }
    __device__ __forceinline__ void fetch(int32_t seg, Slot& o) const { load_vinv(Vinv, seg, o.A); }
    __device__ __forceinline__ void finish(int32_t seg, const Slot& o, const TC* v) const {
        TC Ac[6], y[3];
#pragma unroll
        for (int k = 0; k < 6; ++k) Ac[k] = TC(o.A[k]);
        sym3_apply(Ac, v, y);
        TS ys[3] = {TS(y[0]), TS(y[1]), TS(y[2])};
        store_s(sout, seg, ys);
    }
};

// The back-substitution (Sec. 4.2, eq. back_substitution, reading R9):
// dx_l = -(V^-1 b_l + V^-1 t) for the landmark l = nel[g] of segment g, with
// V^-1 and V^-1 b_l in float64 from the solve's preparation (a flag 0 there
// marks a landmark of an inactive problem, whose step is left as it was).
struct BacksubTail {
    const int32_t* __restrict__ nel;
    const double* __restrict__ vinv64;
    const double* __restrict__ ybl;
    double* __restrict__ dxl;
    struct Slot {
        int32_t l;
        double A[6], y[4];
    };
    __device__ __forceinline__ static bool skip(const Ctrl* ctrl) { return ctrl->active == 0; }
    __device__ __forceinline__ void fetch(int32_t seg, Slot& o) const {
        o.l = nel[seg];
        const double2* a = reinterpret_cast<const double2*>(vinv64 + 6 * int64_t(seg));
        const double2* y = reinterpret_cast<const double2*>(ybl + 4 * int64_t(seg));
        const double2 a0 = a[0], a1 = a[1], a2 = a[2], y0 = y[0], y1 = y[1];
        o.A[0] = a0.x; o.A[1] = a0.y; o.A[2] = a1.x; o.A[3] = a1.y; o.A[4] = a2.x; o.A[5] = a2.y;
        o.y[0] = y0.x; o.y[1] = y0.y; o.y[2] = y1.x; o.y[3] = y1.y;
    }
    template <typename TC>
    __device__ __forceinline__ void finish(int32_t, const Slot& o, const TC* v) const {
        if (o.y[3] == 0.0) return;
        const double t[3] = {double(v[0]), double(v[1]), double(v[2])};
        double w[3];
        sym3_apply(o.A, t, w);
        double* d = dxl + 3 * int64_t(o.l);
#pragma unroll
        for (int k = 0; k < 3; ++k) d[k] = -(o.y[k] + w[k]);
    }
};

// Camera vector of one observation from the LDS copy (stride 9).
template <typename TS>
__device__ __forceinline__ void load_cam_vec_lds(const TS* cv, int64_t cam, TS* x) {
#pragma unroll
    for (int k = 0; k < 9; ++k) x[k] = cv[9 * cam + k];
}

// Landmark pass over global memory: each wavefront takes `tpw` consecutive
// tiles; the camera vector is gathered from the L2-resident copy.
template <typename TJ, typename TC, typename TS, typename Tail>
__global__ __launch_bounds__(kBlock) void k_lm_pass(Buffers b, Sizes z, int tpw, Tail tail, const Ctrl* ctrl) {
    if (Tail::skip(ctrl)) return;
    const int64_t wave = int64_t(blockIdx.x) * kWavesPerBlock + wave_in_block();
    const int64_t t0 = wave * tpw;
    if (t0 >= z.ntiles) return;
    const int64_t t1 = min(t0 + int64_t(tpw), z.ntiles);
    lm_pass_range<TJ, TC, TS, false>(b, z, t0, t1, reinterpret_cast<const TS*>(b.vq), tail);
}

// Landmark pass with the camera vector staged in LDS: as many blocks as fit
// on the device at once copy the n_c x 9 vector, then every wavefront takes
// one contiguous range of `per` tiles (one pipeline start per wavefront, and
// equal work for all).
template <typename TJ, typename TC, typename TS, typename Tail>
__global__ __launch_bounds__(kBlock) void k_lm_pass_lds(Buffers b, Sizes z, int64_t per, Tail tail,
                                                        const Ctrl* ctrl) {
    extern __shared__ unsigned char lds_raw[];
    if (Tail::skip(ctrl)) return;
    TS* cv = reinterpret_cast<TS*>(lds_raw);
    const TS* __restrict__ vq = reinterpret_cast<const TS*>(b.vq);
    {
        // R cameras per thread requested before the first is written, so the
        // copy takes a few round trips instead of one per element
        constexpr int R = sizeof(TS) == 4 ? 4 : 2;
        for (int64_t c0 = threadIdx.x; c0 < z.nc; c0 += int64_t(R) * kBlock) {
            TS x[R][9];
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (c0 + r * kBlock < z.nc) load_cam_vec(vq, c0 + r * kBlock, x[r]);
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (c0 + r * kBlock < z.nc)
#pragma unroll
                    for (int k = 0; k < 9; ++k) cv[9 * (c0 + r * kBlock) + k] = x[r][k];
        }
    }
    __syncthreads();
    const int64_t t0 = (int64_t(blockIdx.x) * kWavesPerBlock + wave_in_block()) * per;
    if (t0 >= z.ntiles) return;
    lm_pass_range<TJ, TC, TS, true>(b, z, t0, min(t0 + per, z.ntiles), cv, tail);
}

// The stream over a range of tiles in chunks of 64 positions, as a software
// pipeline over a ring of D record slots (three; two for float64 records):
// while chunk c is summed, the records (camera word first, then the blocks)
// of chunk c + D - 1 are in flight, and the V^-1 of the landmarks ending in
// chunk c + 1 has been requested (its camera words were the first loads of
// their group, so that request waits for nothing younger).  Every record load
// is unconditional (lanes past the end read the last position and are masked
// where the slot is used), and the ring is walked in whole rounds followed by
// the remaining chunks, so no path reaches a slot's reuse with its load
// unconsumed.
template <typename TJ, typename TC, typename TS, bool LDS_CAM, typename Tail>
__device__ __forceinline__ void lm_pass_range(const Buffers& b, const Sizes& z, int64_t t0, int64_t t1,
                                              const TS* __restrict__ vq, const Tail& tail) {
    constexpr int D = sizeof(TJ) == 8 ? 2 : 3;
    const uint32_t* __restrict__ lo_cam = b.lo_cam;
    const int lane = lane_id();
    const int32_t start = b.tile_start[t0];
    const int32_t end = b.tile_start[t1];
    if (start >= end) return;
    const int32_t nch = (end - start + kWave - 1) / kWave;
    RawRec<TJ> rec[D];
    uint32_t w[D];
    typename Tail::Slot A[2];
    int32_t my_seg[2];
    uint64_t hms[2];
    auto fetch = [&](int u, int32_t c) {
        const int32_t i = min(start + c * kWave + lane, end - 1);
        w[u] = lo_cam[i];
        load_raw<TJ>(b.J_lo, z.npad, i, rec[u]);
    };
    auto flags = [&](int u, int32_t c) -> uint32_t { return start + c * kWave + lane < end ? w[u] : 0u; };
    int32_t seg_v = b.seg_base[t0] - 1;  // segment open at the start of the next chunk to prepare
    auto prep = [&](int u, int a, int32_t c) {  // chunk c (slot u): heads, segments, V^-1 request into A[a]
        const uint32_t wu = flags(u, c);
        const uint64_t hm = ballot64(wu & kHeadBit);
        hms[a] = hm;
        my_seg[a] = seg_v + __popcll(hm & mask_upto(lane));
        if (wu & kTailBit) tail.fetch(my_seg[a], A[a]);
        seg_v += __popcll(hm);
    };
#pragma unroll
    for (int u = 0; u < D; ++u) fetch(u, u);
    prep(0, 0, 0);
    TC carry[3] = {TC(0), TC(0), TC(0)};
    auto chunk = [&](auto U, int32_t c) {  // chunk c from record slot u = c % D, gather slot a = c % 2
        constexpr int u = decltype(U)::value % D;
        constexpr int a = decltype(U)::value % 2;
        if (c + 1 < nch) prep((u + 1) % D, 1 - a, c + 1);
        const int32_t pos = start + c * kWave;
        const uint32_t wc = flags(u, c);
        TC v[3] = {TC(0), TC(0), TC(0)};
        if (pos + lane < end) {
            TS xs[9];
            if (LDS_CAM) load_cam_vec_lds(vq, int64_t(wc & kIndexMask), xs);
            else load_cam_vec(vq, int64_t(wc & kIndexMask), xs);
            TC J[24];
            unpack<TC>(rec[u], J);
            TC q0 = TC(0), q1 = TC(0);
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                const TC xk = TC(xs[k]);
                q0 += J[k] * xk;
                q1 += J[9 + k] * xk;
            }
            v[0] = J[18] * q0 + J[21] * q1;
            v[1] = J[19] * q0 + J[22] * q1;
            v[2] = J[20] * q0 + J[23] * q1;
        }
        const bool head = wc & kHeadBit;
        if (lane == 0 && !head) {
            v[0] += carry[0];
            v[1] += carry[1];
            v[2] += carry[2];
        }
        const uint64_t hu = hms[a] & mask_upto(lane);
        const int seg_start = hu ? 63 - __builtin_clzll(hu) : 0;
        segmented_scan<TC, 3>(v, lane, seg_start);
        if (wc & kTailBit) tail.finish(my_seg[a], A[a], v);
        const int last = min(end - pos, kWave) - 1;
#pragma unroll
        for (int k = 0; k < 3; ++k) carry[k] = readlane(v[k], last);
        fetch(u, c + D);
    };
    // rounds of lcm(D, 2) chunks keep both rings aligned
    constexpr int RND = D == 3 ? 6 : 2;
    int32_t c = 0;
    for (; c + RND <= nch; c += RND) {
        chunk(std::integral_constant<int, 0>{}, c);
        chunk(std::integral_constant<int, 1>{}, c + 1);
        if constexpr (RND == 6) {
            chunk(std::integral_constant<int, 2>{}, c + 2);
            chunk(std::integral_constant<int, 3>{}, c + 3);
            chunk(std::integral_constant<int, 4>{}, c + 4);
            chunk(std::integral_constant<int, 5>{}, c + 5);
        }
    }
    if (c < nch) chunk(std::integral_constant<int, 0>{}, c);
    if constexpr (RND == 6) {
        if (c + 1 < nch) chunk(std::integral_constant<int, 1>{}, c + 1);
        if (c + 2 < nch) chunk(std::integral_constant<int, 2>{}, c + 2);
        if (c + 3 < nch) chunk(std::integral_constant<int, 3>{}, c + 3);
        if (c + 4 < nch) chunk(std::integral_constant<int, 4>{}, c + 4);
    }
}

// Launches the landmark pass: with the camera vector in LDS when it fits
// (persistent blocks, a few per compute unit), else gathering it from L2.
constexpr size_t kLdsCamMax = 64 << 10;

template <typename TJ, typename TC, typename TS, typename Tail>
void launch_lm_stream(Problem* p, const Tail& tail, hipStream_t s) {
    const Buffers& b = p->b;
    const Sizes& z = p->z;
    const int tpw = p->tiles_per_wave;
    const int64_t ngroups = ceil_div(z.ntiles, tpw);
    const size_t lds = size_t(z.nc) * 9 * sizeof(TS);
    if (p->lds_cam && lds <= kLdsCamMax) {
        // as many persistent blocks as fit at once (registers and LDS), at most four per compute unit
        int fit = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&fit, k_lm_pass_lds<TJ, TC, TS, Tail>, kBlock, lds) !=
                hipSuccess ||
            fit < 1)
            fit = 1;
        const int64_t per_cu = std::min<int64_t>(4, fit);
        const int64_t waves = p->n_cus * per_cu * kWavesPerBlock;
        const int64_t per = std::max<int64_t>(1, ceil_div(z.ntiles, waves));
        const int64_t nblk = std::max<int64_t>(1, ceil_div(ceil_div(z.ntiles, per), kWavesPerBlock));
        hipLaunchKernelGGL((k_lm_pass_lds<TJ, TC, TS, Tail>), dim3(unsigned(nblk)), dim3(kBlock), lds, s, b, z, per,
                           tail, b.ctrl);
    } else {
        hipLaunchKernelGGL((k_lm_pass<TJ, TC, TS, Tail>), dim3(unsigned(ceil_div(ngroups, kWavesPerBlock))),
                           dim3(kBlock), 0, s, b, z, tpw, tail, b.ctrl);
    }
}

template <typename TJ, typename TC, typename TS>
void launch_lm_pass(Problem* p, hipStream_t s) {
    const Buffers& b = p->b;
    launch_lm_stream<TJ, TC, TS>(
        p, SeriesTail<TS, TC>{reinterpret_cast<const TS*>(b.Vinv), reinterpret_cast<TS*>(b.s)}, s);
}

// Folded camera data (24 slots) of camera `cam` from LDS or global memory.
template <typename TS, typename TC>
__device__ __forceinline__ void load_fold(const TS* src, int64_t cam, TC* c) {
    if constexpr (std::is_same<TS, float>::value) {
        const float4* q = reinterpret_cast<const float4*>(src + kFoldStride<TS> * cam);
#pragma unroll
        for (int g = 0; g < 6; ++g) {
            const float4 x = q[g];
            c[4 * g] = TC(x.x);
            c[4 * g + 1] = TC(x.y);
            c[4 * g + 2] = TC(x.z);
            c[4 * g + 3] = TC(x.w);
        }
    } else {
        const double2* q = reinterpret_cast<const double2*>(src + kFoldStride<TS> * cam);
#pragma unroll
        for (int g = 0; g < 12; ++g) {
            const double2 x = q[g];
            c[2 * g] = TC(x.x);
            c[2 * g + 1] = TC(x.y);
        }
    }
}

// J_l^T J_p v of one observation from its point record and folded camera data.
template <typename TC>
__device__ __forceinline__ void point_lm_term(const TC* P, TC sw, const TC* c, TC* v) {
    const PointShape<TC> sh(P, c[9], c[10], c[11]);
    TC wv[3];
    wv[0] = c[1] * P[2] - c[2] * P[1] + c[3];
    wv[1] = c[2] * P[0] - c[0] * P[2] + c[4];
    wv[2] = c[0] * P[1] - c[1] * P[0] + c[5];
    TC q0, q1;
    sh.JP(wv, q0, q1);
    const TC ci = sh.d * c[6] + c[9] * sh.n * (c[7] + sh.n * c[8]);
    q0 += ci * sh.p0;
    q1 += ci * sh.p1;
    TC g[3];
    sh.JPt(q0, q1, g);
    const TC w = sw * sw;
    // R^T g with R row-major in c[12..20]
    v[0] = w * (c[12] * g[0] + c[15] * g[1] + c[18] * g[2]);
    v[1] = w * (c[13] * g[0] + c[16] * g[1] + c[19] * g[2]);
    v[2] = w * (c[14] * g[0] + c[17] * g[1] + c[20] * g[2]);
}

// Folded camera data of the camera step x (float64), for the back-substitution
// over point records.
__global__ __launch_bounds__(kBlock) void k_fold_x(Buffers b, Sizes z, const double* __restrict__ x,
                                                   const Ctrl* ctrl) {
    if (!ctrl->active) return;
    const int32_t c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= z.nc) return;
    fold_camera<double>(b.lin_rec + kCamRec * int64_t(c), x + 9 * int64_t(c), b.xq + kFoldStride<double> * int64_t(c));
}

// The camera step x (float64) in the landmark stream's camera-vector layout
// (stride 12, storage type), for the back-substitution over Jacobian records.
template <typename TS>
__global__ __launch_bounds__(kBlock) void k_x_to_vq(Buffers b, Sizes z, const double* __restrict__ x,
                                                    const Ctrl* ctrl) {
    if (!ctrl->active) return;
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= int64_t(z.nc) * 9) return;
    reinterpret_cast<TS*>(b.vq)[12 * (i / 9) + i % 9] = TS(x[i]);
}

// Back-substitution over point records: dx_l = -V_lambda^-1 (b_l + sum_{i in
// l} J_l^T J_p x_c) in float64 with V_lambda^-1 recomputed from the float64 V.
// (Over Jacobian records it is the landmark stream with BacksubTail.)
template <typename TJ>
__global__ __launch_bounds__(kBlock) void k_backsub_pt(Buffers b, Sizes z, double* __restrict__ dxl,
                                                       const Ctrl* ctrl) {
    if (!ctrl->active) return;
    const int64_t tile = int64_t(blockIdx.x) * kWavesPerBlock + wave_in_block();
    if (tile >= z.ntiles) return;
    tile_landmarks<double, 3, kLookupLate>(
        b.lo_cam, b.tile_start, b.seg_base, b.nel, z.nl, tile,
        [&](int32_t i, bool valid, int32_t cam, int32_t, int32_t, double* v) {
            v[0] = v[1] = v[2] = 0.0;
            if (!valid) return;
            // J_l^T J_p x from the point record and the camera's folded x (float64)
            double P[3], sw, c[24];
            load_point<TJ, double>(b.J_lo, z.npad, i, P, sw);
            load_fold(b.xq, int64_t(cam), c);
            point_lm_term(P, sw, c, v);
        },
        [&](int32_t seg, int32_t lmk, const double* t) {
            const int64_t l = lmk;
            const PCtrl& q = b.pctl[b.lm_prob[l]];
            if (!q.active) return;
            double Vd[6], inv[6], rhs[3], y[3], dd[3];
#pragma unroll
            for (int k = 0; k < 6; ++k) Vd[k] = b.V[6 * l + k];
#pragma unroll
            for (int k = 0; k < 3; ++k) dd[k] = b.Dl[3 * int64_t(seg) + k];
            inv3_damped(Vd, q.lambda, dd, inv);
#pragma unroll
            for (int k = 0; k < 3; ++k) rhs[k] = b.bl[3 * l + k] + t[k];
            sym3_apply(inv, rhs, y);
#pragma unroll
            for (int k = 0; k < 3; ++k) dxl[3 * l + k] = -y[k];
        });
}

// Compact float64 folded camera data for LDS (144 bytes per camera): slots
// 0..11 of the fold (a, e, v_intrinsics, f, k1, k2) and w, A, B and |w|^2 of
// the linearisation's camera record, from which each observation rebuilds R
// with the operations of make_cam_record (so R is the same to the bit).
struct __attribute__((aligned(16))) CompactFold {
    double c[12];
    double w[3], A, B, th2;
};
static_assert(sizeof(CompactFold) == 144, "144-byte camera slots");

// The block stages the compact fold of every camera from a float64 fold
// (stride kFoldStride<double>) and the camera records; ends synchronised.
__device__ __forceinline__ void stage_compact_fold(const double* __restrict__ fold, const double* __restrict__ lin_rec,
                                                   int32_t nc, CompactFold* cams) {
    for (int32_t c = threadIdx.x; c < nc; c += blockDim.x) {
        const double* f = fold + kFoldStride<double> * int64_t(c);
        const double* r = lin_rec + kCamRec * int64_t(c);
        CompactFold x;
#pragma unroll
        for (int k = 0; k < 12; ++k) x.c[k] = f[k];
        x.w[0] = r[0];
        x.w[1] = r[1];
        x.w[2] = r[2];
        x.A = r[9];
        x.B = r[10];
        {
#pragma clang fp contract(off)
            x.th2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        }
        cams[c] = x;
    }
    __syncthreads();
}

// The 24-slot fold of one camera from its compact form (slots 21..23 unused).
__device__ __forceinline__ void load_compact_fold(const CompactFold& x, double* c) {
#pragma unroll
    for (int k = 0; k < 12; ++k) c[k] = x.c[k];
    {
#pragma clang fp contract(off)
        const double* w = x.w;
        const double A = x.A, B = x.B, th2 = x.th2;
        double* R = c + 12;
        R[0] = 1.0 + B * (w[0] * w[0] - th2);
        R[4] = 1.0 + B * (w[1] * w[1] - th2);
        R[8] = 1.0 + B * (w[2] * w[2] - th2);
        R[1] = -A * w[2] + B * w[0] * w[1];
        R[3] = A * w[2] + B * w[0] * w[1];
        R[2] = A * w[1] + B * w[0] * w[2];
        R[6] = -A * w[1] + B * w[0] * w[2];
        R[5] = -A * w[0] + B * w[1] * w[2];
        R[7] = A * w[0] + B * w[1] * w[2];
    }
}

// Landmarks without observations get dx_l = -V^-1 b_l = 0.
__global__ __launch_bounds__(kBlock) void k_zero_empty(Buffers b, Sizes z, double* dxl, const Ctrl* ctrl) {
    if (!ctrl->active) return;
    const int32_t l = blockIdx.x * kBlock + threadIdx.x;
    if (l >= z.nl) return;
    if (b.lm_off[l + 1] == b.lm_off[l] && b.pctl[b.lm_prob[l]].active) {
        dxl[3 * int64_t(l)] = 0.0;
        dxl[3 * int64_t(l) + 1] = 0.0;
        dxl[3 * int64_t(l) + 2] = 0.0;
    }
}

// -------------------------------------------------------------- camera pass --

// The three stored scalars of s at segment l, kept in the storage type.
__device__ __forceinline__ void load_s3_raw(const float* s, int64_t l, float* o) {
    const float4 a = reinterpret_cast<const float4*>(s)[l];
    o[0] = a.x; o[1] = a.y; o[2] = a.z;
}
__device__ __forceinline__ void load_s3_raw(const double* s, int64_t l, double* o) {
    const double2* p = reinterpret_cast<const double2*>(s + 4 * l);
    const double2 a = p[0];
    o[0] = a.x; o[1] = a.y; o[2] = s[4 * l + 2];
}

__device__ __forceinline__ void load_s3(const float* s, int64_t l, double* o) {
    const float4 a = reinterpret_cast<const float4*>(s)[l];
    o[0] = a.x; o[1] = a.y; o[2] = a.z;
}
__device__ __forceinline__ void load_s3(const double* s, int64_t l, double* o) {
    const double2* p = reinterpret_cast<const double2*>(s + 4 * l);
    const double2 a = p[0];
    o[0] = a.x; o[1] = a.y; o[2] = s[4 * l + 2];
}

// Camera pass, one workgroup of NT threads per camera piece: u = sum_i
// J_p^T (J_l s_g(i)) over the piece in float64, written to the piece's partial
// slot.  Two-stage pipeline per thread: the next observation's record and
// segment index are in flight while the current one is accumulated; its s
// gather is issued after.  A piece averages a few hundred observations, so a
// small workgroup streams it in several pipelined steps.
// Threads per piece (measured at the city size): one wavefront for float64
// records (192 bytes per observation; 7% faster than four), four for the
// narrower ones (one or two wavefronts were 6% and 3% slower).
constexpr int cam_pass_threads(size_t jbytes) { return jbytes == 8 ? kWave : kBlock; }

template <typename TJ, typename TSin, int NT>
__global__ __launch_bounds__(NT) void k_cam_pass(Buffers b, Sizes z, const TSin* __restrict__ sin,
                                                 const Ctrl* ctrl) {
    __shared__ double lds[(NT / kWave) * 9];
    // The control word and the piece are read together, and the problem's
    // active and stopped flags (adjacent) in one request after them, so a
    // workgroup knows within two scalar round trips whether it has work.
    // Nothing is read from the records before that: the launches that follow
    // a stopped series must cost no bandwidth.
    static_assert(sizeof(PieceRec) == 32 && offsetof(PieceRec, prob) == 16, "piece record: two 16-byte words");
    static_assert(offsetof(PCtrl, stopped) == offsetof(PCtrl, active) + 4 && offsetof(PCtrl, active) % 8 == 0 &&
                      sizeof(PCtrl) % 8 == 0,
                  "active and stopped form one aligned 8-byte word");
    const int32_t running = ctrl->running;
    const int4* rec = reinterpret_cast<const int4*>(b.sched_rec) + 2 * int64_t(blockIdx.x);
    const int4 r0 = rec[0], r1 = rec[1];  // (p, begin, end, cam), (prob, ...)
    // (a problem index is never negative: testing it keeps the second word in
    // the first request instead of after the branch)
    if (running == 0 || r0.x < 0 || r1.x < 0) return;
    const int2 flags = *reinterpret_cast<const int2*>(&b.pctl[r1.x].active);
    if (!flags.x || flags.y) return;
    const int32_t p = r0.x, a = r0.y, e = r0.z;
    const int32_t* __restrict__ co_seg = b.co_seg;
    // records stay in their storage width (float for float32 and bfloat16
    // storage) and are widened to float64 at use
    using TL = typename std::conditional<std::is_same<TJ, double>::value, double, float>::type;
    int32_t i = a + threadIdx.x;
    TL J[24];
    double sv[3];
    if (i < e) {
        const int64_t g = co_seg[i];
        load_J<TJ, TL>(b.J_co, z.npad, i, J);
        load_s3(sin, g, sv);
    }
    double acc[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) acc[k] = 0.0;
    for (; i < e; i += NT) {
        const int32_t ni = i + NT;
        int64_t gn = 0;
        TL Jn[24];
        if (ni < e) {
            gn = co_seg[ni];
            load_J<TJ, TL>(b.J_co, z.npad, ni, Jn);
        }
        const double z0 = double(J[18]) * sv[0] + double(J[19]) * sv[1] + double(J[20]) * sv[2];
        const double z1 = double(J[21]) * sv[0] + double(J[22]) * sv[1] + double(J[23]) * sv[2];
#pragma unroll
        for (int k = 0; k < 9; ++k) acc[k] += double(J[k]) * z0 + double(J[9 + k]) * z1;
#pragma unroll
        for (int k = 0; k < 24; ++k) J[k] = Jn[k];
        if (ni < e) load_s3(sin, gn, sv);
    }
    block_sum<9>(acc, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < 9; ++k) b.part[9 * int64_t(p) + k] = acc[k];
    }
}

// Camera finish: nine threads per camera, one per row of U^-1.  u_c is the
// sum of the camera's pieces in piece order, then
//   rhs:    b~_c = b_p - u_c,  v_c = -U^-1 b~_c,  x_c = v_c
//   series: v_c = U^-1 u_c,    x_c += v_c
//   apply:  vout_c = U^-1 u_c
// Cameras of problems that are inactive or stopped are left alone.  The
// camera's squared norms of v and x go to cam_red; k_norm_stop sums them per
// problem and applies the stop rule of eq. qcriterion.
constexpr int kFinCams = kBlock / 9;  // cameras per block (28)

template <typename TS, bool FOLD>
__global__ __launch_bounds__(kBlock) void k_cam_fin(Buffers b, Sizes z, int mode, double* vout, const Ctrl* ctrl) {
    __shared__ double us[kFinCams][9];
    __shared__ double vs[kFinCams][9];
    __shared__ double n2[kFinCams][9][2];
    if (ctrl->running == 0) return;
    const int lc = threadIdx.x / 9, r = threadIdx.x % 9;
    const int32_t c = blockIdx.x * kFinCams + lc;
    const bool valid = lc < kFinCams && c < z.nc;
    // every load that does not depend on the problem's state is issued before
    // its check (camera 0 stands in for threads without a camera)
    const int64_t cc = valid ? c : 0;
    const int32_t prob = b.cam_prob[cc];
    const int32_t q0 = b.cam_piece[cc], q1 = b.cam_piece[cc + 1];
    double Ui[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) Ui[k] = b.Uinv[81 * cc + 9 * r + k];
    const double xo = b.x[9 * cc + r];
    const double bpr = b.bp[9 * cc + r];
    bool own = valid;
    if (own) {
        const PCtrl& q = b.pctl[prob];
        own = q.active && !q.stopped;
    }
    if (own) {
        double u = 0.0;
#pragma unroll 4
        for (int32_t q = q0; q < q1; ++q) u += b.part[9 * int64_t(q) + r];
        if (mode == kFinRhs) {
            u = bpr - u;
            b.bt[9 * int64_t(c) + r] = u;
        }
        us[lc][r] = u;
    }
    __syncthreads();
    if (own) {
        double sacc = 0.0;
#pragma unroll
        for (int k = 0; k < 9; ++k) sacc += Ui[k] * us[lc][k];
        const double v = mode == kFinRhs ? -sacc : sacc;
        if (mode == kFinApply) {
            vout[9 * int64_t(c) + r] = v;
        } else {
            double* xc = b.x + 9 * int64_t(c) + r;
            const double xn = mode == kFinRhs ? v : xo + v;
            *xc = xn;
            b.v[9 * int64_t(c) + r] = v;
            if (FOLD) vs[lc][r] = v;
            else reinterpret_cast<TS*>(b.vq)[12 * int64_t(c) + r] = TS(v);
            n2[lc][r][0] = v * v;
            n2[lc][r][1] = xn * xn;
        }
    }
    if (mode == kFinApply) return;
    __syncthreads();
    if (own && r == 0) {
        double sv = 0.0, sx = 0.0;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            sv += n2[lc][k][0];
            sx += n2[lc][k][1];
        }
        b.cam_red[2 * int64_t(c)] = sv;
        b.cam_red[2 * int64_t(c) + 1] = sx;
        if (FOLD) fold_camera<TS>(b.lin_rec + kCamRec * int64_t(c), vs[lc], reinterpret_cast<TS*>(b.vq) + kFoldStride<TS> * int64_t(c));
    }
}

// Norms of v and x of one problem (its cameras in order, one block per
// problem) and the stop rule of eq. qcriterion for series order `order`.
__global__ __launch_bounds__(kBlock) void k_norm_stop(Buffers b, int mode, int order, double eps, Ctrl* ctrl) {
    __shared__ double lds[kWavesPerBlock * 2];
    if (ctrl->running == 0) return;
    PCtrl& q = b.pctl[blockIdx.x];
    if (!q.active || q.stopped) return;
    const int32_t c0 = b.prob_cam_off[blockIdx.x], c1 = b.prob_cam_off[blockIdx.x + 1];
    double tot[2];
    sum_partials<2>(b.cam_red + 2 * int64_t(c0), uint32_t(c1 - c0), tot, lds);
    if (threadIdx.x == 0) {
        q.norm_v2 = tot[0];
        q.norm_x2 = tot[1];
        q.stop_order = order;
        if (mode == kFinSeries && eps > 0.0 &&
            (tot[1] == 0.0 || double(order + 1) * sqrt(tot[0]) < eps * sqrt(tot[1]))) {
            q.stopped = 1;
            atomicSub(&ctrl->running, 1);
        }
    }
}

template <typename TS>
// `norms`: the per-problem norms (and with eps > 0 the stop rule) are needed
// after this order; with eps = 0 only the last order's are (they go into the
// solve info), so the others are skipped.
void launch_cam_fin(Problem* p, const Buffers& b, int mode, int order, double eps, double* vout, hipStream_t s,
                    bool norms = true) {
    const unsigned nblk = unsigned(ceil_div(p->z.nc, kFinCams));
    if (p->z.point)
        hipLaunchKernelGGL((k_cam_fin<TS, true>), dim3(nblk), dim3(kBlock), 0, s, b, p->z, mode, vout, b.ctrl);
    else
        hipLaunchKernelGGL((k_cam_fin<TS, false>), dim3(nblk), dim3(kBlock), 0, s, b, p->z, mode, vout, b.ctrl);
    if (mode != kFinApply && norms)
        hipLaunchKernelGGL(k_norm_stop, dim3(unsigned(p->z.np)), dim3(kBlock), 0, s, b, mode, order, eps, b.ctrl);
}

// Copies x into the caller's camera step (cameras of active problems) and
// fills the per-problem solve info.
__global__ __launch_bounds__(kBlock) void k_finish(Buffers b, Sizes z, double* dx_cams, poba_solve_info* info,
                                                   const Ctrl* ctrl) {
    if (!ctrl->active) return;
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i < int64_t(z.nc) * 9 && b.pctl[b.cam_prob[i / 9]].active) dx_cams[i] = b.x[i];
    if (info && i < z.np) {
        const PCtrl& q = b.pctl[i];
        if (!q.active) return;
        poba_solve_info& o = info[i];
        o.stop_order = q.stop_order;
        o.stopped = q.stopped;
        o.status = q.status;
        o.reserved = 0;
        o.norm_x = sqrt(q.norm_x2);
        o.norm_v = sqrt(q.norm_v2);
    }
}

__global__ __launch_bounds__(kBlock) void k_zero_f64v(double* p, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// Camera vector into the gather copy (stride 12, storage type), or folded
// into the point-record camera data (stride 24).
template <typename TS, bool FOLD>
__global__ __launch_bounds__(kBlock) void k_load_v(Buffers b, Sizes z, const double* vin, const Ctrl* ctrl) {
    if (!ctrl->active) return;
    const int32_t c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= z.nc) return;
    if (FOLD) {
        double v[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) v[k] = vin[9 * int64_t(c) + k];
        fold_camera<TS>(b.lin_rec + kCamRec * int64_t(c), v, reinterpret_cast<TS*>(b.vq) + kFoldStride<TS> * int64_t(c));
        return;
    }
    TS* vq = reinterpret_cast<TS*>(b.vq) + 12 * int64_t(c);
#pragma unroll
    for (int k = 0; k < 9; ++k) vq[k] = TS(vin[9 * int64_t(c) + k]);
}

// ---------------------------------------------------- point-record passes --
//
// The same two products of P as above with the blocks rebuilt in registers
// from the 4-scalar point records (J depends on an observation only through
// its camera-frame point):
//   landmark pass: J_p v = J_P (a x P + e) + p (d v_f + f n v_k1 + f n^2 v_k2)
//                  with the camera's folded data (a, e, v_i, f, k1, k2, R),
//                  J_l^T q = R^T J_P^T q, times the IRLS weight sw^2;
//   camera pass:   J_l s = J_P (R s); J_p^T z = (J_l(w)^T ((P - t) x h), h,
//                  (d, f n, f n^2) p.z) with h = J_P^T z, the rotation part
//                  multiplied by J_l(w)^T once per piece.

// Landmark pass over point records, one wavefront over the positions of a
// contiguous range of tiles in chunks of 64, as a software pipeline: the
// records (camera word, point, weight) of chunk c + kPtDepth are requested
// when chunk c is done, and the V^-1 of the landmarks ending in chunk
// c + kPtAhead when chunk c starts; each request is consumed at least
// kPtAhead chunks later, so with in-order completion no wait covers a load
// issued in the last kPtAhead chunks.  fold_at(c, cd) gives the folded
// data of camera c (from LDS or from global memory); the tail (the series'
// s = V^-1 t, or the back-substitution's step) fetches its data for the
// segments ending in chunk c + kPtAhead and finishes each segment.
constexpr int kPtDepth = 4;
constexpr int kPtAhead = 2;

template <typename TP, typename TC, typename FoldAt, typename Tail>
__device__ __forceinline__ void lm_pass_stream_pt(const Buffers& b, const Sizes& z, int64_t t0, int64_t t1,
                                                  const FoldAt& fold_at, const Tail& tail) {
    const uint32_t* __restrict__ lo_cam = b.lo_cam;
    const int lane = lane_id();
    const int32_t start = b.tile_start[t0];
    const int32_t end = b.tile_start[t1];
    if (start >= end) return;
    const int32_t seg0 = b.seg_base[t0] - 1;  // segment open at the range start
    const int32_t nch = (end - start + kWave - 1) / kWave;  // chunks of 64 positions
    uint32_t w[kPtDepth];
    TC P[kPtDepth][3], sw[kPtDepth];
    typename Tail::Slot A[kPtDepth];
    // records of chunk c into slot u; every load is unconditional (lanes past
    // the end read the last position and are masked where the slot is used),
    // so a slot's registers are only ever written by its own loads
    auto fetch = [&](int u, int32_t c) {
        const int32_t i = min(start + c * kWave + lane, end - 1);
        w[u] = lo_cam[i];
        load_point<TP, TC>(b.J_lo, z.npad, i, P[u], sw[u]);
    };
    auto flags = [&](int u, int32_t c) -> uint32_t { return start + c * kWave + lane < end ? w[u] : 0u; };
    int32_t seg_v = seg0;  // segment open at the start of the chunk whose V^-1 is requested next
    auto request_vinv = [&](int u, int32_t c) {
        const uint32_t wu = flags(u, c);
        const uint64_t hm = ballot64(wu & kHeadBit);
        const int32_t my = seg_v + __popcll(hm & mask_upto(lane));
        if (wu & kTailBit) tail.fetch(my, A[u]);
        seg_v += __popcll(hm);
    };
#pragma unroll
    for (int u = 0; u < kPtDepth; ++u) fetch(u, u);
#pragma unroll
    for (int u = 0; u < kPtAhead; ++u)
        if (u < nch) request_vinv(u, u);
    int32_t seg = seg0;
    TC carry[3] = {TC(0), TC(0), TC(0)};
    auto chunk = [&](auto U, int32_t c) {  // chunk c from slot u = c % kPtDepth
        constexpr int u = decltype(U)::value;
        constexpr int ua = (u + kPtAhead) % kPtDepth;
        if (c + kPtAhead < nch) request_vinv(ua, c + kPtAhead);
        const int32_t pos = start + c * kWave;
        const uint32_t wc = flags(u, c);
        TC v[3] = {TC(0), TC(0), TC(0)};
        if (pos + lane < end) {
            TC cd[24];
            fold_at(int64_t(wc & kIndexMask), cd);
            point_lm_term(P[u], sw[u], cd, v);
        }
        const uint64_t hm = ballot64(wc & kHeadBit);
        const bool head = wc & kHeadBit;
        if (lane == 0 && !head) {
            v[0] += carry[0];
            v[1] += carry[1];
            v[2] += carry[2];
        }
        const uint64_t hu = hm & mask_upto(lane);
        const int seg_start = hu ? 63 - __builtin_clzll(hu) : 0;
        segmented_scan<TC, 3>(v, lane, seg_start);
        if (wc & kTailBit) tail.finish(seg + __popcll(hu), A[u], v);
        const int last = min(end - pos, kWave) - 1;
#pragma unroll
        for (int k = 0; k < 3; ++k) carry[k] = readlane(v[k], last);
        seg += __popcll(hm);
        fetch(u, c + kPtDepth);
    };
    // whole rounds of kPtDepth chunks, then the rest: no path re-enters the
    // loop with a slot's load unconsumed, so no wait drains the pipeline
    static_assert(kPtDepth == 4, "the round below is written out for four slots");
    int32_t c = 0;
    for (; c + kPtDepth <= nch; c += kPtDepth) {
        chunk(std::integral_constant<int, 0>{}, c);
        chunk(std::integral_constant<int, 1>{}, c + 1);
        chunk(std::integral_constant<int, 2>{}, c + 2);
        chunk(std::integral_constant<int, 3>{}, c + 3);
    }
    if (c < nch) chunk(std::integral_constant<int, 0>{}, c);
    if (c + 1 < nch) chunk(std::integral_constant<int, 1>{}, c + 1);
    if (c + 2 < nch) chunk(std::integral_constant<int, 2>{}, c + 2);
}

constexpr int kPtBlock = 1024;  // persistent LDS variant: one block of 16 waves per compute unit

// Folded camera data staged in LDS once per block; every wavefront of the
// grid takes one contiguous range of tiles.
template <typename TP, typename TC, typename TS>
__global__ __launch_bounds__(kPtBlock) void k_lm_pass_pt_lds(Buffers b, Sizes z, int64_t tiles_per_wave,
                                                              TS* __restrict__ sout, const Ctrl* ctrl) {
    extern __shared__ unsigned char lds_raw[];
    if (ctrl->running == 0) return;
    TS* cf = reinterpret_cast<TS*>(lds_raw);
    // 16-byte units (a camera's padded fold makes whole units)
    static_assert(kFoldStride<TS> * sizeof(TS) % 16 == 0, "whole 16-byte units per camera");
    copy_to_lds(reinterpret_cast<const uint4*>(b.vq), reinterpret_cast<uint4*>(lds_raw),
                int64_t(z.nc) * kFoldStride<TS> * int64_t(sizeof(TS)) / 16);
    const int64_t wave = int64_t(blockIdx.x) * (kPtBlock / kWave) + wave_in_block();
    const int64_t t0 = wave * tiles_per_wave;
    if (t0 >= z.ntiles) return;
    lm_pass_stream_pt<TP, TC>(b, z, t0, min(t0 + tiles_per_wave, z.ntiles),
                              [&](int64_t c, TC* cd) { load_fold(cf, c, cd); },
                              SeriesTail<TS, TC>{reinterpret_cast<const TS*>(b.Vinv), sout});
}

// Float64 series with the compact fold in LDS (144 bytes per camera, where the
// full 208-byte fold does not fit): R is rebuilt per observation.  Blocks of
// eight wavefronts, one per compute unit: the float64 pipeline needs about
// 170 registers per lane.
constexpr int kPtCompactBlock = 512;

template <typename TP>
__global__ __launch_bounds__(kPtCompactBlock) void k_lm_pass_pt_compact(Buffers b, Sizes z, int64_t tiles_per_wave,
                                                                  double* __restrict__ sout, const Ctrl* ctrl) {
    extern __shared__ unsigned char lds_raw[];
    if (ctrl->running == 0) return;
    CompactFold* cams = reinterpret_cast<CompactFold*>(lds_raw);
    stage_compact_fold(reinterpret_cast<const double*>(b.vq), b.lin_rec, z.nc, cams);
    const int64_t wave = int64_t(blockIdx.x) * (kPtCompactBlock / kWave) + wave_in_block();
    const int64_t t0 = wave * tiles_per_wave;
    if (t0 >= z.ntiles) return;
    lm_pass_stream_pt<TP, double>(b, z, t0, min(t0 + tiles_per_wave, z.ntiles),
                                  [&](int64_t c, double* cd) { load_compact_fold(cams[c], cd); },
                                  SeriesTail<double, double>{reinterpret_cast<const double*>(b.Vinv), sout});
}

// Back-substitution over point records as the same stream: the camera
// step's compact fold in LDS, dx_l = -(V^-1 b_l + V^-1 t) at each segment's
// tail from the float64 V^-1 and V^-1 b_l of the solve's preparation
// (BacksubTail), all in float64.
template <typename TP>
__global__ __launch_bounds__(kPtCompactBlock) void k_backsub_pt_stream(Buffers b, Sizes z, int64_t tiles_per_wave,
                                                                       BacksubTail tail, const Ctrl* ctrl) {
    extern __shared__ unsigned char lds_raw[];
    if (BacksubTail::skip(ctrl)) return;
    CompactFold* cams = reinterpret_cast<CompactFold*>(lds_raw);
    stage_compact_fold(b.xq, b.lin_rec, z.nc, cams);
    const int64_t wave = int64_t(blockIdx.x) * (kPtCompactBlock / kWave) + wave_in_block();
    const int64_t t0 = wave * tiles_per_wave;
    if (t0 >= z.ntiles) return;
    lm_pass_stream_pt<TP, double>(b, z, t0, min(t0 + tiles_per_wave, z.ntiles),
                                  [&](int64_t c, double* cd) { load_compact_fold(cams[c], cd); }, tail);
}

// Folded camera data gathered from global memory (L2-resident).
template <typename TP, typename TC, typename TS>
__global__ __launch_bounds__(kBlock) void k_lm_pass_pt(Buffers b, Sizes z, int64_t tiles_per_wave,
                                                       TS* __restrict__ sout, const Ctrl* ctrl) {
    if (ctrl->running == 0) return;
    const int64_t wave = int64_t(blockIdx.x) * kWavesPerBlock + wave_in_block();
    const int64_t t0 = wave * tiles_per_wave;
    if (t0 >= z.ntiles) return;
    const TS* __restrict__ fold = reinterpret_cast<const TS*>(b.vq);
    lm_pass_stream_pt<TP, TC>(b, z, t0, min(t0 + tiles_per_wave, z.ntiles),
                              [&](int64_t c, TC* cd) { load_fold(fold, c, cd); },
                              SeriesTail<TS, TC>{reinterpret_cast<const TS*>(b.Vinv), sout});
}

template <typename TP, typename TC, typename TS>
void launch_lm_pass_pt(Problem* p, hipStream_t s) {
    const Buffers& b = p->b;
    const Sizes& z = p->z;
    const size_t lds = size_t(z.nc) * kFoldStride<TS> * sizeof(TS);
    TS* sout = reinterpret_cast<TS*>(b.s);
    constexpr bool f64 = std::is_same<TS, double>::value && std::is_same<TC, double>::value;
    const size_t lds_compact = size_t(z.nc) * sizeof(CompactFold);
    const bool full = p->lds_cam && lds <= size_t(p->lds_max);
    const bool compact = f64 && !full && p->lds_cam && lds_compact <= size_t(p->lds_max);
    if (full || compact) {
        // one block per compute unit; the tiles are split evenly over all wavefronts
        const int block = full ? kPtBlock : kPtCompactBlock;
        const int64_t waves = p->n_cus * (block / kWave);
        const int64_t per = std::max<int64_t>(1, ceil_div(z.ntiles, waves));
        const int64_t nblk = ceil_div(ceil_div(z.ntiles, per), block / kWave);
        if (full) {
            hipLaunchKernelGGL((k_lm_pass_pt_lds<TP, TC, TS>), dim3(unsigned(nblk)), dim3(block), lds, s, b, z, per,
                               sout, b.ctrl);
        } else if constexpr (f64) {
            hipLaunchKernelGGL((k_lm_pass_pt_compact<TP>), dim3(unsigned(nblk)), dim3(block), lds_compact, s, b, z,
                               per, sout, b.ctrl);
        }
    } else {
        const int64_t per = p->tiles_per_wave;
        hipLaunchKernelGGL((k_lm_pass_pt<TP, TC, TS>), dim3(unsigned(ceil_div(ceil_div(z.ntiles, per), kWavesPerBlock))),
                           dim3(kBlock), 0, s, b, z, per, sout, b.ctrl);
    }
}

// Camera pass over point records, one block per camera piece: per
// observation z = J_P (R s), h = J_P^T z; the piece accumulates
// (P - t) x h, h and (d, f n, f n^2) p.z, weighted by sw^2, in float64, and
// multiplies the first by J_l(w)^T at the end.  TC: per-observation arithmetic.
template <typename TP, typename TSin, typename TC, int NT>
__global__ __launch_bounds__(NT) void k_cam_pass_pt(Buffers b, Sizes z, const TSin* __restrict__ sin,
                                                    const Ctrl* ctrl) {
    __shared__ double lds[(NT / kWave) * 9];
    if (ctrl->running == 0) return;
    const PieceRec pr = b.sched_rec[blockIdx.x];
    if (pr.p < 0) return;
    const int32_t p = pr.p, a = pr.begin, e = pr.end;
    const int64_t cam = pr.cam;
    const int32_t* __restrict__ co_seg = b.co_seg;
    // three-stage pipeline per thread over a ring of three slots (unrolled,
    // so no register of a load in flight is ever copied): the records of
    // observation k + 2 and the gather of s for observation k + 1 are in
    // flight while k is added.  Lanes past the piece read its first
    // observation and add it with weight 0, so every load is unconditional
    // and the wave runs a uniform number of steps.
    struct Obs {
        int32_t g;
        TC P[3], sw;
        bool valid;
    };
    const int32_t lane = threadIdx.x;
    const int32_t n_it = (e - a + NT - 1) / NT;
    auto fetch = [&](int32_t it, Obs& o) {
        const int32_t i = a + lane + it * NT;
        o.valid = i < e;
        const int32_t ic = o.valid ? i : a;
        o.g = co_seg[ic];
        load_point<TP, TC>(b.J_co, z.npad, ic, o.P, o.sw);
    };
    Obs o[3];
    TSin sr[3][3];
    fetch(0, o[0]);
    fetch(1, o[1]);
    const double* rec = b.lin_rec + kCamRec * cam;
    TC R[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) R[k] = TC(rec[13 + k]);
    const TC t0 = TC(rec[3]), t1 = TC(rec[4]), t2 = TC(rec[5]);
    const TC f = TC(rec[6]), k1 = TC(rec[7]), k2 = TC(rec[8]);
    {
        const PCtrl& q = b.pctl[pr.prob];
        if (!q.active || q.stopped) return;
    }
    load_s3_raw(sin, o[0].g, sr[0]);
    // per-lane sums in the arithmetic type (each lane adds a few dozen terms
    // at most), combined across the wave in float64
    TC accl[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) accl[k] = TC(0);
    for (int32_t it = 0; it < n_it; it += 3) {
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            if (it + u >= n_it) break;
            fetch(it + u + 2, o[(u + 2) % 3]);
            load_s3_raw(sin, o[(u + 1) % 3].g, sr[(u + 1) % 3]);
            const Obs& c = o[u];
            const PointShape<TC> sh(c.P, f, k1, k2);
            const TC s0 = TC(sr[u][0]), s1 = TC(sr[u][1]), s2 = TC(sr[u][2]);
            const TC Rs[3] = {R[0] * s0 + R[1] * s1 + R[2] * s2, R[3] * s0 + R[4] * s1 + R[5] * s2,
                              R[6] * s0 + R[7] * s1 + R[8] * s2};
            TC z0, z1, h[3];
            sh.JP(Rs, z0, z1);
            sh.JPt(z0, z1, h);
            const TC w = c.valid ? c.sw * c.sw : TC(0);
            const TC X0 = c.P[0] - t0, X1 = c.P[1] - t1, X2 = c.P[2] - t2;
            const TC wpz = w * (sh.p0 * z0 + sh.p1 * z1);
            accl[0] += w * (X1 * h[2] - X2 * h[1]);
            accl[1] += w * (X2 * h[0] - X0 * h[2]);
            accl[2] += w * (X0 * h[1] - X1 * h[0]);
            accl[3] += w * h[0];
            accl[4] += w * h[1];
            accl[5] += w * h[2];
            accl[6] += sh.d * wpz;
            accl[7] += f * sh.n * wpz;
            accl[8] += f * sh.n * sh.n * wpz;
        }
    }
    double acc[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) acc[k] = double(accl[k]);
    if constexpr (NT == kWave) {
        wave_total_last<9>(acc);
#pragma unroll
        for (int k = 0; k < 9; ++k) acc[k] = readlane_f64(acc[k], kWave - 1);
    } else {
        block_sum<9>(acc, lds);
    }
    if (threadIdx.x == 0) {
        // rotation part: J_l(w)^T times the accumulated (P - t) x h
        const double w0 = rec[0], w1 = rec[1], w2 = rec[2], B = rec[10], E = rec[22];
        const double th2 = w0 * w0 + w1 * w1 + w2 * w2;
        const double ww[3] = {w0, w1, w2};
        const double W[3][3] = {{0.0, -w2, w1}, {w2, 0.0, -w0}, {-w1, w0, 0.0}};
        double u[3];
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int i2 = 0; i2 < 3; ++i2) {
                const double jl = (i2 == j ? 1.0 - E * th2 : 0.0) + B * W[i2][j] + E * ww[i2] * ww[j];
                s += jl * acc[i2];
            }
            u[j] = s;
        }
        double* out = b.part + 9 * int64_t(p);
        out[0] = u[0];
        out[1] = u[1];
        out[2] = u[2];
#pragma unroll
        for (int k = 3; k < 9; ++k) out[k] = acc[k];
    }
}

// Camera pass over point records with the landmark vector staged in LDS,
// one landmark range r per workgroup of NW wavefronts.  The workgroup copies
// its range's slice of s into LDS (structure of arrays); each wavefront then
// walks its list of (camera, r) groups (non-empty; consecutive fours are the
// batches that set-up dealt to it, longest first) in windows of 64: lane k of
// a window holds group k's run in the camera-major order and its camera data.
// A window is taken in batches of four groups; in a batch each set of sixteen lanes (one DPP row) serves one
// group, sixteen consecutive observations per step (records from global
// memory, s from LDS), each lane summing its terms; at the batch's last step
// every set adds its sixteen lanes (DPP shifts within the row) and its last
// lane writes the group's nine sums (the
// rotation part still without J_l(w)^T, which the finish applies per camera)
// to the slot [camera][range][9].  Steps run as one stream across the batches
// of a window: the records of step t + 2 and s of step t + 1 are in flight
// while step t is added (a ring of three unrolled slots; lanes past their
// group read position 0 with weight 0, so every load is unconditional).
// Cameras of inactive or stopped problems contribute no group.
static_assert(kSets * kSetLanes == kWave, "a batch's sets fill the wavefront");
constexpr int kRangeRing = 3;             // steps in flight (records of step t + 2 requested at step t)

// f(integral_constant<int, k>) for k in the sequence, unrolled.
template <typename F, int... k>
__device__ __forceinline__ void unrolled(F&& f, std::integer_sequence<int, k...>) {
    (f(std::integral_constant<int, k>{}), ...);
}
static_assert(kSetLanes == 16, "a set is one DPP row");

template <typename TS, typename TC>
struct RangeSlot {
    int32_t seg;
    bool valid;
    TC P[3], sw;
    TS s[3];
};

template <typename TP, typename TS, typename TC, int NW>
__global__ __launch_bounds__(NW * kWave) void k_cam_pass_range(Buffers b, Sizes z, int32_t R, int32_t spr,
                                                               int64_t nseg, const TS* __restrict__ sin,
                                                               const Ctrl* ctrl) {
    extern __shared__ unsigned char lds_raw[];
    if (ctrl->running == 0) return;
    TS* ls = reinterpret_cast<TS*>(lds_raw);  // [3][spr]
    // the wavefront's record: uniform values, kept in scalar registers so
    // that the window and batch cursors below are scalar too
    const int wave = wave_in_block();
    const int4 wr = b.cw_rec[int64_t(blockIdx.x) * NW + wave];
    const int32_t r = b.cw_rec[int64_t(blockIdx.x) * NW].x;
    const int64_t seg0 = int64_t(r) * spr;
    const int32_t nloc = int32_t(max<int64_t>(0, min<int64_t>(seg0 + spr, nseg) - seg0));
    {
        // the slice is at most kRangeLdsMax bytes: at most kStage landmarks per
        // thread, all requested before the first is written
        constexpr int kStage = int(kRangeLdsMax / (3 * sizeof(TS) * NW * kWave));
        static_assert(int64_t(kStage) * NW * kWave * 3 * sizeof(TS) >= kRangeLdsMax, "staging covers the slice");
        TS v[kStage][3];
#pragma unroll
        for (int u = 0; u < kStage; ++u) {
            const int32_t k = threadIdx.x + u * NW * kWave;
            if (k < nloc) load_s3_raw(sin, seg0 + k, v[u]);
        }
#pragma unroll
        for (int u = 0; u < kStage; ++u) {
            const int32_t k = threadIdx.x + u * NW * kWave;
            if (k < nloc) {
                ls[k] = v[u][0];
                ls[spr + k] = v[u][1];
                ls[2 * spr + k] = v[u][2];
            }
        }
    }
    __syncthreads();
    const int lane = lane_id();
    const int set = lane / kSetLanes, sl = lane % kSetLanes;
    TS* __restrict__ out = reinterpret_cast<TS*>(b.part_grp);
    const int32_t* __restrict__ co_seg = b.co_seg;
    using Slot = RangeSlot<TS, TC>;
    for (int32_t wb = wr.y; wb < wr.z; wb += kWave) {
        // lane k: group k of the window
        const int32_t k = wb + lane;
        int32_t cam = 0, start = 0, len = 0;
        TC prm[15];  // R (9, row-major), t (3), f, k1, k2
#pragma unroll
        for (int q = 0; q < 15; ++q) prm[q] = TC(0);
        {
            // every lane reads an entry (lanes past the list the last one) and
            // its camera data, so all these loads are in flight together
            const int4 e = b.cw_list[min(k, wr.z - 1)];
            cam = e.x;
            const int2 f = *reinterpret_cast<const int2*>(&b.pctl[e.w].active);  // (active, stopped)
            const double* rec = b.lin_rec + kCamRec * int64_t(cam);
#pragma unroll
            for (int q = 0; q < 9; ++q) prm[q] = TC(rec[13 + q]);
#pragma unroll
            for (int q = 0; q < 6; ++q) prm[9 + q] = TC(rec[3 + q]);
            if (k < wr.z && f.x && !f.y) {
                start = e.y;
                len = e.z;
            }
        }
        // steps of each batch: the longest group of its kSets, in units of kSetLanes
        int32_t nit = (len + kSetLanes - 1) / kSetLanes;
#pragma unroll
        for (int m = 1; m < kSets; m *= 2) nit = max(nit, __shfl_xor(nit, m, kWave));
        const int nbat = int((min(wr.z - wb, kWave) + kSets - 1) / kSets);
        auto steps_of = [&](int bt) -> int { return __builtin_amdgcn_readlane(nit, bt * kSets); };
        int32_t T = 0;
        for (int bt = 0; bt < nbat; ++bt) T += steps_of(bt);
        if (T == 0) continue;
        auto advance = [&](int& bt, int& it) {
            ++it;
            while (bt < nbat && it >= steps_of(bt)) {
                ++bt;
                it = 0;
            }
        };
        int bi = 0, ii = -1;  // issue cursor (batch, step)
        advance(bi, ii);
        // the issue batch's group of this lane's set: its run, fetched again
        // only when the cursor enters the next batch
        int32_t gs = 0, gl = 0;
        auto issue_group = [&]() {
            const int g = (bi < nbat ? bi : 0) * kSets + set;
            gs = __shfl(start, g, kWave);
            gl = __shfl(len, g, kWave);
        };
        issue_group();
        auto issue = [&](Slot& o) {
            const bool live = bi < nbat;
            const int32_t j = ii * kSetLanes + sl;
            o.valid = live && j < gl;
            const int32_t mem = o.valid ? gs + j : 0;
            o.seg = co_seg[mem];
            load_point<TP, TC>(b.J_co, z.npad, mem, o.P, o.sw);
            if (live) {
                const int b0 = bi;
                advance(bi, ii);
                if (bi != b0) issue_group();
            }
        };
        auto gather = [&](Slot& o) {
            const int32_t l = o.seg - int32_t(seg0);
            const int32_t lc = (o.valid && l >= 0 && l < nloc) ? l : 0;
            o.s[0] = ls[lc];
            o.s[1] = ls[spr + lc];
            o.s[2] = ls[2 * spr + lc];
        };
        int bc = 0, ic = -1;  // compute cursor
        advance(bc, ic);
        TC acc[9], cp[15];
        auto add = [&](const Slot& o) {
            if (ic == 0) {
                const int g = bc * kSets + set;
#pragma unroll
                for (int q = 0; q < 15; ++q) cp[q] = __shfl(prm[q], g, kWave);
#pragma unroll
                for (int q = 0; q < 9; ++q) acc[q] = TC(0);
            }
            const PointShape<TC> sh(o.P, cp[12], cp[13], cp[14]);
            const TC s0 = TC(o.s[0]), s1 = TC(o.s[1]), s2 = TC(o.s[2]);
            const TC Rs[3] = {cp[0] * s0 + cp[1] * s1 + cp[2] * s2, cp[3] * s0 + cp[4] * s1 + cp[5] * s2,
                              cp[6] * s0 + cp[7] * s1 + cp[8] * s2};
            TC z0, z1, h[3];
            sh.JP(Rs, z0, z1);
            sh.JPt(z0, z1, h);
            const TC w = o.valid ? o.sw * o.sw : TC(0);
            const TC X0 = o.P[0] - cp[9], X1 = o.P[1] - cp[10], X2 = o.P[2] - cp[11];
            const TC wpz = w * (sh.p0 * z0 + sh.p1 * z1);
            acc[0] += w * (X1 * h[2] - X2 * h[1]);
            acc[1] += w * (X2 * h[0] - X0 * h[2]);
            acc[2] += w * (X0 * h[1] - X1 * h[0]);
            acc[3] += w * h[0];
            acc[4] += w * h[1];
            acc[5] += w * h[2];
            acc[6] += sh.d * wpz;
            acc[7] += cp[12] * sh.n * wpz;
            acc[8] += cp[12] * sh.n * sh.n * wpz;
            if (ic == steps_of(bc) - 1) {
                // sum of the set's sixteen lanes into its last lane (row shifts)
#pragma unroll
                for (int q = 0; q < 9; ++q) {
                    acc[q] += dpp<0x111, 0xf>(acc[q]);
                    acc[q] += dpp<0x112, 0xf>(acc[q]);
                    acc[q] += dpp<0x114, 0xf>(acc[q]);
                    acc[q] += dpp<0x118, 0xf>(acc[q]);
                }
                const int g = bc * kSets + set;
                const int32_t gl = __shfl(len, g, kWave);
                const int32_t gc = __shfl(cam, g, kWave);
                if (sl == kSetLanes - 1 && gl > 0) {
                    TS* dst = out + (int64_t(gc) * R + r) * 9;
#pragma unroll
                    for (int q = 0; q < 9; ++q) dst[q] = TS(acc[q]);
                }
            }
            advance(bc, ic);
        };
        Slot o[kRangeRing];
        auto step = [&](auto U) {
            constexpr int u = decltype(U)::value;
            issue(o[(u + kRangeRing - 1) % kRangeRing]);
            gather(o[(u + 1) % kRangeRing]);
            add(o[u]);
        };
        unrolled([&](auto K) { issue(o[decltype(K)::value]); }, std::make_integer_sequence<int, kRangeRing - 1>{});
        gather(o[0]);
        // whole rounds of kRangeRing steps, then the rest: no path re-enters
        // the loop with a slot's load unconsumed, so no wait drains the ring
        int32_t t = 0;
        for (; t + kRangeRing <= T; t += kRangeRing) unrolled(step, std::make_integer_sequence<int, kRangeRing>{});
        unrolled([&](auto K) {
            if (t + decltype(K)::value < T) step(K);
        }, std::make_integer_sequence<int, kRangeRing - 1>{});
    }
}

// Camera finish after a range-staged pass (series mode), one wavefront per
// camera: the camera's group sums over the landmark ranges (lane-strided in
// range order, then DPP shifts into the last lane, read back as wave-uniform
// values),
// the rotation part multiplied by J_l(w)^T, then v_c = U^-1 u_c, x_c += v_c,
// the squared norms of v_c and x_c, and the folded camera data of v_c.
// Cameras of inactive or stopped problems are left alone.
constexpr int kFinRangeCams = kBlock / kWave;

template <typename TS>
__global__ __launch_bounds__(kBlock) void k_cam_fin_range(Buffers b, Sizes z, int32_t R, const Ctrl* ctrl) {
    if (ctrl->running == 0) return;
    const int lane = lane_id();
    const int32_t c = blockIdx.x * kFinRangeCams + wave_in_block();
    if (c >= z.nc) return;
    // every load that does not depend on the problem's state is issued before
    // its check, so the camera's data arrive in one round trip
    const int32_t prob = b.cam_prob[c];
    const TS* __restrict__ src = reinterpret_cast<const TS*>(b.part_grp);
    double a[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) a[k] = 0.0;
    for (int32_t r = lane; r < R; r += kWave) {
        const TS* g = src + (int64_t(c) * R + r) * 9;
#pragma unroll
        for (int k = 0; k < 9; ++k) a[k] += double(g[k]);
    }
    const double* rec = b.lin_rec + kCamRec * int64_t(c);
    const double w0 = rec[0], w1 = rec[1], w2 = rec[2], B = rec[10], E = rec[22];
    double Ui[9], xo = 0.0;
    {
        const int row = lane < 9 ? lane : 0;
        const double* Up = b.Uinv + 81 * int64_t(c) + 9 * row;
#pragma unroll
        for (int k = 0; k < 9; ++k) Ui[k] = Up[k];
        xo = b.x[9 * int64_t(c) + row];
    }
    {
        const PCtrl& q = b.pctl[prob];
        if (!q.active || q.stopped) return;
    }
    wave_total_last<9>(a);
#pragma unroll
    for (int k = 0; k < 9; ++k) a[k] = readlane_f64(a[k], kWave - 1);
    double u[9];
    {
        // J_l(w)^T times the accumulated (P - t) x h
        const double th2 = w0 * w0 + w1 * w1 + w2 * w2;
        const double ww[3] = {w0, w1, w2};
        const double W[3][3] = {{0.0, -w2, w1}, {w2, 0.0, -w0}, {-w1, w0, 0.0}};
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double t = 0.0;
#pragma unroll
            for (int i2 = 0; i2 < 3; ++i2) {
                const double jl = (i2 == j ? 1.0 - E * th2 : 0.0) + B * W[i2][j] + E * ww[i2] * ww[j];
                t += jl * a[i2];
            }
            u[j] = t;
        }
#pragma unroll
        for (int k = 3; k < 9; ++k) u[k] = a[k];
    }
    double v = 0.0, xn = 0.0;
    if (lane < 9) {
#pragma unroll
        for (int k = 0; k < 9; ++k) v += Ui[k] * u[k];
        xn = xo + v;
        b.x[9 * int64_t(c) + lane] = xn;
        b.v[9 * int64_t(c) + lane] = v;
    }
    double vs[9], sv = 0.0, sx = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        vs[k] = readlane_f64(v, k);
        const double xk = readlane_f64(xn, k);
        sv += vs[k] * vs[k];
        sx += xk * xk;
    }
    if (lane == 0) {
        b.cam_red[2 * int64_t(c)] = sv;
        b.cam_red[2 * int64_t(c) + 1] = sx;
        fold_camera<TS>(rec, vs, reinterpret_cast<TS*>(b.vq) + kFoldStride<TS> * int64_t(c));
    }
}

// --------------------------------------------------------------- host side --

// Camera pass of one order over the handle's records.
// A series pass over point records (sin in the storage type) stages the
// landmark ranges in LDS when the handle allows it; its finish is then
// k_cam_fin_range (uses_range_pass tells which).
inline bool uses_range_pass(const Problem* p, bool series) {
    return series && p->range_lds && p->range_lds_ok;
}

template <typename TJ, typename TSin, typename TCL, bool PT>
void launch_cam_pass(Problem* p, const Buffers& b, const TSin* sin, hipStream_t s, bool series = false) {
    const dim3 g(unsigned(std::max<int64_t>(p->sched_len, 1)));
    if constexpr (PT) {
        if (uses_range_pass(p, series)) {
            constexpr int NW = range_pass_waves(sizeof(TSin));
            const size_t lds = size_t(p->seg_per_range) * 3 * sizeof(TSin);
            hipLaunchKernelGGL((k_cam_pass_range<TJ, TSin, TCL, NW>), dim3(unsigned(p->cw_blocks)), dim3(NW * kWave),
                               lds, s, b, p->z, p->lm_ranges, p->seg_per_range, p->nnel, sin, b.ctrl);
        } else {
            hipLaunchKernelGGL((k_cam_pass_pt<TJ, TSin, TCL, kWave>), g, dim3(kWave), 0, s, b, p->z, sin, b.ctrl);
        }
    } else {
        constexpr int NT = cam_pass_threads(sizeof(TJ));
        if (NT > kWave && small_pieces(p)) {
            hipLaunchKernelGGL((k_cam_pass<TJ, TSin, kWave>), g, dim3(kWave), 0, s, b, p->z, sin, b.ctrl);
        } else {
            hipLaunchKernelGGL((k_cam_pass<TJ, TSin, NT>), g, dim3(NT), 0, s, b, p->z, sin, b.ctrl);
        }
    }
}

template <typename TJ, typename TCL, typename TS, bool PT>
void launch_lm_pass_any(Problem* p, hipStream_t s) {
    if constexpr (PT) launch_lm_pass_pt<TJ, TCL, TS>(p, s);
    else launch_lm_pass<TJ, TCL, TS>(p, s);
}

// TJ: record storage (Jacobian blocks, or the point-record type when PT),
// TS: landmark-side storage, TCL: landmark-pass arithmetic.
// Damped inverses of every block (float64) and the reduced right-hand side
// b~ = b_p - W V^-1 b_l, with x = v = -U^-1 b~ as order 0 of the series;
// `norms0`: the per-problem norms of order 0 are computed (the solve info
// needs them when the series ends there).
template <typename TJ, typename TS, typename TCL, bool PT>
void solve_prepare(Problem* p, const Buffers& b, double eps, bool norms0, hipStream_t s) {
    const int frozen = p->damping_frozen;
    const Sizes& z = p->z;
    const int damping = p->d.damping;
    const dim3 blk(kBlock);
    const dim3 g_cam(unsigned(ceil_div(z.nc, kBlock)));
    const int32_t nseg = int32_t(p->nnel);
    const dim3 g_seg(unsigned(std::max<int64_t>(ceil_div(nseg, kBlock), 1)));
    {
        ProfScope pr(p, POBA_K_INVERSE, s);
        hipLaunchKernelGGL(k_inv_cam, g_cam, blk, 0, s, b, z, damping, frozen, b.ctrl);
        hipLaunchKernelGGL(k_inv_lm<TS>, g_seg, blk, 0, s, b, nseg, damping, frozen, b.ctrl);
    }
    if (p->npieces > 0) {
        // the reduced right-hand side (not a series order)
        ProfScope pr(p, POBA_K_OTHER, s);
        launch_cam_pass<TJ, double, double, PT>(p, b, reinterpret_cast<const double*>(b.s), s);
        launch_cam_fin<TS>(p, b, kFinRhs, 0, eps, nullptr, s, norms0);
    }
}

// Orders 1..m of the series from the current term (v and its gather copy or
// folded data) and sum x.  `last_norms`: the per-problem norms of order m are
// computed (with eps > 0 every order's are, for the stop rule).
template <typename TJ, typename TS, typename TCL, bool PT>
void series_orders(Problem* p, const Buffers& b, int m, double eps, bool last_norms, hipStream_t s) {
    if (p->npieces == 0) return;
    const Sizes& z = p->z;
    const dim3 blk(kBlock);
    for (int i = 1; i <= m; ++i) {
        {
            ProfScope pr(p, POBA_K_LM_PASS, s);
            launch_lm_pass_any<TJ, TCL, TS, PT>(p, s);
        }
        const bool range = PT && uses_range_pass(p, true);
        {
            ProfScope pr(p, POBA_K_CAM_PASS, s);
            launch_cam_pass<TJ, TS, TCL, PT>(p, b, reinterpret_cast<const TS*>(b.s), s, true);
        }
        {
            ProfScope pr(p, POBA_K_CAM_FIN, s);
            const bool norms = eps > 0.0 || (i == m && last_norms);
            if (range) {
                hipLaunchKernelGGL(k_cam_fin_range<TS>, dim3(unsigned(ceil_div(z.nc, kFinRangeCams))), blk, 0, s,
                                   b, z, p->lm_ranges, b.ctrl);
                if (norms)
                    hipLaunchKernelGGL(k_norm_stop, dim3(unsigned(z.np)), blk, 0, s, b, kFinSeries, i, eps,
                                       b.ctrl);
            } else {
                launch_cam_fin<TS>(p, b, kFinSeries, i, eps, nullptr, s, norms);
            }
        }
    }
}

// dx_l = -V^-1 (b_l + W^T x) for the camera step x = b.x, which is copied to
// dx_cams; the solve info of every active problem to info (may be null).
template <typename TJ, typename TS, typename TCL, bool PT>
void solve_backsub(Problem* p, const Buffers& b, double* dx_cams, double* dx_lms, poba_solve_info* info,
                   hipStream_t s) {
    const Sizes& z = p->z;
    const dim3 blk(kBlock);
    const dim3 g_cam(unsigned(ceil_div(z.nc, kBlock)));
    const dim3 g_lm(unsigned(ceil_div(z.nl, kBlock)));
    const dim3 g_tiles(unsigned(ceil_div(z.ntiles, kWavesPerBlock)));
    ProfScope pr(p, POBA_K_BACKSUB, s);
    if constexpr (PT) {
        hipLaunchKernelGGL(k_fold_x, g_cam, blk, 0, s, b, z, b.x, b.ctrl);
        const size_t lds = size_t(z.nc) * sizeof(CompactFold);
        if (p->lds_cam && lds <= size_t(p->lds_max)) {
            // one block per compute unit; the tiles are split evenly over all wavefronts
            const int64_t waves = p->n_cus * (kPtCompactBlock / kWave);
            const int64_t per = std::max<int64_t>(1, ceil_div(z.ntiles, waves));
            const int64_t nblk = ceil_div(ceil_div(z.ntiles, per), kPtCompactBlock / kWave);
            hipLaunchKernelGGL((k_backsub_pt_stream<TJ>), dim3(unsigned(nblk)), dim3(kPtCompactBlock), lds, s, b, z,
                               per, BacksubTail{b.nel, b.vinv64, b.ybl, dx_lms}, b.ctrl);
        } else {
            hipLaunchKernelGGL((k_backsub_pt<TJ>), g_tiles, blk, 0, s, b, z, dx_lms, b.ctrl);
        }
    } else {
        // the series' landmark stream (its storage and arithmetic types) on x
        hipLaunchKernelGGL((k_x_to_vq<TS>), dim3(unsigned(ceil_div(int64_t(z.nc) * 9, kBlock))), blk, 0, s, b, z,
                           b.x, b.ctrl);
        launch_lm_stream<TJ, TCL, TS>(p, BacksubTail{b.nel, b.vinv64, b.ybl, dx_lms}, s);
    }
    hipLaunchKernelGGL(k_zero_empty, g_lm, blk, 0, s, b, z, dx_lms, b.ctrl);
    const int64_t nfin = std::max<int64_t>(int64_t(z.nc) * 9, z.np);
    hipLaunchKernelGGL(k_finish, dim3(unsigned(ceil_div(nfin, kBlock))), blk, 0, s, b, z, dx_cams, info, b.ctrl);
}

template <typename TJ, typename TS, typename TCL, bool PT>
poba_status run_solve(Problem* p, int m, double eps, double* dx_cams, double* dx_lms, poba_solve_info* info,
                      const double* rhs_p, const double* rhs_l, hipStream_t s) {
    // a replacement right-hand side stands in for (b_p, b_l) in every kernel
    // of this solve (the buffers are passed by value)
    Buffers b = p->b;
    if (rhs_p) b.bp = const_cast<double*>(rhs_p);
    if (rhs_l) b.bl = const_cast<double*>(rhs_l);
    solve_prepare<TJ, TS, TCL, PT>(p, b, eps, m == 0, s);
    series_orders<TJ, TS, TCL, PT>(p, b, m, eps, true, s);
    solve_backsub<TJ, TS, TCL, PT>(p, b, dx_cams, dx_lms, info, s);
    return hipGetLastError() == hipSuccess ? POBA_OK : POBA_ERR_HIP;
}

poba_status launch_solve(Problem* p, int m, double eps, double* dx_cams, double* dx_lms, poba_solve_info* info,
                         hipStream_t s, const double* rhs_p, const double* rhs_l) {
    if (p->z.point) {
        if (p->d.precision == POBA_F64)
            return run_solve<double, double, double, true>(p, m, eps, dx_cams, dx_lms, info, rhs_p, rhs_l, s);
        return run_solve<float, float, float, true>(p, m, eps, dx_cams, dx_lms, info, rhs_p, rhs_l, s);
    }
    switch (p->d.precision) {
        case POBA_F64: return run_solve<double, double, double, false>(p, m, eps, dx_cams, dx_lms, info, rhs_p, rhs_l, s);
        case POBA_F32: return run_solve<float, float, float, false>(p, m, eps, dx_cams, dx_lms, info, rhs_p, rhs_l, s);
        default: return run_solve<bf16_t, float, float, false>(p, m, eps, dx_cams, dx_lms, info, rhs_p, rhs_l, s);
    }
}

poba_status launch_begin_solve(Problem* p, double lam, hipStream_t s) {
    hipLaunchKernelGGL(k_begin_solve, dim3(1), dim3(kReduceBlock), 0, s, p->b.ctrl, p->b.pctl, p->z.np, lam);
    return hipGetLastError() == hipSuccess ? POBA_OK : POBA_ERR_HIP;
}

template <typename TJ, typename TS, typename TCL, bool PT>
poba_status run_apply_P(Problem* p, const double* vin, double* vout, hipStream_t s) {
    const Buffers& b = p->b;
    const Sizes& z = p->z;
    const dim3 blk(kBlock);
    const dim3 g_cam(unsigned(ceil_div(z.nc, kBlock)));
    const int tpw = p->tiles_per_wave;
    hipLaunchKernelGGL((k_load_v<TS, PT>), g_cam, blk, 0, s, b, z, vin, b.ctrl);
    hipLaunchKernelGGL(k_zero_f64v, dim3(unsigned(ceil_div(int64_t(z.nc) * 9, kBlock))), blk, 0, s, vout,
                       int64_t(z.nc) * 9);
    launch_lm_pass_any<TJ, TCL, TS, PT>(p, s);
    if (p->npieces > 0) {
        launch_cam_pass<TJ, TS, TCL, PT>(p, b, reinterpret_cast<const TS*>(b.s), s);
        launch_cam_fin<TS>(p, b, kFinApply, 0, 0.0, vout, s);
    }
    return hipGetLastError() == hipSuccess ? POBA_OK : POBA_ERR_HIP;
}

// ------------------------------------------------ reduced-system residual --
//
// |S x + b~| / |b~| for a camera step x, S x = U_lambda x - W V^-1 W^T x
// (eq. Schur), in float64 with V^-1 recomputed in float64, for every problem
// of the last solve (its damping, D and b~).

// Series flags cleared so that the camera pass covers every active problem.
__global__ __launch_bounds__(kReduceBlock) void k_begin_residual(Ctrl* ctrl, PCtrl* pctl, int32_t np) {
    int n = 0;
    for (int32_t base = 0; base < np; base += blockDim.x) {
        const int32_t j = base + threadIdx.x;
        int a = 0;
        if (j < np) {
            pctl[j].stopped = 0;
            a = pctl[j].active;
        }
        n += __syncthreads_count(a);
    }
    if (threadIdx.x == 0) ctrl->running = n;
}

// s_l = V_lambda^-1 sum_{i in l} J_l^T J_p x_c in float64 (float64 view of s).
template <typename TJ, bool PT>
__global__ __launch_bounds__(kBlock) void k_lm_apply64(Buffers b, Sizes z, const double* __restrict__ x,
                                                       const Ctrl* ctrl) {
    if (!ctrl->active) return;
    const int64_t tile = int64_t(blockIdx.x) * kWavesPerBlock + wave_in_block();
    if (tile >= z.ntiles) return;
    tile_landmarks<double, 3, kLookupTail>(
        b.lo_cam, b.tile_start, b.seg_base, b.nel, z.nl, tile,
        [&](int32_t i, bool valid, int32_t cam, int32_t, int32_t, double* v) {
            v[0] = v[1] = v[2] = 0.0;
            if (!valid) return;
            double J[24];
            Rec<TJ, PT>::template jac<double>(b, z, b.J_lo, i, cam, J);
            const double* vc = x + 9 * int64_t(cam);
            double q0 = 0.0, q1 = 0.0;
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                q0 += J[k] * vc[k];
                q1 += J[9 + k] * vc[k];
            }
            v[0] = J[18] * q0 + J[21] * q1;
            v[1] = J[19] * q0 + J[22] * q1;
            v[2] = J[20] * q0 + J[23] * q1;
        },
        [&](int32_t seg, int32_t lmk, const double* t) {
            const int64_t l = lmk;
            const PCtrl& q = b.pctl[b.lm_prob[l]];
            if (!q.active) return;
            double Vd[6], inv[6], y[3], dd[3];
#pragma unroll
            for (int k = 0; k < 6; ++k) Vd[k] = b.V[6 * l + k];
#pragma unroll
            for (int k = 0; k < 3; ++k) dd[k] = b.Dl[3 * int64_t(seg) + k];
            inv3_damped(Vd, q.lambda, dd, inv);
            sym3_apply(inv, t, y);
            double* o = reinterpret_cast<double*>(b.s) + 4 * int64_t(seg);
            o[0] = y[0];
            o[1] = y[1];
            o[2] = y[2];
            o[3] = 0.0;
        });
}

// Per camera: r_c = U_lambda x_c - (W s)_c + b~_c; squared norms of r_c and
// b~_c to cam_red.
__global__ __launch_bounds__(kBlock) void k_residual_cam(Buffers b, Sizes z, const double* __restrict__ x,
                                                         const Ctrl* ctrl) {
    if (!ctrl->active) return;
    const int32_t c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= z.nc) return;
    const PCtrl& q = b.pctl[b.cam_prob[c]];
    if (!q.active) return;
    double u[9], xc[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        u[k] = 0.0;
        xc[k] = x[9 * int64_t(c) + k];
    }
    for (int32_t p = b.cam_piece[c]; p < b.cam_piece[c + 1]; ++p) {
#pragma unroll
        for (int k = 0; k < 9; ++k) u[k] += b.part[9 * int64_t(p) + k];
    }
    const double* U = b.U + 81 * int64_t(c);
    double r2 = 0.0, b2 = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        double acc = q.lambda * b.Dp[9 * int64_t(c) + k] * xc[k];
#pragma unroll
        for (int j = 0; j < 9; ++j) acc += U[9 * k + j] * xc[j];
        const double btk = b.bt[9 * int64_t(c) + k];
        const double r = acc - u[k] + btk;
        r2 += r * r;
        b2 += btk * btk;
    }
    b.cam_red[2 * int64_t(c)] = r2;
    b.cam_red[2 * int64_t(c) + 1] = b2;
}

// Per problem: |r| / |b~| from its cameras' squared norms (compensated sums).
__global__ __launch_bounds__(kBlock) void k_residual_norm(Buffers b, double* out, const Ctrl* ctrl) {
    __shared__ double lds[kWavesPerBlock * 2];
    if (!ctrl->active) return;
    const PCtrl& q = b.pctl[blockIdx.x];
    if (!q.active) return;
    const int32_t c0 = b.prob_cam_off[blockIdx.x], c1 = b.prob_cam_off[blockIdx.x + 1];
    double tot[2];
    sum_partials<2>(b.cam_red + 2 * int64_t(c0), uint32_t(c1 - c0), tot, lds);
    if (threadIdx.x == 0) out[blockIdx.x] = tot[1] > 0.0 ? sqrt(tot[0]) / sqrt(tot[1]) : 0.0;
}

template <typename TJ, bool PT>
poba_status run_residual(Problem* p, const double* x, double* out, hipStream_t s) {
    const Buffers& b = p->b;
    const Sizes& z = p->z;
    hipLaunchKernelGGL(k_begin_residual, dim3(1), dim3(kReduceBlock), 0, s, b.ctrl, b.pctl, z.np);
    hipLaunchKernelGGL((k_lm_apply64<TJ, PT>), dim3(unsigned(ceil_div(z.ntiles, kWavesPerBlock))), dim3(kBlock), 0,
                       s, b, z, x, b.ctrl);
    if (p->npieces > 0) launch_cam_pass<TJ, double, double, PT>(p, b, reinterpret_cast<const double*>(b.s), s);
    hipLaunchKernelGGL(k_residual_cam, dim3(unsigned(ceil_div(z.nc, kBlock))), dim3(kBlock), 0, s, b, z, x, b.ctrl);
    hipLaunchKernelGGL(k_residual_norm, dim3(unsigned(z.np)), dim3(kBlock), 0, s, b, out, b.ctrl);
    return hipGetLastError() == hipSuccess ? POBA_OK : POBA_ERR_HIP;
}

// Widens the blocks of one order (stored, or rebuilt from point records) to
// float64 in original observation order.
template <typename TJ, bool PT>
__global__ __launch_bounds__(kBlock) void k_get_jac(Buffers b, Sizes z, int order, double* Jp, double* Jl, double* r) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= z.N) return;
    int64_t cam = 0;
    if (PT) {
        if (order == 0) {
            cam = b.lo_cam[i] & kIndexMask;
        } else {  // camera of a camera-major position: last cam_off[c] <= i
            int32_t lo = 0, hi = z.nc - 1;
            while (lo < hi) {
                const int32_t mid = (lo + hi + 1) >> 1;
                if (b.cam_off[mid] <= i) lo = mid; else hi = mid - 1;
            }
            cam = lo;
        }
    }
    double J[24];
    Rec<TJ, PT>::template jac<double>(b, z, order == 0 ? b.J_lo : b.J_co, i, cam, J);
    const int64_t o = order == 0 ? b.perm_l[i] : b.perm_c[i];
#pragma unroll
    for (int k = 0; k < 18; ++k) Jp[18 * o + k] = J[k];
#pragma unroll
    for (int k = 0; k < 6; ++k) Jl[6 * o + k] = J[18 + k];
    if (r) {  // residuals live camera-major
        const int64_t oc = b.perm_c[i];
        r[2 * oc] = b.r_co[2 * i];
        r[2 * oc + 1] = b.r_co[2 * i + 1];
    }
}

__global__ __launch_bounds__(kBlock) void k_get_blocks(Buffers b, Sizes z, double* U, double* V, double* bp,
                                                       double* bl) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (U && i < int64_t(z.nc) * 81) U[i] = b.U[i];
    if (bp && i < int64_t(z.nc) * 9) bp[i] = b.bp[i];
    if (V && i < int64_t(z.nl)) {
        const double* s = b.V + 6 * i;
        double* o = V + 9 * i;
        o[0] = s[0]; o[1] = s[1]; o[2] = s[2];
        o[3] = s[1]; o[4] = s[3]; o[5] = s[4];
        o[6] = s[2]; o[7] = s[4]; o[8] = s[5];
    }
    if (bl && i < int64_t(z.nl) * 3) bl[i] = b.bl[i];
}

// ------------------------------------ building blocks for other solvers --

template <typename TJ_, typename TS_, typename TCL_, bool PT_>
struct Types {
    using TJ = TJ_;
    using TS = TS_;
    using TCL = TCL_;
    static constexpr bool PT = PT_;
};

// Calls f with the Types of the handle's records and precision.
template <typename F>
poba_status with_types(const Problem* p, F&& f) {
    if (p->z.point) {
        if (p->d.precision == POBA_F64) return f(Types<double, double, double, true>{});
        return f(Types<float, float, float, true>{});
    }
    switch (p->d.precision) {
        case POBA_F64: return f(Types<double, double, double, false>{});
        case POBA_F32: return f(Types<float, float, float, false>{});
        default: return f(Types<bf16_t, float, float, false>{});
    }
}

inline poba_status last_error() { return hipGetLastError() == hipSuccess ? POBA_OK : POBA_ERR_HIP; }

poba_status launch_solve_prepare(Problem* p, hipStream_t s) {
    return with_types(p, [&](auto t) {
        using T = decltype(t);
        solve_prepare<typename T::TJ, typename T::TS, typename T::TCL, T::PT>(p, p->b, 0.0, false, s);
        return last_error();
    });
}

poba_status launch_series_orders(Problem* p, int m, hipStream_t s) {
    return with_types(p, [&](auto t) {
        using T = decltype(t);
        series_orders<typename T::TJ, typename T::TS, typename T::TCL, T::PT>(p, p->b, m, 0.0, false, s);
        return last_error();
    });
}

poba_status launch_load_v(Problem* p, const double* v, hipStream_t s) {
    return with_types(p, [&](auto t) {
        using T = decltype(t);
        hipLaunchKernelGGL((k_load_v<typename T::TS, T::PT>), dim3(unsigned(ceil_div(p->z.nc, kBlock))),
                           dim3(kBlock), 0, s, p->b, p->z, v, p->b.ctrl);
        return last_error();
    });
}

poba_status launch_schur_part64(Problem* p, const double* x, hipStream_t s) {
    return with_types(p, [&](auto t) {
        using T = decltype(t);
        const Buffers& b = p->b;
        {
            ProfScope pr(p, POBA_K_LM_PASS, s);
            hipLaunchKernelGGL((k_lm_apply64<typename T::TJ, T::PT>),
                               dim3(unsigned(ceil_div(p->z.ntiles, kWavesPerBlock))), dim3(kBlock), 0, s, b, p->z, x,
                               b.ctrl);
        }
        if (p->npieces > 0) {
            ProfScope pr(p, POBA_K_CAM_PASS, s);
            launch_cam_pass<typename T::TJ, double, double, T::PT>(p, b, reinterpret_cast<const double*>(b.s), s);
        }
        return last_error();
    });
}

poba_status launch_backsub_from_x(Problem* p, double* dx_cams, double* dx_lms, hipStream_t s) {
    return with_types(p, [&](auto t) {
        using T = decltype(t);
        solve_backsub<typename T::TJ, typename T::TS, typename T::TCL, T::PT>(p, p->b, dx_cams, dx_lms, nullptr, s);
        return last_error();
    });
}

}  // namespace poba

using namespace poba;

extern "C" {

poba_status poba_power_solve(poba_problem p, double lambda, int32_t m, double eps, double* dx_cams, double* dx_lms,
                             poba_solve_info* info, poba_stream stream) {
    (void)hipGetLastError();  // report only this call's launch errors
    if (!p || !dx_cams || !dx_lms) return POBA_ERR_INVALID_ARG;
    if (!(lambda > 0.0) || m < 0 || m > 100000 || !(eps >= 0.0)) return POBA_ERR_INVALID_ARG;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    poba_status st = launch_begin_solve(p, lambda, s);
    if (st) return st;
    return launch_solve(p, m, eps, dx_cams, dx_lms, info, s);
}

poba_status poba_solve_residual(poba_problem p, const double* dx_cams, double* rel_residual, poba_stream stream) {
    (void)hipGetLastError();  // report only this call's launch errors
    if (!p || !dx_cams || !rel_residual) return POBA_ERR_INVALID_ARG;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (p->z.point) {
        if (p->d.precision == POBA_F64) return run_residual<double, true>(p, dx_cams, rel_residual, s);
        return run_residual<float, true>(p, dx_cams, rel_residual, s);
    }
    switch (p->d.precision) {
        case POBA_F64: return run_residual<double, false>(p, dx_cams, rel_residual, s);
        case POBA_F32: return run_residual<float, false>(p, dx_cams, rel_residual, s);
        default: return run_residual<bf16_t, false>(p, dx_cams, rel_residual, s);
    }
}

poba_status poba_apply_P(poba_problem p, const double* v_in, double* v_out, poba_stream stream) {
    (void)hipGetLastError();  // report only this call's launch errors
    if (!p || !v_in || !v_out) return POBA_ERR_INVALID_ARG;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_begin_solve, dim3(1), dim3(kReduceBlock), 0, s, p->b.ctrl, p->b.pctl, p->z.np, 0.0);
    // k_begin_solve overwrote lambda; the inverses of the last solve are kept,
    // and apply-P does not read lambda.
    if (p->z.point) {
        if (p->d.precision == POBA_F64) return run_apply_P<double, double, double, true>(p, v_in, v_out, s);
        return run_apply_P<float, float, float, true>(p, v_in, v_out, s);
    }
    switch (p->d.precision) {
        case POBA_F64: return run_apply_P<double, double, double, false>(p, v_in, v_out, s);
        case POBA_F32: return run_apply_P<float, float, float, false>(p, v_in, v_out, s);
        default: return run_apply_P<bf16_t, float, float, false>(p, v_in, v_out, s);
    }
}

poba_status poba_get_jacobians(poba_problem p, int32_t order, double* Jp, double* Jl, double* r, poba_stream stream) {
    (void)hipGetLastError();  // report only this call's launch errors
    if (!p || !Jp || !Jl || (order != 0 && order != 1)) return POBA_ERR_INVALID_ARG;
    if (p->z.N == 0) return POBA_OK;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const dim3 g(unsigned(ceil_div(p->z.N, kBlock)));
    if (p->z.point) {
        if (p->d.precision == POBA_F64)
            hipLaunchKernelGGL((k_get_jac<double, true>), g, dim3(kBlock), 0, s, p->b, p->z, order, Jp, Jl, r);
        else
            hipLaunchKernelGGL((k_get_jac<float, true>), g, dim3(kBlock), 0, s, p->b, p->z, order, Jp, Jl, r);
        return hipGetLastError() == hipSuccess ? POBA_OK : POBA_ERR_HIP;
    }
    switch (p->d.precision) {
        case POBA_F64: hipLaunchKernelGGL((k_get_jac<double, false>), g, dim3(kBlock), 0, s, p->b, p->z, order, Jp, Jl, r); break;
        case POBA_F32: hipLaunchKernelGGL((k_get_jac<float, false>), g, dim3(kBlock), 0, s, p->b, p->z, order, Jp, Jl, r); break;
        default: hipLaunchKernelGGL((k_get_jac<bf16_t, false>), g, dim3(kBlock), 0, s, p->b, p->z, order, Jp, Jl, r); break;
    }
    return hipGetLastError() == hipSuccess ? POBA_OK : POBA_ERR_HIP;
}

poba_status poba_get_blocks(poba_problem p, double* U, double* V, double* bp, double* bl, poba_stream stream) {
    (void)hipGetLastError();  // report only this call's launch errors
    if (!p) return POBA_ERR_INVALID_ARG;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int64_t n = std::max<int64_t>(int64_t(p->z.nc) * 81, int64_t(p->z.nl) * 3);
    hipLaunchKernelGGL(k_get_blocks, dim3(unsigned(ceil_div(n, kBlock))), dim3(kBlock), 0, s, p->b, p->z, U, V, bp, bl);
    return hipGetLastError() == hipSuccess ? POBA_OK : POBA_ERR_HIP;
}

}  // extern "C"
