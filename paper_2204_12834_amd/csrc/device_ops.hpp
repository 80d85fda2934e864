// Device building blocks shared by the passes: the landmark-tile iteration with
// its segmented reduction, deterministic block and grid reductions, and the
// small symmetric block inverses.
#pragma once

#include "camera_model.hpp"
#include "common.hpp"

namespace poba {

// ------------------------------------------------------ observation blocks --

// The 24 block scalars of observation i of one order in arithmetic TC: the
// stored blocks (POINT = false, storage TJ), or the blocks rebuilt from the
// point record (storage TJ) and the camera record of the linearisation.
template <typename TJ, bool POINT>
struct Rec {
    template <typename TC>
    __device__ __forceinline__ static void jac(const Buffers& b, const Sizes& z, const void* base, int64_t i,
                                               int64_t cam, TC* J) {
        if constexpr (POINT) {
            TC P[3], sw;
            load_point<TJ, TC>(base, z.npad, i, P, sw);
            point_jacobian<TC>(b.lin_rec + kCamRec * cam, P, sw, J);
        } else {
            load_J<TJ, TC>(base, z.npad, i, J);
        }
    }
};

// Per-camera data of the point-record landmark pass for the camera vector v
// (24 slots): a = J_l(w) v_w, e = v_t - a x t, v_intrinsics, f, k1, k2, R.
// Cameras are kFoldStride values apart: 28 floats (112 bytes) or 26 doubles
// (208 bytes), 4 x an odd number of 4-byte words, so that the 16-byte LDS
// reads of lanes with different cameras start on all the banks that a
// 16-byte access can start on (with 24 values only a quarter or half of them).
template <typename TS>
constexpr int kFoldStride = sizeof(TS) == 4 ? 28 : 26;
// With them J_p v = J_P (a x P + e) + p (d v_f + f n v_k1 + f n^2 v_k2).
template <typename TS>
__device__ __forceinline__ void fold_camera(const double* rec, const double* v, TS* out) {
    const double w0 = rec[0], w1 = rec[1], w2 = rec[2];
    const double B = rec[10], E = rec[22];
    const double th2 = w0 * w0 + w1 * w1 + w2 * w2;
    const double ww[3] = {w0, w1, w2};
    const double W[3][3] = {{0.0, -w2, w1}, {w2, 0.0, -w0}, {-w1, w0, 0.0}};
    double a[3];
    for (int i = 0; i < 3; ++i) {
        double s = 0.0;
        for (int j = 0; j < 3; ++j) {
            const double jl = (i == j ? 1.0 - E * th2 : 0.0) + B * W[i][j] + E * ww[i] * ww[j];
            s += jl * v[j];
        }
        a[i] = s;
    }
    const double t0 = rec[3], t1 = rec[4], t2 = rec[5];
    out[0] = TS(a[0]);
    out[1] = TS(a[1]);
    out[2] = TS(a[2]);
    out[3] = TS(v[3] - (a[1] * t2 - a[2] * t1));
    out[4] = TS(v[4] - (a[2] * t0 - a[0] * t2));
    out[5] = TS(v[5] - (a[0] * t1 - a[1] * t0));
    out[6] = TS(v[6]);
    out[7] = TS(v[7]);
    out[8] = TS(v[8]);
    out[9] = TS(rec[6]);
    out[10] = TS(rec[7]);
    out[11] = TS(rec[8]);
    for (int k = 0; k < 9; ++k) out[12 + k] = TS(rec[13 + k]);
    out[21] = out[22] = out[23] = TS(0);
}

// Shape factors of a camera-frame point shared by the point-record passes:
// iz = 1 / P_z, p = -P_xy iz, n = |p|^2, d = 1 + k1 n + k2 n^2 and
// A = dpi/dp = f (d I + 2 (k1 + 2 k2 n) p p^T).
template <typename T>
struct PointShape {
    T iz, p0, p1, n, d, A00, A01, A11;
    __device__ __forceinline__ PointShape(const T* P, T f, T k1, T k2) {
        // float32: the hardware reciprocal (1 ulp) instead of a correctly
        // rounded division
        if constexpr (sizeof(T) == 4) iz = __builtin_amdgcn_rcpf(P[2]);
        else iz = T(1) / P[2];
        p0 = -P[0] * iz;
        p1 = -P[1] * iz;
        n = p0 * p0 + p1 * p1;
        d = T(1) + k1 * n + k2 * n * n;
        const T dd = T(2) * (k1 + T(2) * k2 * n);
        A00 = f * (d + dd * p0 * p0);
        A01 = f * dd * p0 * p1;
        A11 = f * (d + dd * p1 * p1);
    }
    // J_P y (2) for a camera-frame vector y (3)
    __device__ __forceinline__ void JP(const T* y, T& z0, T& z1) const {
        const T u0 = y[0] + p0 * y[2], u1 = y[1] + p1 * y[2];
        z0 = -iz * (A00 * u0 + A01 * u1);
        z1 = -iz * (A01 * u0 + A11 * u1);
    }
    // J_P^T z (3)
    __device__ __forceinline__ void JPt(T z0, T z1, T* h) const {
        const T y0 = A00 * z0 + A01 * z1, y1 = A01 * z0 + A11 * z1;
        h[0] = -iz * y0;
        h[1] = -iz * y1;
        h[2] = -iz * (p0 * y0 + p1 * y1);
    }
};

// One observation's record words as loaded (unpacked to the arithmetic type
// only where they are used, so that no instruction touches a load in flight).
template <typename TJ>
struct RawRec;
template <>
struct RawRec<double> {
    d2v g[12];
};
template <>
struct RawRec<float> {
    f4v g[6];
};
template <>
struct RawRec<bf16_t> {
    u4v g[3];
};

template <typename TJ>
__device__ __forceinline__ void load_raw(const void* base, int64_t npad, int64_t i, RawRec<TJ>& r) {
    using G = typename std::remove_reference<decltype(r.g[0])>::type;
    const G* p = reinterpret_cast<const G*>(base);
    constexpr int n = sizeof(r.g) / sizeof(r.g[0]);
#pragma unroll
    for (int g = 0; g < n; ++g) r.g[g] = __builtin_nontemporal_load(&p[g * npad + i]);
}

template <typename TC>
__device__ __forceinline__ void unpack(const RawRec<double>& r, TC* v) {
#pragma unroll
    for (int g = 0; g < 12; ++g) {
        v[2 * g] = TC(r.g[g].x);
        v[2 * g + 1] = TC(r.g[g].y);
    }
}
template <typename TC>
__device__ __forceinline__ void unpack(const RawRec<float>& r, TC* v) {
#pragma unroll
    for (int g = 0; g < 6; ++g) {
        v[4 * g] = TC(r.g[g].x);
        v[4 * g + 1] = TC(r.g[g].y);
        v[4 * g + 2] = TC(r.g[g].z);
        v[4 * g + 3] = TC(r.g[g].w);
    }
}
template <typename TC>
__device__ __forceinline__ void unpack(const RawRec<bf16_t>& r, TC* v) {
#pragma unroll
    for (int g = 0; g < 3; ++g) {
        const uint32_t w4[4] = {r.g[g].x, r.g[g].y, r.g[g].z, r.g[g].w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[8 * g + 2 * k] = TC(bf16_to_float(uint16_t(w4[k] & 0xffffu)));
            v[8 * g + 2 * k + 1] = TC(bf16_to_float(uint16_t(w4[k] >> 16)));
        }
    }
}

// ------------------------------------------------------ landmark-tile loop --
//
// One wavefront walks the landmark-major positions of its tile in chunks of
// 64.  `obs(i, valid, cam, seg, l, v)` fills K values for position i (zero
// when !valid); seg indexes the non-empty-landmark list nel of the landmark l
// owning i.  A segmented inclusive scan over the chunk (carrying the open
// segment into the next chunk) leaves every landmark's total in its last
// position, where `tail(seg, l, v)` is called.  No other wavefront touches the
// tile's landmarks.
//
// The segments that can start in a chunk are the 64 after the open one, so
// every lane loads one entry of that window of nel together with its camera
// word and takes its own landmark from the window by a lane shuffle: the
// landmark gather then waits on one load instead of two in a row.  A tile
// starts at a head, so its first chunk never needs the open segment's
// landmark; later chunks take it from the previous chunk's last lane.  Lanes
// past the end get the chunk's last segment, so every lane holds a valid
// landmark index (window entries at or past the number of non-empty landmarks
// are read, clamped to the array, but never selected).  The lookup mode says
// when the landmark is taken (`obs` gets l = 0 unless it is kLookupEarly):
//   kLookupEarly: before `obs`, which needs it;
//   kLookupLate:  after `obs`, so that a kernel whose per-observation step
//                 does not need it issues that step's loads before it waits
//                 for the window;
//   kLookupTail:  no window: the tail lanes read nel at their segment.
// Which one is fastest depends on the kernel (measured per kernel).
enum TileLookup { kLookupEarly = 0, kLookupLate = 1, kLookupTail = 2 };
template <typename T, int K, int LOOKUP = kLookupEarly, typename Obs, typename Tail>
__device__ __forceinline__ void tile_landmarks(const uint32_t* __restrict__ lo_cam, const int32_t* __restrict__ tile_start,
                                               const int32_t* __restrict__ seg_base, const int32_t* __restrict__ nel,
                                               int32_t nl, int64_t tile, Obs&& obs, Tail&& tail) {
    const int lane = lane_id();
    const int32_t start = tile_start[tile];
    const int32_t end = tile_start[tile + 1];
    int32_t seg = seg_base[tile] - 1;  // segment open at the chunk start
    int32_t l_open = 0;                // its landmark (unused in the first chunk)
    T carry[K];
#pragma unroll
    for (int k = 0; k < K; ++k) carry[k] = T(0);
    for (int32_t base = start; base < end; base += kWave) {
        const int32_t i = base + lane;
        const bool valid = i < end;
        const uint32_t w = valid ? lo_cam[i] : 0u;
        const int32_t lw = LOOKUP == kLookupTail ? 0 : nel[min(seg + 1 + lane, nl - 1)];
        const bool head = valid && (w & kHeadBit);
        const uint64_t hm = ballot64(head);
        const uint64_t hu = hm & mask_upto(lane);
        const int seg_start = hu ? 63 - __builtin_clzll(hu) : 0;
        const int nh = __popcll(hu);
        const int32_t my_seg = seg + nh;
        auto pick = [&]() {
            const int32_t lk = __shfl(lw, nh > 0 ? nh - 1 : 0, kWave);
            return nh > 0 ? lk : l_open;
        };
        int32_t l = 0;
        if constexpr (LOOKUP == kLookupEarly) l = pick();
        T v[K];
        obs(i, valid, int32_t(w & kIndexMask), my_seg, l, v);
        if constexpr (LOOKUP == kLookupLate) l = pick();
        if (lane == 0 && !head) {
#pragma unroll
            for (int k = 0; k < K; ++k) v[k] += carry[k];
        }
        segmented_scan<T, K>(v, lane, seg_start);
        const int last = min(end - base, kWave) - 1;
        if (w & kTailBit) tail(my_seg, LOOKUP == kLookupTail ? nel[my_seg] : l, v);
#pragma unroll
        for (int k = 0; k < K; ++k) carry[k] = readlane(v[k], last);
        if constexpr (LOOKUP != kLookupTail) l_open = readlane(l, last);
        seg += __popcll(hm);
    }
}

// ------------------------------------------- landmark-major stream (pipelined) --
//
// The tile loop for kernels whose per-position work needs the landmark's
// position X and the observation (the landmark-major linearisation): one
// wavefront walks the tiles [t0, t1) as one stream of 64-position chunks (a
// range of whole tiles starts at a landmark head, and the open segment is
// carried across chunks and tiles as in the tile loop).  Three chunks are in
// flight: while chunk c is evaluated, the landmark positions of chunk c + 1
// have been requested, and the loads of chunk c + 2 that need nothing of
// earlier chunks (camera words, observations, the window of the
// non-empty-landmark list) too; a chunk then waits only for what its own work
// gathers from L2 (the camera record).
// obs(i, valid, cam, X, ox, oy, v) fills K values (zero when !valid);
// tail(seg, l, v) runs at each landmark's last position.
template <int K, typename Obs, typename Tail>
__device__ __forceinline__ void lm_tile_stream(const uint32_t* __restrict__ lo_cam,
                                               const int32_t* __restrict__ tile_start,
                                               const int32_t* __restrict__ seg_base, const int32_t* __restrict__ nel,
                                               const double* __restrict__ obs_lo, const double* __restrict__ lms,
                                               int32_t nl, int64_t t0, int64_t t1, Obs&& obs, Tail&& tail) {
    const int lane = lane_id();
    const int32_t start = tile_start[t0];
    const int32_t end = tile_start[t1];
    if (start >= end) return;
    // raw loads of a chunk (camera word, observation, window entry)
    struct Raw {
        uint32_t w;
        double ox, oy;
        int32_t lw;
    };
    auto fetch = [&](int32_t base, int32_t seg_open, Raw& r) {
        const int32_t i = min(base + lane, end - 1);  // lanes past the end read the last position
        r.w = lo_cam[i];
        r.ox = obs_lo[2 * int64_t(i)];
        r.oy = obs_lo[2 * int64_t(i) + 1];
        r.lw = nel[min(seg_open + 1 + lane, nl - 1)];
    };
    // a located chunk: its heads, each position's landmark and that landmark's position
    struct Loc {
        uint64_t hm;
        int32_t l;
        double X[3];
    };
    auto locate = [&](int32_t base, const Raw& r, int32_t l_prev, Loc& c) {
        const bool head = base + lane < end && (r.w & kHeadBit);
        c.hm = ballot64(head);
        const int nh = __popcll(c.hm & mask_upto(lane));
        const int32_t lk = __shfl(r.lw, nh > 0 ? nh - 1 : 0, kWave);
        c.l = nh > 0 ? lk : l_prev;
#pragma unroll
        for (int k = 0; k < 3; ++k) c.X[k] = lms[3 * int64_t(c.l) + k];
    };
    int32_t seg = seg_base[t0] - 1;  // segment open at the start of the current chunk
    Raw rc, rn;
    Loc cur;
    fetch(start, seg, rc);
    locate(start, rc, 0, cur);  // a range starts at a head: l_prev is never taken
    const bool two = start + kWave < end;
    if (two) fetch(start + kWave, seg + int32_t(__popcll(cur.hm)), rn);
    double carry[K];
#pragma unroll
    for (int k = 0; k < K; ++k) carry[k] = 0.0;
    for (int32_t base = start; base < end; base += kWave) {
        const int32_t i = base + lane;
        const bool valid = i < end;
        const uint32_t wc = valid ? rc.w : 0u;
        const int last = min(end - base, kWave) - 1;
        const int32_t seg_next = seg + int32_t(__popcll(cur.hm));
        // chunk c + 1: landmarks requested; chunk c + 2: raw loads requested
        const bool more = base + kWave < end;
        Loc nxt;
        Raw rn2;
        if (more) {
            locate(base + kWave, rn, readlane(cur.l, last), nxt);
            if (base + 2 * kWave < end) fetch(base + 2 * kWave, seg_next + int32_t(__popcll(nxt.hm)), rn2);
        }
        double v[K];
        obs(i, valid, int32_t(wc & kIndexMask), cur.X, rc.ox, rc.oy, v);
        if (lane == 0 && !(wc & kHeadBit)) {
#pragma unroll
            for (int k = 0; k < K; ++k) v[k] += carry[k];
        }
        const uint64_t hu = cur.hm & mask_upto(lane);
        const int seg_start = hu ? 63 - __builtin_clzll(hu) : 0;
        segmented_scan<double, K>(v, lane, seg_start);
        if (wc & kTailBit) tail(seg + int32_t(__popcll(hu)), cur.l, v);
#pragma unroll
        for (int k = 0; k < K; ++k) carry[k] = readlane(v[k], last);
        seg = seg_next;
        if (more) {
            rc = rn;
            cur = nxt;
            rn = rn2;
        }
    }
}

// --------------------------------------------------------- block reductions --

// Sum of K values over the block; the result is valid in thread 0.  lds holds
// kWavesPerBlock * K doubles.
template <int K>
__device__ __forceinline__ void block_sum(double* v, double* lds) {
    wave_total_last<K>(v);
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int nw = blockDim.x / kWave;
    if (lane == kWave - 1) {
#pragma unroll
        for (int k = 0; k < K; ++k) lds[w * K + k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double s = 0.0;
            for (int j = 0; j < nw; ++j) s += lds[j * K + k];
            v[k] = s;
        }
    }
    __syncthreads();
}

// Block totals (thread 0's v) to the block's slot of a partials array; a
// later single-block kernel combines them (kernel boundaries order the
// writes, so no device-scope fence is needed inside the producing kernel).
template <int K>
__device__ __forceinline__ void store_block_partial(const double* v, double* partials) {
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) partials[size_t(blockIdx.x) * K + k] = v[k];
    }
}

// Single-block sum of the first K entries of n partial records (record q at
// partials[q * stride]) in record order, with compensated (TwoSum)
// per-thread accumulation; the totals are valid in thread 0.  Each thread
// requests its next kSumAhead records before adding them (in the same order),
// so their loads are in flight together instead of one round trip each.
constexpr int kSumAhead = 8;

template <int K>
__device__ __forceinline__ void sum_partials(const double* partials, uint32_t n, double* out, double* lds,
                                             int stride = K) {
    double s[K], e[K];
#pragma unroll
    for (int k = 0; k < K; ++k) s[k] = e[k] = 0.0;
    for (uint32_t i0 = threadIdx.x; i0 < n; i0 += kSumAhead * blockDim.x) {
        double v[kSumAhead][K];
#pragma unroll
        for (int u = 0; u < kSumAhead; ++u) {
            const uint32_t i = i0 + uint32_t(u) * blockDim.x;
#pragma unroll
            for (int k = 0; k < K; ++k) v[u][k] = i < n ? partials[size_t(i) * stride + k] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kSumAhead; ++u) {
            if (i0 + uint32_t(u) * blockDim.x >= n) break;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                double t, err;
                two_sum(s[k], v[u][k], t, err);
                s[k] = t;
                e[k] += err;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) s[k] += e[k];
    block_sum<K>(s, lds);
#pragma unroll
    for (int k = 0; k < K; ++k) out[k] = s[k];
}

constexpr int kReduceBlock = 1024;

// -------------------------------------------------------- small inverses --

// Damping diagonal of one block entry (Sec. 4.1 D^T D): Marquardt uses the
// clamped diagonal of J^T J, identity uses 1.
__device__ __forceinline__ double damp_diag(double diag, int damping) {
    return damping == POBA_DAMP_MARQUARDT ? fmin(fmax(diag, 1e-6), 1e32) : 1.0;
}

// Damping diagonal of a packed 3x3 block (entries 0, 3, 5 are the diagonal).
__device__ __forceinline__ void damp_diag3(const double* V, int damping, double* dd) {
    dd[0] = damp_diag(V[0], damping);
    dd[1] = damp_diag(V[3], damping);
    dd[2] = damp_diag(V[5], damping);
}

// Inverse of the damped 3x3 block V + lambda diag(dd) (packed 00 01 02 11 12
// 22) by Cholesky; returns false (and the inverse of the damping diagonal) if
// a pivot is not positive.
__device__ __forceinline__ bool inv3_damped(const double* V, double lam, const double* dd, double* out) {
    const double d0 = dd[0], d1 = dd[1], d2 = dd[2];
    const double a00 = V[0] + lam * d0, a01 = V[1], a02 = V[2];
    const double a11 = V[3] + lam * d1, a12 = V[4], a22 = V[5] + lam * d2;
    bool ok = a00 > 0.0;
    const double l00 = sqrt(a00);
    const double l10 = a01 / l00, l20 = a02 / l00;
    const double q11 = a11 - l10 * l10;
    ok = ok && q11 > 0.0;
    const double l11 = sqrt(q11);
    const double l21 = (a12 - l20 * l10) / l11;
    const double q22 = a22 - l20 * l20 - l21 * l21;
    ok = ok && q22 > 0.0;
    const double l22 = sqrt(q22);
    // M = L^-1 (lower)
    const double m00 = 1.0 / l00, m11 = 1.0 / l11, m22 = 1.0 / l22;
    const double m10 = -l10 * m00 * m11;
    const double m21 = -l21 * m11 * m22;
    const double m20 = -(l20 * m00 + l21 * m10) * m22;
    // inverse = M^T M
    out[0] = m00 * m00 + m10 * m10 + m20 * m20;
    out[1] = m10 * m11 + m20 * m21;
    out[2] = m20 * m22;
    out[3] = m11 * m11 + m21 * m21;
    out[4] = m21 * m22;
    out[5] = m22 * m22;
    ok = ok && isfinite(out[0]) && isfinite(out[3]) && isfinite(out[5]);
    if (!ok) {
        const double e0 = lam * d0, e1 = lam * d1, e2 = lam * d2;
        out[0] = e0 > 0.0 ? 1.0 / e0 : 0.0;
        out[1] = out[2] = out[4] = 0.0;
        out[3] = e1 > 0.0 ? 1.0 / e1 : 0.0;
        out[5] = e2 > 0.0 ? 1.0 / e2 : 0.0;
    }
    return ok;
}

// Inverse of a symmetric positive definite 9x9 matrix in float64 by Cholesky
// factorisation A = L L^T and A^-1 = L^-T L^-1.  L holds A (row-major) on
// entry and its factor on return; out receives the 81 entries of A^-1.
// Returns false if a pivot is not positive or an entry is not finite.
__device__ __forceinline__ bool spd_inverse9(double* L, double* out) {
    bool ok = true;
#pragma unroll
    for (int j = 0; j < 9; ++j) {
        double d = L[9 * j + j];
#pragma unroll
        for (int k = 0; k < j; ++k) d -= L[9 * j + k] * L[9 * j + k];
        ok = ok && d > 0.0;
        const double ljj = sqrt(d);
        L[9 * j + j] = ljj;
#pragma unroll
        for (int i = j + 1; i < 9; ++i) {
            double sacc = L[9 * i + j];
#pragma unroll
            for (int k = 0; k < j; ++k) sacc -= L[9 * i + k] * L[9 * j + k];
            L[9 * i + j] = sacc / ljj;
        }
    }
    double M[81];  // L^-1, lower
#pragma unroll
    for (int k = 0; k < 81; ++k) M[k] = 0.0;
#pragma unroll
    for (int j = 0; j < 9; ++j) {
        M[9 * j + j] = 1.0 / L[9 * j + j];
#pragma unroll
        for (int i = j + 1; i < 9; ++i) {
            double sacc = 0.0;
#pragma unroll
            for (int k = j; k < i; ++k) sacc -= L[9 * i + k] * M[9 * k + j];
            M[9 * i + j] = sacc / L[9 * i + i];
        }
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) {
#pragma unroll
        for (int j = i; j < 9; ++j) {
            double sacc = 0.0;
#pragma unroll
            for (int k = j; k < 9; ++k) sacc += M[9 * k + i] * M[9 * k + j];
            ok = ok && isfinite(sacc);
            out[9 * i + j] = sacc;
            out[9 * j + i] = sacc;
        }
    }
    return ok;
}

template <typename T>
__device__ __forceinline__ void sym3_apply(const T* A, const T* x, T* y) {
    y[0] = A[0] * x[0] + A[1] * x[1] + A[2] * x[2];
    y[1] = A[1] * x[0] + A[3] * x[1] + A[4] * x[2];
    y[2] = A[2] * x[0] + A[4] * x[1] + A[5] * x[2];
}

}  // namespace poba
