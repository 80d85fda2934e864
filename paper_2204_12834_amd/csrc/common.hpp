// Shared definitions of the gfx950 power-series bundle-adjustment library:
// the problem handle, the workspace layout, storage types and wave helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <type_traits>

#include <cstdint>
#include <cstring>
#include <vector>

#include "poba.h"

namespace poba {
using Problem = ::poba_problem_s;

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kDefaultPiece = 1024;
constexpr int kXcds = 8;                      // dies of an MI355X; workgroups are dealt to them in turn
constexpr int64_t kRangeBytes = 2ll << 20;   // landmark-vector slice gathered by one die
constexpr int64_t kRangeLds = 144 << 10;     // landmark-vector slice per range when staged in LDS (target)
constexpr int64_t kRangeLdsMax = 156 << 10;  // the same, upper bound (one workgroup per compute unit)
constexpr int kMaxCwWaves = 16;              // wavefronts per workgroup of the range-staged camera pass (max)
constexpr int kMaxRangeBlocks = 16;          // workgroups per landmark range in that pass

// Wavefronts per workgroup of the range-staged camera pass: 16 with float32
// arithmetic, 8 with float64 (whose registers allow two waves per SIMD).
inline constexpr int range_pass_waves(int sbytes) { return sbytes == 8 ? 8 : 16; }
// Lanes per group in a batch of that pass, and groups per batch.  With groups
// of about 70 observations (the city workload), sets of 16 take 13% fewer
// steps per wavefront than sets of 8: fewer idle lanes in each batch's
// longest group.
constexpr int kSetLanes = 16;
constexpr int kSets = 64 / kSetLanes;
constexpr uint32_t kHeadBit = 0x80000000u;  // first observation of its landmark
constexpr uint32_t kTailBit = 0x40000000u;  // last observation of its landmark
constexpr uint32_t kIndexMask = 0x3fffffffu;
constexpr int kMaxProfiled = 65536;

// ---------------------------------------------------------------- storage --

// bfloat16 payload (upper half of a float32).
struct bf16_t {
    uint16_t bits;
};

__host__ __device__ inline float bf16_to_float(uint16_t b) {
    uint32_t u = uint32_t(b) << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

__host__ __device__ inline uint16_t float_to_bf16(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return uint16_t((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
    return uint16_t(u >> 16);
}

// Per-observation Jacobian record: 24 scalars, J_p row 0 (9), J_p row 1 (9),
// J_l row 0 (3), J_l row 1 (3).  Stored structure-of-arrays in 16-byte groups:
// group g of observation i lives at byte (g * npad + i) * 16.
template <typename TJ>
struct JLayout;
template <>
struct JLayout<double> {
    static constexpr int kPerGroup = 2;
    static constexpr int kGroups = 12;
};
template <>
struct JLayout<float> {
    static constexpr int kPerGroup = 4;
    static constexpr int kGroups = 6;
};
template <>
struct JLayout<bf16_t> {
    static constexpr int kPerGroup = 8;
    static constexpr int kGroups = 3;
};

template <typename TJ>
__device__ __forceinline__ void store_J(void* base, int64_t npad, int64_t i, const double* v);

template <>
__device__ __forceinline__ void store_J<double>(void* base, int64_t npad, int64_t i, const double* v) {
    double2* b = reinterpret_cast<double2*>(base);
#pragma unroll
    for (int g = 0; g < 12; ++g) b[g * npad + i] = make_double2(v[2 * g], v[2 * g + 1]);
}
template <>
__device__ __forceinline__ void store_J<float>(void* base, int64_t npad, int64_t i, const double* v) {
    float4* b = reinterpret_cast<float4*>(base);
#pragma unroll
    for (int g = 0; g < 6; ++g)
        b[g * npad + i] = make_float4(float(v[4 * g]), float(v[4 * g + 1]), float(v[4 * g + 2]), float(v[4 * g + 3]));
}
template <>
__device__ __forceinline__ void store_J<bf16_t>(void* base, int64_t npad, int64_t i, const double* v) {
    uint4* b = reinterpret_cast<uint4*>(base);
#pragma unroll
    for (int g = 0; g < 3; ++g) {
        uint32_t w[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            uint32_t lo = float_to_bf16(float(v[8 * g + 2 * k]));
            uint32_t hi = float_to_bf16(float(v[8 * g + 2 * k + 1]));
            w[k] = lo | (hi << 16);
        }
        b[g * npad + i] = make_uint4(w[0], w[1], w[2], w[3]);
    }
}

// Stores blocks computed in float32 arithmetic (float32 storage).
__device__ __forceinline__ void store_J_f32(void* base, int64_t npad, int64_t i, const float* v) {
    float4* b = reinterpret_cast<float4*>(base);
#pragma unroll
    for (int g = 0; g < 6; ++g) b[g * npad + i] = make_float4(v[4 * g], v[4 * g + 1], v[4 * g + 2], v[4 * g + 3]);
}

// Rounds a record to the storage type and back (the values every pass sees).
template <typename TJ>
__device__ __forceinline__ double round_to_storage(double v);
template <>
__device__ __forceinline__ double round_to_storage<double>(double v) { return v; }
template <>
__device__ __forceinline__ double round_to_storage<float>(double v) { return double(float(v)); }
template <>
__device__ __forceinline__ double round_to_storage<bf16_t>(double v) {
    return double(bf16_to_float(float_to_bf16(float(v))));
}

template <typename TJ, typename TC>
__device__ __forceinline__ void load_J(const void* base, int64_t npad, int64_t i, TC* v);

typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));

template <typename TC>
__device__ __forceinline__ void load_J_d(const void* base, int64_t npad, int64_t i, TC* v) {
    const d2v* b = reinterpret_cast<const d2v*>(base);
#pragma unroll
    for (int g = 0; g < 12; ++g) {
        d2v x = __builtin_nontemporal_load(&b[g * npad + i]);
        v[2 * g] = TC(x.x);
        v[2 * g + 1] = TC(x.y);
    }
}
template <typename TC>
__device__ __forceinline__ void load_J_f(const void* base, int64_t npad, int64_t i, TC* v) {
    const f4v* b = reinterpret_cast<const f4v*>(base);
#pragma unroll
    for (int g = 0; g < 6; ++g) {
        f4v x = __builtin_nontemporal_load(&b[g * npad + i]);
        v[4 * g] = TC(x.x);
        v[4 * g + 1] = TC(x.y);
        v[4 * g + 2] = TC(x.z);
        v[4 * g + 3] = TC(x.w);
    }
}
template <typename TC>
__device__ __forceinline__ void load_J_b(const void* base, int64_t npad, int64_t i, TC* v) {
    const u4v* b = reinterpret_cast<const u4v*>(base);
#pragma unroll
    for (int g = 0; g < 3; ++g) {
        u4v x = __builtin_nontemporal_load(&b[g * npad + i]);
        uint32_t w[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[8 * g + 2 * k] = TC(bf16_to_float(uint16_t(w[k] & 0xffffu)));
            v[8 * g + 2 * k + 1] = TC(bf16_to_float(uint16_t(w[k] >> 16)));
        }
    }
}
template <>
__device__ __forceinline__ void load_J<double, double>(const void* b, int64_t n, int64_t i, double* v) { load_J_d(b, n, i, v); }
template <>
__device__ __forceinline__ void load_J<float, float>(const void* b, int64_t n, int64_t i, float* v) { load_J_f(b, n, i, v); }
template <>
__device__ __forceinline__ void load_J<float, double>(const void* b, int64_t n, int64_t i, double* v) { load_J_f(b, n, i, v); }
template <>
__device__ __forceinline__ void load_J<bf16_t, float>(const void* b, int64_t n, int64_t i, float* v) { load_J_b(b, n, i, v); }
template <>
__device__ __forceinline__ void load_J<bf16_t, double>(const void* b, int64_t n, int64_t i, double* v) { load_J_b(b, n, i, v); }

// Point record of an observation: (P_x, P_y, P_z, sqrt(w)).  float32: one
// 16-byte group at byte i * 16; float64: two groups (P_x, P_y), (P_z, sqrt(w))
// at (g * npad + i) * 16.
template <typename TP>
__device__ __forceinline__ void store_point(void* base, int64_t npad, int64_t i, const double* P, double sw);
template <>
__device__ __forceinline__ void store_point<float>(void* base, int64_t, int64_t i, const double* P, double sw) {
    reinterpret_cast<float4*>(base)[i] = make_float4(float(P[0]), float(P[1]), float(P[2]), float(sw));
}
template <>
__device__ __forceinline__ void store_point<double>(void* base, int64_t npad, int64_t i, const double* P, double sw) {
    double2* b = reinterpret_cast<double2*>(base);
    b[i] = make_double2(P[0], P[1]);
    b[npad + i] = make_double2(P[2], sw);
}

template <typename TP, typename TC>
__device__ __forceinline__ void load_point(const void* base, int64_t npad, int64_t i, TC* P, TC& sw);
template <>
__device__ __forceinline__ void load_point<float, float>(const void* base, int64_t, int64_t i, float* P, float& sw) {
    const f4v x = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(base) + i);
    P[0] = x.x; P[1] = x.y; P[2] = x.z; sw = x.w;
}
template <>
__device__ __forceinline__ void load_point<float, double>(const void* base, int64_t, int64_t i, double* P,
                                                          double& sw) {
    const f4v x = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(base) + i);
    P[0] = x.x; P[1] = x.y; P[2] = x.z; sw = x.w;
}
template <>
__device__ __forceinline__ void load_point<double, double>(const void* base, int64_t npad, int64_t i, double* P,
                                                           double& sw) {
    const d2v* b = reinterpret_cast<const d2v*>(base);
    const d2v a = __builtin_nontemporal_load(b + i);
    const d2v c = __builtin_nontemporal_load(b + npad + i);
    P[0] = a.x; P[1] = a.y; P[2] = c.x; sw = c.y;
}

// Rounds a value to the point-record type and back.
template <typename TP>
__device__ __forceinline__ double round_point(double v) { return double(TP(v)); }

// ------------------------------------------------------------ wave helpers --

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Index of the calling wavefront in its workgroup, as a wave-uniform value
// (scalar register), so that per-wavefront records, loop bounds and cursors
// derived from it stay scalar.
__device__ __forceinline__ int wave_in_block() { return __builtin_amdgcn_readfirstlane(int(threadIdx.x) / kWave); }

__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }

// Mask of lanes 0..lane inclusive.
__device__ __forceinline__ uint64_t mask_upto(int lane) {
    return lane == 63 ? ~0ull : ((1ull << (lane + 1)) - 1ull);
}

// Lane exchange through the DPP crossbar (no LDS): a 32-bit word of another
// lane chosen by the DPP control; rows outside row_mask keep `old`.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_f32(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROW_MASK, 0xf,
                                                                  false));
}
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double v) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_update_dpp(0, int(uint32_t(u)), CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, int(uint32_t(u >> 32)), CTRL, ROW_MASK, 0xf, false);
    return __builtin_bit_cast(double, (uint64_t(uint32_t(hi)) << 32) | uint32_t(lo));
}
template <int CTRL, int ROW_MASK, typename T>
__device__ __forceinline__ T dpp(T v) {
    if constexpr (sizeof(T) == 8) return dpp_f64<CTRL, ROW_MASK>(v);
    else return dpp_f32<CTRL, ROW_MASK>(v);
}

// The same exchange for callers that never read the lanes the control does
// not write (their value is unspecified): no register has to be cleared first.
template <int CTRL, int ROW_MASK, typename T>
__device__ __forceinline__ T dpp_masked(T v) {
    if constexpr (sizeof(T) == 8) {
        const uint64_t u = __builtin_bit_cast(uint64_t, v);
        const int lo = __builtin_amdgcn_mov_dpp(int(uint32_t(u)), CTRL, ROW_MASK, 0xf, false);
        const int hi = __builtin_amdgcn_mov_dpp(int(uint32_t(u >> 32)), CTRL, ROW_MASK, 0xf, false);
        return __builtin_bit_cast(double, (uint64_t(uint32_t(hi)) << 32) | uint32_t(lo));
    } else {
        return __builtin_bit_cast(T, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, ROW_MASK, 0xf, false));
    }
}

// Copies n 16-byte units from global memory to LDS (dst, from the block's
// dynamic LDS) with the global-to-LDS load: each instruction moves one
// contiguous KB per wavefront (lane i to the wavefront's LDS base + 16 i), no
// registers hold the data, so every unit of the copy is in flight at once.
// Ends with the block synchronised and the data visible to every wavefront.
// blockDim.x must be a multiple of the wavefront size.
__device__ __forceinline__ void copy_to_lds(const uint4* __restrict__ src, uint4* dst, int64_t n) {
    const int64_t wave_base = int64_t(threadIdx.x) - lane_id();
    for (int64_t k = threadIdx.x; k < n; k += blockDim.x)
        __builtin_amdgcn_global_load_lds(src + k, dst + (k - threadIdx.x + wave_base), 16, 0, 0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
}

// v plus the value of v D lanes lower in its row of 16 (DPP row_shr:D), for
// callers that use the result only in lanes with D <= lane % 16.  For 4-byte
// values the shift fills the other lanes with 0, which lets the compiler fold
// it into the add (one DPP add instead of a DPP move and an add).
template <int D, typename T>
__device__ __forceinline__ T dpp_row_shr_add(T v) {
    if constexpr (sizeof(T) == 8) {
        return v + dpp_masked<0x110 | D, 0xf>(v);
    } else {
        return v + __builtin_bit_cast(
                       T, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x110 | D, 0xf, 0xf, false));
    }
}

// Inclusive segmented scan over the wave.  seg_start is the first lane of the
// calling lane's segment; after the call v[k] holds the sum of v[k] over
// lanes seg_start..lane.  Within each row of 16 lanes the scan shifts by 1,
// 2, 4, 8 (DPP row_shr); the rows are then joined by broadcasting the last
// lane of row 0 into row 1 and of row 2 into row 3 (row_bcast:15), and of
// row 1 into rows 2 and 3 (row_bcast:31), each taken only by lanes whose
// segment reaches back past that lane.
template <typename T, int K>
__device__ __forceinline__ void segmented_scan(T* v, int lane, int seg_start) {
    const int rl = lane & 15;
#define POBA_ROW_STEP(D)                                                   \
    {                                                                      \
        const bool take = rl >= D && lane - D >= seg_start;                \
        _Pragma("unroll") for (int k = 0; k < K; ++k) {                    \
            const T y = dpp_row_shr_add<D>(v[k]);                          \
            if (take) v[k] = y;                                            \
        }                                                                  \
    }
    POBA_ROW_STEP(1)
    POBA_ROW_STEP(2)
    POBA_ROW_STEP(4)
    POBA_ROW_STEP(8)
#undef POBA_ROW_STEP
    {
        // rows 1 and 3 read lane 16 * row - 1, the lane before their row
        const bool take = (lane & 16) && seg_start < (lane & 48);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const T y = dpp_masked<0x142, 0xa>(v[k]);
            if (take) v[k] += y;
        }
    }
    {
        const bool take = lane >= 32 && seg_start <= 31;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const T y = dpp_masked<0x143, 0xc>(v[k]);
            if (take) v[k] += y;
        }
    }
}

// Sum of K values over the wavefront into its last lane (DPP shifts within
// rows of 16, then row broadcasts; the other lanes' results are not used).
template <int K>
__device__ __forceinline__ void wave_total_last(double* v) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
        v[k] += dpp_masked<0x111, 0xf>(v[k]);
        v[k] += dpp_masked<0x112, 0xf>(v[k]);
        v[k] += dpp_masked<0x114, 0xf>(v[k]);
        v[k] += dpp_masked<0x118, 0xf>(v[k]);
        v[k] += dpp_masked<0x142, 0xa>(v[k]);
        v[k] += dpp_masked<0x143, 0xc>(v[k]);
    }
}

// The value of x in lane l (l the same in every lane): a wave-uniform result,
// read without a trip through LDS.
__device__ __forceinline__ double readlane_f64(double x, int l) {
    const uint64_t u = __builtin_bit_cast(uint64_t, x);
    const uint32_t lo = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(u)), l));
    const uint32_t hi = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(u >> 32)), l));
    return __builtin_bit_cast(double, (uint64_t(hi) << 32) | lo);
}
template <typename T>
__device__ __forceinline__ T readlane(T x, int l) {
    if constexpr (sizeof(T) == 8) {
        return __builtin_bit_cast(T, readlane_f64(__builtin_bit_cast(double, x), l));
    } else {
        static_assert(sizeof(T) == 4, "4- or 8-byte values");
        return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), l));
    }
}

// Error-free sum (Knuth TwoSum) for compensated float64 accumulation.
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
    s = a + b;
    double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// ---------------------------------------------------------------- control --

// Device control of a handle: flags over all of its problems.  Kernels that
// cover every problem return early when no problem is active or when the
// series of every active problem has stopped.
struct Ctrl {
    int32_t active;   // number of problems the current call works on
    int32_t lin;      // 1 if the current lm step linearises
    int32_t running;  // active problems whose series has not stopped
    int32_t pad;
};

// Per-problem control (one per independent sub-problem of a batch).
struct PCtrl {
    double lambda;       // damping of the current solve
    double cost;         // F of the last linearisation
    double cost_new;     // F at the trial state
    double model;        // L(0) - L(dx)
    double norm_x2, norm_v2;
    int32_t active;      // 1 while the current call works on the problem
    int32_t stopped;     // series ended by the stop rule
    int32_t stop_order;  // last order summed
    int32_t status;      // OR of POBA_ERR_* bits
    int32_t accepted;    // last lm step accepted
    int32_t pad;
};

// Per-problem state of preconditioned conjugate gradients on the reduced
// camera system.
struct PcgCtl {
    double rz;          // r . z of the current residual
    double b2;          // |b|^2 of the right-hand side
    double r2;          // |r|^2 of the current residual
    double alpha, beta; // coefficients of the last iteration
    int32_t iterations; // iterations taken
    int32_t converged;  // |r| <= tol |b| reached
    int32_t pad[2];
};

// One camera-pass work item as a block reads it in a single request: the
// piece (-1: idle slot), its camera-major range, camera and problem.
struct alignas(32) PieceRec {
    int32_t p, begin, end, cam, prob, pad0, pad1, pad2;
};

// ---------------------------------------------------------------- handle --

struct Buffers {
    // observation orders
    int32_t* perm_l;      // [N] original index at each landmark-major position
    int32_t* perm_c;      // [N] original index at each camera-major position
    uint32_t* lo_cam;     // [N] camera at each landmark-major position | head bit | tail bit
    int32_t* co_lm;       // [N] landmark at each camera-major position
    int32_t* co_seg;      // [N] segment (rank among non-empty landmarks) at each camera-major position
    int32_t* lm_off;      // [nl+1]
    int32_t* cam_off;     // [nc+1]
    int32_t* nel;         // [nl] non-empty landmarks in order
    int32_t* tile_start;  // [ntiles+1] first landmark-major position of each 64-tile
    int32_t* seg_base;    // [ntiles] index into nel of each tile's first segment
    int32_t* piece_cam;   // [npieces_max]
    int32_t* piece_begin; // [npieces_max]
    int32_t* piece_end;   // [npieces_max]
    int32_t* piece_grp;   // [npieces_max] (camera, range) group of each piece
    int32_t* cam_piece;   // [nc+1] first piece of each camera
    int32_t* grp_off;     // [nc*R+1] camera-major offsets of the (camera, range) groups
    int32_t* grp_piece;   // [nc*R+1] first piece of each group
    int32_t* dgrp_off;    // [nc*8+1] camera-major offsets of the (camera, die) groups (point records, R % 8 == 0)
    int32_t* sched;       // [kXcds*npieces_max] camera-pass block -> piece (-1: idle)
    PieceRec* sched_rec;  // [kXcds*npieces_max] the same slots with their piece data
    int4* cw_rec;         // [R*kMaxRangeBlocks*kMaxCwWaves] range-staged camera pass: per wavefront
                          // {landmark range, list begin, list end, 0} into cw_list
    int4* cw_list;        // [R*nc] the non-empty (camera, range) groups of each wavefront:
                          // {camera, first camera-major position, length, problem}
    double* obs_lo;       // [N][2] observations, landmark-major
    double* obs_co;       // [N][2] observations, camera-major
    // linearisation
    void* J_lo;           // Jacobian records, landmark-major
    void* J_co;           // Jacobian records, camera-major
    double* r_co;         // [N][2] reweighted residual, camera-major
    double* U;            // [nc][81] undamped
    double* bp;           // [nc][9]
    double* V;            // [nl][6] undamped, packed (00 01 02 11 12 22)
    double* bl;           // [nl][3]
    // solve
    double* Uinv;         // [nc][81]
    double* Dp;           // [nc][9] damping diagonal of the last solve
    double* Dl;           // [nseg][3] damping diagonal of the last solve, by segment
    void* Vinv;           // [nseg][6] storage type, indexed by segment
    double* vinv64;       // [nseg][6] the same damped inverses in float64 (back-substitution)
    double* ybl;          // [nseg][4] V^-1 b_l in float64 and 1 (0 for a landmark of an inactive problem)
    void* s;              // [nseg][4] storage type (landmark vector of the series), by segment
    double* v;            // [nc][9] current series term
    void* vq;             // [nc][12] current term in storage type (gather copy), or its folded camera data
                          // at stride kFoldStride (point records)
    double* x;            // [nc][9] series sum
    double* bt;           // [nc][9] reduced right-hand side b~ of the last solve
    double* part;         // [npieces_max][54] per-piece partial sums
    void* part_grp;       // [nc][R][9] storage type: per (camera, range) group sums of the camera pass
    double* dxl;          // [nl][3] landmark step (lm step)
    double* dxp;          // [nc][9] camera step (lm step)
    double* cam_rec;      // [nc][24] camera records of the state being evaluated (trial state)
    double* lin_rec;      // [nc][24] camera records of the last linearisation
    double* cams_new;     // [nc][9]
    double* lm_trial;     // [nl][8] trial landmark x + dx_l (0..2) and its step dx_l (3..5), one 64-byte line
    double* piece_red;    // [npieces_max][3] per-piece partial sums (cost, model, flags)
    double* cam_red;      // [nc][2] per-camera squared norms of v and x
    double* xq;           // [nc][kFoldStride] folded camera data of the camera step (point-record back-substitution),
                          // or the camera step at stride 12 (Jacobian-record back-substitution)
    double* cg;           // [5][nc][9] conjugate-gradient vectors x, r, z, p, q
    double* sj;           // [nc][81] inverted diagonal blocks of S (Schur-Jacobi preconditioner)
    PcgCtl* pcg_ctl;      // [np]
    // independent problems: contiguous camera and landmark ranges
    int32_t* prob_cam_off;   // [np+1]
    int32_t* prob_lm_off;    // [np+1]
    int32_t* prob_piece_off; // [np+1] first camera piece of each problem
    int32_t* cam_prob;       // [nc] problem of each camera
    int32_t* lm_prob;        // [nl] problem of each landmark
    PCtrl* pctl;             // [np]

    Ctrl* ctrl;
    void* sort_tmp;       // radix-sort scratch
    size_t sort_tmp_bytes;
    int32_t* keys_tmp;    // [N]
    int32_t* vals_tmp;    // [N]
    int32_t* keys_out;    // [N]
    int32_t* iota;        // [N]
    int32_t* scratch_i;   // [max(nc, nl) + 2] set-up scratch; afterwards word 0 is the repeated-pair flag
};

struct Sizes {
    int32_t nc, nl;
    int32_t np;  // independent problems
    int64_t N, npad, ntiles, npieces_max, ranges_max;
    int piece;
    int jbytes;  // bytes per stored Jacobian scalar
    int sbytes;  // bytes per stored landmark-side scalar
    int point;   // 1: point records (P, sqrt(w)) instead of Jacobian blocks
    int rbytes;  // bytes of one observation's record
};

struct ProfileSlot {
    hipEvent_t start, stop;
    int cls;
};

}  // namespace poba

struct poba_problem_s {
    poba_desc d;
    poba::Sizes z;
    poba::Buffers b;
    int64_t npieces = 0;
    int64_t nnel = 0;
    int tiles_per_wave = 4;     // landmark-tile groups handled by one wavefront
    int32_t lm_ranges = 1;      // landmark ranges of the camera-major order
    int64_t sched_len = 0;      // camera-pass grid size
    int32_t seg_per_range = 1;  // non-empty landmarks per landmark range
    int range_lds_ok = 0;       // pieces and wave records of the range-staged camera pass exist
    int range_lds = 0;          // series camera passes over point records stage the ranges in LDS
    int64_t cw_blocks = 0;      // grid of the range-staged camera pass
    int64_t n_cus = 256;        // compute units of the device
    int lds_cam = 1;            // stage the camera vector in LDS when it fits
    int64_t lds_max = 65536;    // bytes of LDS one workgroup may allocate
    int damping_frozen = 0;     // solves reuse the damping diagonal of the last unfrozen solve
    int repeats = -1;           // some (camera, landmark) pair is observed twice (-1: not yet known)
    hipStream_t last_stream = nullptr;
    // profiling
    bool profiling = false;
    std::vector<poba::ProfileSlot> slots;
    size_t slot_used = 0;
    double prof_ms[POBA_K_COUNT] = {0};
    int64_t prof_n[POBA_K_COUNT] = {0};
};

namespace poba {
// Pieces averaging fewer observations than a workgroup of four wavefronts
// has lanes (cameras that see few landmarks per landmark range, as on the
// ladybug-shaped problem: about 50 per piece) leave most of such a workgroup
// idle; the per-piece kernels then run one wavefront per piece.
inline bool small_pieces(const Problem* p) { return p->npieces > 0 && p->z.N < int64_t(kBlock) * p->npieces; }
}  // namespace poba

namespace poba {

// Workspace layout (defined in setup.hip).
bool compute_sizes(const poba_desc* d, int32_t n_problems, Sizes* z);
size_t layout(const poba_desc* d, const Sizes& z, char* base, Buffers* b, size_t sort_tmp_bytes);
size_t sort_tmp_upper_bound(int64_t N);

// Launch bracketing for profiling.
void prof_begin(Problem* p, int cls, hipStream_t s, ProfileSlot** slot);
void prof_end(ProfileSlot* slot, hipStream_t s);

struct ProfScope {
    ProfileSlot* slot = nullptr;
    hipStream_t s;
    ProfScope(Problem* p, int cls, hipStream_t st) : s(st) { prof_begin(p, cls, st, &slot); }
    ~ProfScope() { prof_end(slot, s); }
};

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

inline poba_status hip_check(hipError_t e) { return e == hipSuccess ? POBA_OK : POBA_ERR_HIP; }

#define POBA_LAUNCH_CHECK()                                  \
    do {                                                     \
        if (hipGetLastError() != hipSuccess) return POBA_ERR_HIP; \
    } while (0)

}  // namespace poba
