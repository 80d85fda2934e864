// Linearisation (Sec. 4 and 4.1): residuals, Jacobian blocks, and the
// undamped normal-equation blocks U = J_p^T J_p, V = J_l^T J_l, b_p = J_p^T r,
// b_l = J_l^T r, plus the cost F = 1/2 sum rho(|r_i|^2).
//
// The camera-major pass evaluates every observation (camera data is the same
// for the whole block), stores the camera-major records and residuals, sums
// the cost and reduces U and b_p per camera piece; the landmark-major pass
// evaluates the observations again, stores the landmark-major records and
// reduces V and b_l per landmark segment.  Both accumulate in float64 from the Jacobian values rounded to the
// storage precision, so U, V and W are built from one and the same J.  The
// residual and the cost are float64 in every mode; with float32 storage the
// blocks themselves are float32 arithmetic (evaluate_obs_f32), which halves
// their registers, and with float64 or bfloat16 storage float64 (bfloat16
// records are the float64 blocks rounded to nearest).
#include <type_traits>

#include "camera_model.hpp"
#include "device_ops.hpp"
#include "kernels.hpp"

namespace poba {

// Rotation data of every camera (the only transcendental work per camera).
__global__ __launch_bounds__(kBlock) void k_cam_prep(Sizes z, const double* __restrict__ cams, const int32_t* gate,
                                                     double* __restrict__ out) {
    if (gate && !*gate) return;
    const int32_t c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= z.nc) return;
    double cam[9], rec[kCamRec];
#pragma unroll
    for (int k = 0; k < 9; ++k) cam[k] = cams[9 * int64_t(c) + k];
    make_cam_record(cam, rec);
#pragma unroll
    for (int k = 0; k < kCamRec; ++k) out[kCamRec * int64_t(c) + k] = rec[k];
}

// Camera-major pass, one wavefront per camera piece (pieces dealt to the dies
// as in the camera pass of the series, so the landmark gathers stay
// die-local).  Each observation is evaluated once here: residual, Huber
// weight, Jacobian blocks; the records and the reweighted residual are stored
// camera-major, and every lane adds its observations' rows [J_p row, r] (as
// stored) to the upper triangle of J_p^T J_p (45) and to J_p^T r (9) in
// float64 registers; at the end of the piece the wavefront adds its lanes
// (and the cost) and the last lane writes the piece's partial slots.
// The products of float32 (or bfloat16) values are exact in float64, so the
// sums see the blocks as stored.  On this GPU the float64 matrix cores have
// the vector units' peak, and a 10-column Gram product fills a fifth of a
// 16 x 16 tile, so the vector units do this sum.
constexpr int kGramEntries = 54;  // 45 of U (upper triangle, row-major) and 9 of b_p

// Adds the rank-one terms of one row (J_p row, residual) to the partial sums.
__device__ __forceinline__ void gram_add(double* acc, const double* row, double r) {
    int k = 0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
#pragma unroll
        for (int j = i; j < 9; ++j) {
            acc[k] = fma(row[i], row[j], acc[k]);
            ++k;
        }
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) acc[45 + i] = fma(row[i], r, acc[45 + i]);
}

// The piece's partial sums: acc (54), cost, non-finite flag.
__device__ __forceinline__ void cam_piece_write(const Buffers& b, int32_t p, double* acc, double cost, double bad) {
    double tot[kGramEntries + 2];
#pragma unroll
    for (int k = 0; k < kGramEntries; ++k) tot[k] = acc[k];
    tot[kGramEntries] = cost;
    tot[kGramEntries + 1] = bad;
    wave_total_last<kGramEntries + 2>(tot);
    if (lane_id() == kWave - 1) {
#pragma unroll
        for (int k = 0; k < kGramEntries; ++k) b.part[kGramEntries * int64_t(p) + k] = tot[k];
        b.piece_red[3 * int64_t(p)] = tot[kGramEntries];
        b.piece_red[3 * int64_t(p) + 1] = tot[kGramEntries + 1];
    }
}

template <typename TJ>
__global__ __launch_bounds__(kWave) void k_lin_cam(Buffers b, Sizes z, const double* __restrict__ lms, int loss,
                                                   double delta, const int32_t* gate) {
    if (gate && !*gate) return;
    const PieceRec pr = b.sched_rec[blockIdx.x];  // piece, its range and camera in one load
    // the same for the whole wavefront: uniform, so the camera record comes
    // through the scalar cache once instead of per observation
    const int32_t p = __builtin_amdgcn_readfirstlane(pr.p);
    if (p < 0) return;
    const int32_t cam = __builtin_amdgcn_readfirstlane(pr.cam);
    const int32_t a = __builtin_amdgcn_readfirstlane(pr.begin), e = __builtin_amdgcn_readfirstlane(pr.end);
    // read before the loop's stores: uniform loads the compiler can keep in scalar registers
    double rec[kCamRec];
#pragma unroll
    for (int k = 0; k < kCamRec; ++k) rec[k] = b.lin_rec[kCamRec * int64_t(cam) + k];
    double acc[kGramEntries];
#pragma unroll
    for (int k = 0; k < kGramEntries; ++k) acc[k] = 0.0;
    double cost = 0.0, bad = 0.0;
    // the next observation's landmark position and observation are requested
    // before this one is evaluated (positions past the piece read its last)
    auto at = [&](int32_t i) { return min(i, e - 1); };
    double X[3], ox, oy;
    {
        const int32_t i0 = at(a + lane_id());
        const int64_t l = b.co_lm[i0];
#pragma unroll
        for (int k = 0; k < 3; ++k) X[k] = lms[3 * l + k];
        ox = b.obs_co[2 * int64_t(i0)];
        oy = b.obs_co[2 * int64_t(i0) + 1];
    }
    for (int32_t i = a + lane_id(); i < e; i += kWave) {
        double Xn[3], oxn, oyn;
        {
            const int32_t i1 = at(i + kWave);
            const int64_t l = b.co_lm[i1];
#pragma unroll
            for (int k = 0; k < 3; ++k) Xn[k] = lms[3 * l + k];
            oxn = b.obs_co[2 * int64_t(i1)];
            oyn = b.obs_co[2 * int64_t(i1) + 1];
        }
        double rr[2], row0[9], row1[9];
        if constexpr (!std::is_same<TJ, float>::value) {
            ObsEval ev;
            evaluate_obs_rec(rec, X, ox, oy, ev);
            rr[0] = ev.r[0];
            rr[1] = ev.r[1];
            const double s2 = rr[0] * rr[0] + rr[1] * rr[1];
            double rho = s2, w = 1.0;
            if (loss == POBA_LOSS_HUBER) huber(s2, delta, rho, w);
            cost += 0.5 * rho;
            if (!isfinite(rho)) bad = 1.0;
            const double sw = sqrt(w);
            double J[24];
#pragma unroll
            for (int k = 0; k < 24; ++k) J[k] = sw * ev.J[k];
            store_J<TJ>(b.J_co, z.npad, i, J);
            rr[0] *= sw;
            rr[1] *= sw;
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                row0[k] = round_to_storage<TJ>(J[k]);
                row1[k] = round_to_storage<TJ>(J[9 + k]);
            }
        } else {
            float J[24];
            evaluate_obs_f32(rec, X, ox, oy, rr, J);
            const double s2 = rr[0] * rr[0] + rr[1] * rr[1];
            double rho = s2, w = 1.0;
            if (loss == POBA_LOSS_HUBER) huber(s2, delta, rho, w);
            cost += 0.5 * rho;
            if (!isfinite(rho)) bad = 1.0;
            const double sw = sqrt(w);
            const float swf = float(sw);
#pragma unroll
            for (int k = 0; k < 24; ++k) J[k] = swf * J[k];
            store_J_f32(b.J_co, z.npad, i, J);
            rr[0] *= sw;
            rr[1] *= sw;
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                row0[k] = double(J[k]);
                row1[k] = double(J[9 + k]);
            }
        }
        b.r_co[2 * int64_t(i)] = rr[0];
        b.r_co[2 * int64_t(i) + 1] = rr[1];
        gram_add(acc, row0, rr[0]);
        gram_add(acc, row1, rr[1]);
#pragma unroll
        for (int k = 0; k < 3; ++k) X[k] = Xn[k];
        ox = oxn;
        oy = oyn;
    }
    cam_piece_write(b, p, acc, cost, bad);
}

// Landmark-tile groups handled by one wavefront of the landmark-major
// linearisation (one stream of chunks with three in flight).
constexpr int kLinTilesPerWave = 4;

// Camera records of the landmark-major linearisation staged in LDS: the
// fields its kernels read (R, t, f, k1, k2 in float64; w, B and E only as
// float32 values, which is how the float32 blocks use them and what the
// float64 J_l of point records does not use), 144 bytes per camera (4 x an
// odd number of 4-byte words, so that lanes with different cameras spread
// over the banks).  Up to 1,137 cameras fit in 160 KB.
struct __attribute__((aligned(16))) LinLdsCam {
    double R[9], t[3], fk[3];
    float w[3], B, E, pad;
};
static_assert(sizeof(LinLdsCam) == 144, "144-byte camera slots");
constexpr int kLinLdsBlock = 1024;  // one workgroup of 16 wavefronts per compute unit

__device__ __forceinline__ void stage_lin_cams(const double* __restrict__ lin_rec, int32_t nc, LinLdsCam* cams) {
    for (int32_t c = threadIdx.x; c < nc; c += blockDim.x) {
        const double* r = lin_rec + kCamRec * int64_t(c);
        LinLdsCam x;
#pragma unroll
        for (int k = 0; k < 9; ++k) x.R[k] = r[13 + k];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            x.t[k] = r[3 + k];
            x.fk[k] = r[6 + k];
            x.w[k] = float(r[k]);
        }
        x.B = float(r[10]);
        x.E = float(r[22]);
        x.pad = 0.0f;
        cams[c] = x;
    }
}

// The staged fields at their places in a camera record (the others are not
// read by the landmark-major linearisation).
__device__ __forceinline__ const double* lin_cam_from_lds(const LinLdsCam& x, double* rec) {
#pragma unroll
    for (int k = 0; k < 9; ++k) rec[13 + k] = x.R[k];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        rec[3 + k] = x.t[k];
        rec[6 + k] = x.fk[k];
        rec[k] = double(x.w[k]);
    }
    rec[10] = double(x.B);
    rec[22] = double(x.E);
    return rec;
}

// Landmark-major pass: evaluates every observation again from the per-camera
// records (from L2, or staged in LDS where they fit; gathering the
// camera-major records through the permutation would read a whole line per
// 16 bytes), stores the landmark-major records and reduces V = J_l^T J_l (6)
// and b_l = J_l^T r (3) per landmark segment in float64.  The same
// contraction-free arithmetic as the camera-major pass gives bit-identical
// blocks.  camrec(cam, tmp) returns camera cam's record (tmp: room for a copy).
template <typename TJ, typename CamRec>
__device__ __forceinline__ void lin_lm_tiles(const Buffers& b, const Sizes& z, const double* __restrict__ lms, int loss,
                                             double delta, int64_t t0, int64_t t1, CamRec&& camrec) {
    lm_tile_stream<9>(
        b.lo_cam, b.tile_start, b.seg_base, b.nel, b.obs_lo, lms, z.nl, t0, t1,
        [&](int32_t i, bool valid, int32_t cam, const double* X, double ox, double oy, double* v) {
#pragma unroll
            for (int k = 0; k < 9; ++k) v[k] = 0.0;
            if (!valid) return;
            double tmp[kCamRec];
            const double* rec = camrec(cam, tmp);
            double a[3], c[3], rr[2];  // J_l rows 0 and 1 as stored, in float64
            if constexpr (!std::is_same<TJ, float>::value) {
                ObsEval ev;
                evaluate_obs_rec(rec, X, ox, oy, ev);
                rr[0] = ev.r[0];
                rr[1] = ev.r[1];
                double w = 1.0;
                if (loss == POBA_LOSS_HUBER) {
                    double rho;
                    huber(rr[0] * rr[0] + rr[1] * rr[1], delta, rho, w);
                }
                const double sw = sqrt(w);
                double J[24];
#pragma unroll
                for (int k = 0; k < 24; ++k) J[k] = sw * ev.J[k];
                store_J<TJ>(b.J_lo, z.npad, i, J);
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    a[k] = round_to_storage<TJ>(J[18 + k]);
                    c[k] = round_to_storage<TJ>(J[21 + k]);
                }
                rr[0] *= sw;
                rr[1] *= sw;
            } else {
                float J[24];
                evaluate_obs_f32(rec, X, ox, oy, rr, J);
                double w = 1.0;
                if (loss == POBA_LOSS_HUBER) {
                    double rho;
                    huber(rr[0] * rr[0] + rr[1] * rr[1], delta, rho, w);
                }
                const double sw = sqrt(w);
                const float swf = float(sw);
#pragma unroll
                for (int k = 0; k < 24; ++k) J[k] = swf * J[k];
                store_J_f32(b.J_lo, z.npad, i, J);
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    a[k] = double(J[18 + k]);
                    c[k] = double(J[21 + k]);
                }
                rr[0] *= sw;
                rr[1] *= sw;
            }
            const double r0 = rr[0], r1 = rr[1];
            v[0] = a[0] * a[0] + c[0] * c[0];
            v[1] = a[0] * a[1] + c[0] * c[1];
            v[2] = a[0] * a[2] + c[0] * c[2];
            v[3] = a[1] * a[1] + c[1] * c[1];
            v[4] = a[1] * a[2] + c[1] * c[2];
            v[5] = a[2] * a[2] + c[2] * c[2];
            v[6] = a[0] * r0 + c[0] * r1;
            v[7] = a[1] * r0 + c[1] * r1;
            v[8] = a[2] * r0 + c[2] * r1;
        },
        [&](int32_t, int32_t lmk, const double* v) {
            const int64_t l = lmk;
#pragma unroll
            for (int k = 0; k < 6; ++k) b.V[6 * l + k] = v[k];
#pragma unroll
            for (int k = 0; k < 3; ++k) b.bl[3 * l + k] = v[6 + k];
        });
}

template <typename TJ>
__global__ __launch_bounds__(kBlock) void k_lin_lm(Buffers b, Sizes z, const double* __restrict__ lms, int loss,
                                                   double delta, const int32_t* gate) {
    if (gate && !*gate) return;
    const int64_t t0 = (int64_t(blockIdx.x) * kWavesPerBlock + wave_in_block()) * kLinTilesPerWave;
    if (t0 >= z.ntiles) return;
    const int64_t t1 = min(t0 + kLinTilesPerWave, z.ntiles);
    lin_lm_tiles<TJ>(b, z, lms, loss, delta, t0, t1,
                     [&](int32_t cam, double*) { return b.lin_rec + kCamRec * int64_t(cam); });
}

// The same with the camera records staged in LDS (float32 blocks): one
// workgroup per compute unit, every wavefront one contiguous range of `per`
// tiles.
template <typename TJ>
__global__ __launch_bounds__(kLinLdsBlock) void k_lin_lm_lds(Buffers b, Sizes z, const double* __restrict__ lms,
                                                            int loss, double delta, const int32_t* gate, int64_t per) {
    extern __shared__ unsigned char lds_raw[];
    if (gate && !*gate) return;
    LinLdsCam* cams = reinterpret_cast<LinLdsCam*>(lds_raw);
    stage_lin_cams(b.lin_rec, z.nc, cams);
    __syncthreads();
    const int64_t t0 = (int64_t(blockIdx.x) * (kLinLdsBlock / kWave) + wave_in_block()) * per;
    if (t0 >= z.ntiles) return;
    const int64_t t1 = min(t0 + per, z.ntiles);
    lin_lm_tiles<TJ>(b, z, lms, loss, delta, t0, t1,
                     [&](int32_t cam, double* tmp) { return lin_cam_from_lds(cams[cam], tmp); });
}

// Point records (camera-major pass): stores (P, sqrt(w)) rounded to TP and the
// reweighted residual, and accumulates U and b_p from the blocks rebuilt in
// float64 from the rounded record, the blocks every later pass sees.
template <typename TP>
__global__ __launch_bounds__(kWave) void k_lin_cam_pt(Buffers b, Sizes z, const double* __restrict__ lms, int loss,
                                                      double delta, const int32_t* gate) {
    if (gate && !*gate) return;
    const PieceRec pr = b.sched_rec[blockIdx.x];  // piece, its range and camera in one load
    const int32_t p = __builtin_amdgcn_readfirstlane(pr.p);
    if (p < 0) return;
    const int32_t cam = __builtin_amdgcn_readfirstlane(pr.cam);
    const int32_t a = __builtin_amdgcn_readfirstlane(pr.begin), e = __builtin_amdgcn_readfirstlane(pr.end);
    double rec[kCamRec];
#pragma unroll
    for (int k = 0; k < kCamRec; ++k) rec[k] = b.lin_rec[kCamRec * int64_t(cam) + k];
    double acc[kGramEntries];
#pragma unroll
    for (int k = 0; k < kGramEntries; ++k) acc[k] = 0.0;
    double cost = 0.0, bad = 0.0;
    auto at = [&](int32_t i) { return min(i, e - 1); };
    double X[3], ox, oy;
    {
        const int32_t i0 = at(a + lane_id());
        const int64_t l = b.co_lm[i0];
#pragma unroll
        for (int k = 0; k < 3; ++k) X[k] = lms[3 * l + k];
        ox = b.obs_co[2 * int64_t(i0)];
        oy = b.obs_co[2 * int64_t(i0) + 1];
    }
    for (int32_t i = a + lane_id(); i < e; i += kWave) {
        double Xn[3], oxn, oyn;
        {
            const int32_t i1 = at(i + kWave);
            const int64_t l = b.co_lm[i1];
#pragma unroll
            for (int k = 0; k < 3; ++k) Xn[k] = lms[3 * l + k];
            oxn = b.obs_co[2 * int64_t(i1)];
            oyn = b.obs_co[2 * int64_t(i1) + 1];
        }
        double P[3], r[2];
        camera_point(rec, X, ox, oy, P, r);
        const double s2 = r[0] * r[0] + r[1] * r[1];
        double rho = s2, w = 1.0;
        if (loss == POBA_LOSS_HUBER) huber(s2, delta, rho, w);
        cost += 0.5 * rho;
        if (!isfinite(rho)) bad = 1.0;
        store_point<TP>(b.J_co, z.npad, i, P, sqrt(w));
        double Pr[3] = {round_point<TP>(P[0]), round_point<TP>(P[1]), round_point<TP>(P[2])};
        const double swr = round_point<TP>(sqrt(w));
        double J[24];
        point_jacobian<double>(rec, Pr, swr, J);
        const double r0v = swr * r[0], r1v = swr * r[1];
        b.r_co[2 * int64_t(i)] = r0v;
        b.r_co[2 * int64_t(i) + 1] = r1v;
        gram_add(acc, J, r0v);
        gram_add(acc, J + 9, r1v);
#pragma unroll
        for (int k = 0; k < 3; ++k) X[k] = Xn[k];
        ox = oxn;
        oy = oyn;
    }
    cam_piece_write(b, p, acc, cost, bad);
}

// Point records (landmark-major pass): the same records in landmark-major
// order (bit-identical to the camera-major ones) and V, b_l per landmark from
// the rebuilt blocks (J_l = J_P R needs R, t, f, k1, k2 of the camera only).
template <typename TP, typename CamRec>
__device__ __forceinline__ void lin_lm_pt_tiles(const Buffers& b, const Sizes& z, const double* __restrict__ lms,
                                                int loss, double delta, int64_t t0, int64_t t1, CamRec&& camrec) {
    lm_tile_stream<9>(
        b.lo_cam, b.tile_start, b.seg_base, b.nel, b.obs_lo, lms, z.nl, t0, t1,
        [&](int32_t i, bool valid, int32_t cam, const double* X, double ox, double oy, double* v) {
#pragma unroll
            for (int k = 0; k < 9; ++k) v[k] = 0.0;
            if (!valid) return;
            double tmp[kCamRec];
            const double* rec = camrec(cam, tmp);
            double P[3], r[2];
            camera_point(rec, X, ox, oy, P, r);
            double w = 1.0;
            if (loss == POBA_LOSS_HUBER) {
                double rho;
                huber(r[0] * r[0] + r[1] * r[1], delta, rho, w);
            }
            store_point<TP>(b.J_lo, z.npad, i, P, sqrt(w));
            double Pr[3] = {round_point<TP>(P[0]), round_point<TP>(P[1]), round_point<TP>(P[2])};
            const double swr = round_point<TP>(sqrt(w));
            double J[24];
            point_jacobian<double>(rec, Pr, swr, J);
            const double r0 = swr * r[0], r1 = swr * r[1];
            const double* a = J + 18;
            const double* c = J + 21;
            v[0] = a[0] * a[0] + c[0] * c[0];
            v[1] = a[0] * a[1] + c[0] * c[1];
            v[2] = a[0] * a[2] + c[0] * c[2];
            v[3] = a[1] * a[1] + c[1] * c[1];
            v[4] = a[1] * a[2] + c[1] * c[2];
            v[5] = a[2] * a[2] + c[2] * c[2];
            v[6] = a[0] * r0 + c[0] * r1;
            v[7] = a[1] * r0 + c[1] * r1;
            v[8] = a[2] * r0 + c[2] * r1;
        },
        [&](int32_t, int32_t lmk, const double* v) {
            const int64_t l = lmk;
#pragma unroll
            for (int k = 0; k < 6; ++k) b.V[6 * l + k] = v[k];
#pragma unroll
            for (int k = 0; k < 3; ++k) b.bl[3 * l + k] = v[6 + k];
        });
}

template <typename TP>
__global__ __launch_bounds__(kBlock) void k_lin_lm_pt(Buffers b, Sizes z, const double* __restrict__ lms, int loss,
                                                      double delta, const int32_t* gate) {
    if (gate && !*gate) return;
    const int64_t t0 = (int64_t(blockIdx.x) * kWavesPerBlock + wave_in_block()) * kLinTilesPerWave;
    if (t0 >= z.ntiles) return;
    const int64_t t1 = min(t0 + kLinTilesPerWave, z.ntiles);
    lin_lm_pt_tiles<TP>(b, z, lms, loss, delta, t0, t1,
                        [&](int32_t cam, double*) { return b.lin_rec + kCamRec * int64_t(cam); });
}

template <typename TP>
__global__ __launch_bounds__(kLinLdsBlock) void k_lin_lm_pt_lds(Buffers b, Sizes z, const double* __restrict__ lms,
                                                               int loss, double delta, const int32_t* gate,
                                                               int64_t per) {
    extern __shared__ unsigned char lds_raw[];
    if (gate && !*gate) return;
    LinLdsCam* cams = reinterpret_cast<LinLdsCam*>(lds_raw);
    stage_lin_cams(b.lin_rec, z.nc, cams);
    __syncthreads();
    const int64_t t0 = (int64_t(blockIdx.x) * (kLinLdsBlock / kWave) + wave_in_block()) * per;
    if (t0 >= z.ntiles) return;
    const int64_t t1 = min(t0 + per, z.ntiles);
    lin_lm_pt_tiles<TP>(b, z, lms, loss, delta, t0, t1,
                        [&](int32_t cam, double* tmp) { return lin_cam_from_lds(cams[cam], tmp); });
}

// F of every problem: its pieces' partial costs in piece order (one block per
// problem).  Written to pctl, to cost_out[j] and, for active problems, to the
// LM states st[j] (either pointer may be null).
__global__ __launch_bounds__(kBlock) void k_cost_final(Buffers b, const int32_t* gate, double* cost_out,
                                                       poba_lm_state* st) {
    __shared__ double lds[kWavesPerBlock * 2];
    if (gate && !*gate) return;
    const int32_t j = blockIdx.x;
    const int32_t a = b.prob_piece_off[j], e = b.prob_piece_off[j + 1];
    double out[2];
    sum_partials<2>(b.piece_red + 3 * int64_t(a), uint32_t(e - a), out, lds, 3);
    if (threadIdx.x == 0) {
        PCtrl& q = b.pctl[j];
        q.cost = out[0];
        if (cost_out) cost_out[j] = out[0];
        if (st && q.active) st[j].cost = out[0];
        if (out[1] != 0.0 || !isfinite(out[0])) q.status |= POBA_ERR_NONFINITE;
    }
}

// Sums each camera's pieces into the full symmetric U (81) and b_p (9): one
// wavefront per camera, lane k < 54 adding partial entry k over the camera's
// pieces in piece order.
__global__ __launch_bounds__(kBlock) void k_lin_cam_fin(Buffers b, Sizes z, const int32_t* gate) {
    if (gate && !*gate) return;
    const int32_t c = blockIdx.x * kWavesPerBlock + wave_in_block();
    const int k = lane_id();
    if (c >= z.nc || k >= 54) return;
    double acc = 0.0;
    for (int32_t p = b.cam_piece[c]; p < b.cam_piece[c + 1]; ++p) acc += b.part[54 * int64_t(p) + k];
    if (k >= 45) {
        b.bp[9 * int64_t(c) + (k - 45)] = acc;
        return;
    }
    int e = k, r = 0;
    while (e >= 9 - r) {
        e -= 9 - r;
        ++r;
    }
    const int cc = r + e;
    double* U = b.U + 81 * int64_t(c);
    U[9 * r + cc] = acc;
    U[9 * cc + r] = acc;
}

template <typename TJ>
poba_status launch_linearize_t(Problem* p, const double* cams, const double* lms, const int32_t* gate,
                               double* cost_out, poba_lm_state* st, hipStream_t s) {
    const Buffers& b = p->b;
    const Sizes& z = p->z;
    const double delta = p->d.huber_delta;
    const int loss = p->d.loss;
    ProfScope prof(p, POBA_K_LINEARIZE, s);
    hipLaunchKernelGGL(k_cam_prep, dim3(unsigned(ceil_div(z.nc, kBlock))), dim3(kBlock), 0, s, z, cams, gate,
                       b.lin_rec);
    const unsigned ncb = unsigned(std::max<int64_t>(p->sched_len, 1));
    const dim3 g_tiles(unsigned(ceil_div(z.ntiles, int64_t(kWavesPerBlock) * kLinTilesPerWave)));
    // landmark-major kernels with the camera records staged in LDS (float32
    // blocks and point records, where they fit): one workgroup per compute
    // unit, the tiles split evenly over its wavefronts
    const size_t lds_cams = size_t(z.nc) * sizeof(LinLdsCam);
    const bool lm_lds = lds_cams <= size_t(p->lds_max);
    const int64_t lds_waves = p->n_cus * (kLinLdsBlock / kWave);
    const int64_t lds_per = std::max<int64_t>(1, ceil_div(z.ntiles, lds_waves));
    const dim3 g_lds(unsigned(ceil_div(ceil_div(z.ntiles, lds_per), kLinLdsBlock / kWave)));
    bool done = false;
    if constexpr (!std::is_same<TJ, bf16_t>::value) {
        if (z.point) {
            // point records in the precision of TJ (double or float)
            if (p->sched_len > 0)
                hipLaunchKernelGGL(k_lin_cam_pt<TJ>, dim3(ncb), dim3(kWave), 0, s, b, z, lms, loss, delta, gate);
            hipLaunchKernelGGL(k_cost_final, dim3(unsigned(z.np)), dim3(kBlock), 0, s, b, gate, cost_out, st);
            if (lm_lds)
                hipLaunchKernelGGL(k_lin_lm_pt_lds<TJ>, g_lds, dim3(kLinLdsBlock), lds_cams, s, b, z, lms, loss, delta,
                                   gate, lds_per);
            else
                hipLaunchKernelGGL(k_lin_lm_pt<TJ>, g_tiles, dim3(kBlock), 0, s, b, z, lms, loss, delta, gate);
            done = true;
        }
    }
    if (!done) {
        if (p->sched_len > 0)
            hipLaunchKernelGGL(k_lin_cam<TJ>, dim3(ncb), dim3(kWave), 0, s, b, z, lms, loss, delta, gate);
        hipLaunchKernelGGL(k_cost_final, dim3(unsigned(z.np)), dim3(kBlock), 0, s, b, gate, cost_out, st);
        bool staged = false;
        if constexpr (std::is_same<TJ, float>::value) {
            // (float64 and bfloat16 blocks read more of the record than is staged)
            if (lm_lds) {
                hipLaunchKernelGGL(k_lin_lm_lds<TJ>, g_lds, dim3(kLinLdsBlock), lds_cams, s, b, z, lms, loss, delta,
                                   gate, lds_per);
                staged = true;
            }
        }
        if (!staged) hipLaunchKernelGGL(k_lin_lm<TJ>, g_tiles, dim3(kBlock), 0, s, b, z, lms, loss, delta, gate);
    }
    hipLaunchKernelGGL(k_lin_cam_fin, dim3(unsigned(ceil_div(z.nc, kWavesPerBlock))), dim3(kBlock), 0, s, b, z, gate);
    return hipGetLastError() == hipSuccess ? POBA_OK : POBA_ERR_HIP;
}

poba_status launch_cam_prep(Problem* p, const double* cams, const int32_t* gate, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_cam_prep, dim3(unsigned(ceil_div(p->z.nc, kBlock))), dim3(kBlock), 0, s, p->z, cams, gate,
                       out);
    return hipGetLastError() == hipSuccess ? POBA_OK : POBA_ERR_HIP;
}

poba_status launch_linearize(Problem* p, const double* cams, const double* lms, const int32_t* gate,
                             double* cost_out, poba_lm_state* st, hipStream_t s) {
    switch (p->d.precision) {
        case POBA_F64: return launch_linearize_t<double>(p, cams, lms, gate, cost_out, st, s);
        case POBA_F32: return launch_linearize_t<float>(p, cams, lms, gate, cost_out, st, s);
        default: return launch_linearize_t<bf16_t>(p, cams, lms, gate, cost_out, st, s);
    }
}

}  // namespace poba

using namespace poba;

extern "C" poba_status poba_linearize(poba_problem p, const double* cams, const double* lms, double* cost,
                                      poba_stream stream) {
    (void)hipGetLastError();  // report only this call's launch errors
    if (!p || !cams || !lms) return POBA_ERR_INVALID_ARG;
    return launch_linearize(p, cams, lms, nullptr, cost, nullptr, reinterpret_cast<hipStream_t>(stream));
}
