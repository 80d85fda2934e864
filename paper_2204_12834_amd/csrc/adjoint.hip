// Adjoint of one damped step by implicit differentiation (an extension of the
// method; the paper solves the step, it does not differentiate it).
//
// The step of Sec. 4.1 (eq. normal) at a fixed state, damping lambda and
// damping diagonal D:
//   H dx = -g,   H = J^T J + lambda D,   g = J^T r,   r = pi(theta) - o,
// with theta the intrinsics (f, k1, k2) of every camera.  For an upstream
// gradient gbar of dx and z = H^-1 gbar (H is symmetric, and so is the
// truncated-series inverse, whose adjoint is therefore the same power solve
// run on gbar):
//   obar_i     = J_i z_i
//   thetabar_c = -sum_{i in c} [ e_i^T (d_theta J_i) z_i + a_i^T (d_theta J_i) dx_i + a_i^T d_theta r_i ]
// with a_i = J_i z_i and e_i = J_i dx_i + r_i; (d_theta J_i) w is the mixed
// second derivative of pi along w, in closed form for the intrinsics.
#include "camera_model.hpp"
#include "device_ops.hpp"
#include "kernels.hpp"

namespace poba {

__global__ __launch_bounds__(kBlock) void k_negate(double* p, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i < n) p[i] = -p[i];
}

// Observations into both storage orders.
__global__ __launch_bounds__(kBlock) void k_set_obs(Buffers b, Sizes z, const double* __restrict__ obs_xy) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= z.N) return;
    const int64_t ol = b.perm_l[i], oc = b.perm_c[i];
    b.obs_lo[2 * i] = obs_xy[2 * ol];
    b.obs_lo[2 * i + 1] = obs_xy[2 * ol + 1];
    b.obs_co[2 * i] = obs_xy[2 * oc];
    b.obs_co[2 * i + 1] = obs_xy[2 * oc + 1];
}

// d/d(f, k1, k2) of the directional derivative D pi [w] of one observation,
// for w = (camera part wc[9], landmark part wl[3]); out[k][a].
__device__ __forceinline__ void intrinsic_mixed(const ObsGeom& g, const double* cam, const double* wc,
                                                const double* wl, double (*out)[2]) {
    const double f = cam[6], k1 = cam[7], k2 = cam[8];
    const double n = g.n, n2 = n * n;
    const double d = 1.0 + k1 * n + k2 * n2;
    double dpw[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < 6; ++j) s += g.dp[a][j] * wc[j];
#pragma unroll
        for (int j = 0; j < 3; ++j) s += g.dp[a][6 + j] * wl[j];
        dpw[a] = s;
    }
    const double dnw = 2.0 * (g.p[0] * dpw[0] + g.p[1] * dpw[1]);
    const double cf = wc[7] * n + wc[8] * n2 + (k1 + 2.0 * k2 * n) * dnw;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        out[0][a] = cf * g.p[a] + d * dpw[a];
        out[1][a] = wc[6] * n * g.p[a] + f * dnw * g.p[a] + f * n * dpw[a];
        out[2][a] = wc[6] * n2 * g.p[a] + 2.0 * f * n * dnw * g.p[a] + f * n2 * dpw[a];
    }
}

// One block per camera piece (camera-major order).  Writes obar of every
// observation of the piece at its original index and the piece's partial
// intrinsic gradient (3 values) to its slot of `part`.
template <typename TJ, bool PT>
__global__ __launch_bounds__(kBlock) void k_adjoint(Buffers b, Sizes z, const double* __restrict__ lms,
                                                    const double* __restrict__ zc, const double* __restrict__ zl,
                                                    const double* __restrict__ dxc, const double* __restrict__ dxl,
                                                    double* __restrict__ grad_obs) {
    __shared__ double lds[kWavesPerBlock * 3];
    const int32_t p = b.sched[blockIdx.x];
    if (p < 0) return;
    const int32_t a0 = b.piece_begin[p], e0 = b.piece_end[p];
    const int64_t c = b.piece_cam[p];
    const double* rec = b.lin_rec + kCamRec * c;
    double zcam[9], dcam[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        zcam[k] = zc[9 * c + k];
        dcam[k] = dxc[9 * c + k];
    }
    double acc[3] = {0.0, 0.0, 0.0};
    for (int32_t i = a0 + threadIdx.x; i < e0; i += kBlock) {
        const int64_t l = b.co_lm[i];
        const double X[3] = {lms[3 * l], lms[3 * l + 1], lms[3 * l + 2]};
        const double zlm[3] = {zl[3 * l], zl[3 * l + 1], zl[3 * l + 2]};
        const double dlm[3] = {dxl[3 * l], dxl[3 * l + 1], dxl[3 * l + 2]};
        double J[24];
        Rec<TJ, PT>::template jac<double>(b, z, b.J_co, i, c, J);
        double av[2], ev[2];
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            double sa = 0.0, se = 0.0;
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                sa += J[9 * r + k] * zcam[k];
                se += J[9 * r + k] * dcam[k];
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                sa += J[18 + 3 * r + k] * zlm[k];
                se += J[18 + 3 * r + k] * dlm[k];
            }
            av[r] = sa;
            ev[r] = se + b.r_co[2 * int64_t(i) + r];
        }
        const int64_t o = b.perm_c[i];
        grad_obs[2 * o] = av[0];
        grad_obs[2 * o + 1] = av[1];
        ObsGeom g;
        observation_geometry(rec, X, g);
        double Tz[3][2], Td[3][2];
        intrinsic_mixed(g, rec, zcam, zlm, Tz);
        intrinsic_mixed(g, rec, dcam, dlm, Td);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double t = ev[0] * Tz[k][0] + ev[1] * Tz[k][1] + av[0] * Td[k][0] + av[1] * Td[k][1] +
                             av[0] * J[6 + k] + av[1] * J[15 + k];
            acc[k] -= t;
        }
    }
    block_sum<3>(acc, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) b.part[3 * int64_t(p) + k] = acc[k];
    }
}

// Intrinsic gradient per camera: its pieces' partials in piece order.
__global__ __launch_bounds__(kBlock) void k_adjoint_fin(Buffers b, Sizes z, double* __restrict__ grad_intr) {
    const int32_t c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= z.nc) return;
    double s[3] = {0.0, 0.0, 0.0};
    for (int32_t q = b.cam_piece[c]; q < b.cam_piece[c + 1]; ++q) {
#pragma unroll
        for (int k = 0; k < 3; ++k) s[k] += b.part[3 * int64_t(q) + k];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) grad_intr[3 * int64_t(c) + k] = s[k];
}

}  // namespace poba

using namespace poba;

extern "C" {

poba_status poba_set_observations(poba_problem p, const double* obs_xy, poba_stream stream) {
    (void)hipGetLastError();  // report only this call's launch errors
    if (!p || (!obs_xy && p->z.N > 0)) return POBA_ERR_INVALID_ARG;
    if (p->z.N == 0) return POBA_OK;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_set_obs, dim3(unsigned(ceil_div(p->z.N, kBlock))), dim3(kBlock), 0, s, p->b, p->z, obs_xy);
    return hipGetLastError() == hipSuccess ? POBA_OK : POBA_ERR_HIP;
}

poba_status poba_set_damping_frozen(poba_problem p, int32_t frozen) {
    if (!p || (frozen != 0 && frozen != 1)) return POBA_ERR_INVALID_ARG;
    p->damping_frozen = frozen;
    return POBA_OK;
}

poba_status poba_step_adjoint(poba_problem p, double lambda, int32_t m, const double* cams, const double* lms,
                              const double* dx_cams, const double* dx_lms, const double* grad_dx_cams,
                              const double* grad_dx_lms, double* z_cams, double* z_lms, double* grad_obs,
                              double* grad_intrinsics, poba_solve_info* info, poba_stream stream) {
    (void)hipGetLastError();  // report only this call's launch errors
    if (!p || !cams || !lms || !dx_cams || !dx_lms || !grad_dx_cams || !grad_dx_lms || !z_cams || !z_lms ||
        !grad_intrinsics || (!grad_obs && p->z.N > 0))
        return POBA_ERR_INVALID_ARG;
    if (p->d.loss != POBA_LOSS_L2) return POBA_ERR_INVALID_ARG;
    if (!(lambda > 0.0) || m < 0 || m > 100000) return POBA_ERR_INVALID_ARG;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const Sizes& z = p->z;
    // z = H~^-1 gbar: the solve of H dx = -gbar gives -z
    poba_status st = launch_begin_solve(p, lambda, s);
    if (st) return st;
    st = launch_solve(p, m, 0.0, z_cams, z_lms, info, s, grad_dx_cams, grad_dx_lms);
    if (st) return st;
    const dim3 blk(kBlock);
    hipLaunchKernelGGL(k_negate, dim3(unsigned(ceil_div(int64_t(z.nc) * 9, kBlock))), blk, 0, s, z_cams,
                       int64_t(z.nc) * 9);
    if (z.nl > 0)
        hipLaunchKernelGGL(k_negate, dim3(unsigned(ceil_div(int64_t(z.nl) * 3, kBlock))), blk, 0, s, z_lms,
                           int64_t(z.nl) * 3);
    st = launch_cam_prep(p, cams, nullptr, p->b.lin_rec, s);
    if (st) return st;
    if (p->npieces > 0) {
        const dim3 g(unsigned(p->sched_len));
#define POBA_ADJ(TJ_, PT_)                                                                                      \
    hipLaunchKernelGGL((k_adjoint<TJ_, PT_>), g, blk, 0, s, p->b, z, lms, z_cams, z_lms, dx_cams, dx_lms, grad_obs)
        if (z.point) {
            if (p->d.precision == POBA_F64) POBA_ADJ(double, true);
            else POBA_ADJ(float, true);
        } else if (p->d.precision == POBA_F64) {
            POBA_ADJ(double, false);
        } else if (p->d.precision == POBA_F32) {
            POBA_ADJ(float, false);
        } else {
            POBA_ADJ(bf16_t, false);
        }
#undef POBA_ADJ
    }
    hipLaunchKernelGGL(k_adjoint_fin, dim3(unsigned(ceil_div(z.nc, kBlock))), blk, 0, s, p->b, z, grad_intrinsics);
    return hipGetLastError() == hipSuccess ? POBA_OK : POBA_ERR_HIP;
}

}  // extern "C"
