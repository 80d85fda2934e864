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
#include "device_ops.hpp"
#include "kernels.hpp"

namespace poba {

enum FinMode { kFinRhs = 0, kFinSeries = 1, kFinApply = 2 };

// ---------------------------------------------------------------- control --

__global__ void k_begin_solve(Ctrl* ctrl, double lam) {
    if (threadIdx.x == 0) {
        ctrl->lambda = lam;
        ctrl->active = 1;
        ctrl->stopped = 0;
        ctrl->stop_order = 0;
        ctrl->status = 0;
    }
}

// ---------------------------------------------------------------- inverses --

// U_lambda^-1 per camera by a 9x9 Cholesky factorisation, in float64.
__global__ __launch_bounds__(kBlock) void k_inv_cam(Buffers b, Sizes z, int damping, Ctrl* ctrl) {
    if (!ctrl->active) return;
    const int32_t c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= z.nc) return;
    const double lam = ctrl->lambda;
    const double* U = b.U + 81 * int64_t(c);
    double L[81];
#pragma unroll
    for (int k = 0; k < 81; ++k) L[k] = U[k];
    double dg[9];
#pragma unroll
    for (int j = 0; j < 9; ++j) {
        dg[j] = lam * damp_diag(U[10 * j], damping);
        L[10 * j] += dg[j];
    }
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
    double* out = b.Uinv + 81 * int64_t(c);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
#pragma unroll
        for (int j = i; j < 9; ++j) {
            double sacc = 0.0;
#pragma unroll
            for (int k = j; k < 9; ++k) sacc += M[9 * k + i] * M[9 * k + j];
            ok = ok && isfinite(sacc);
            M[9 * i + j] = M[9 * i + j];  // keep M intact (upper part unused)
            out[9 * i + j] = sacc;
            out[9 * j + i] = sacc;
        }
    }
    if (!ok) {
#pragma unroll
        for (int i = 0; i < 9; ++i)
#pragma unroll
            for (int j = 0; j < 9; ++j) out[9 * i + j] = (i == j && dg[i] > 0.0) ? 1.0 / dg[i] : 0.0;
        atomicOr(&ctrl->status, POBA_ERR_NOT_SPD);
    }
}

// V_lambda^-1 per landmark in float64, stored in the landmark storage type.
template <typename TS>
__global__ __launch_bounds__(kBlock) void k_inv_lm(Buffers b, Sizes z, int damping, Ctrl* ctrl) {
    if (!ctrl->active) return;
    const int32_t l = blockIdx.x * kBlock + threadIdx.x;
    if (l >= z.nl) return;
    double Vd[6], inv[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) Vd[k] = b.V[6 * int64_t(l) + k];
    const bool ok = inv3_damped(Vd, ctrl->lambda, damping, inv);
    TS* o = reinterpret_cast<TS*>(b.Vinv) + 6 * int64_t(l);
#pragma unroll
    for (int k = 0; k < 6; ++k) o[k] = TS(inv[k]);
    if (!ok) atomicOr(&ctrl->status, POBA_ERR_NOT_SPD);
}

// y_l = V_lambda^-1 b_l in float64 (first half of b~), into the float64 view of s.
__global__ __launch_bounds__(kBlock) void k_rhs_lm(Buffers b, Sizes z, int damping, const Ctrl* ctrl) {
    if (!ctrl->active) return;
    const int32_t l = blockIdx.x * kBlock + threadIdx.x;
    if (l >= z.nl) return;
    double Vd[6], inv[6], bl[3], y[3];
#pragma unroll
    for (int k = 0; k < 6; ++k) Vd[k] = b.V[6 * int64_t(l) + k];
#pragma unroll
    for (int k = 0; k < 3; ++k) bl[k] = b.bl[3 * int64_t(l) + k];
    inv3_damped(Vd, ctrl->lambda, damping, inv);
    sym3_apply(inv, bl, y);
    double* o = reinterpret_cast<double*>(b.s) + 4 * int64_t(l);
    o[0] = y[0];
    o[1] = y[1];
    o[2] = y[2];
    o[3] = 0.0;
}

// ------------------------------------------------------------ landmark pass --

// s_l = V_l^-1 sum_{i in l} J_l^T (J_p v_c(i)) for every non-empty landmark.
// TJ: Jacobian storage, TC: arithmetic, TV: camera-vector type (stride vstride),
// TS: landmark storage (V^-1 in, s out).
template <typename TJ, typename TC, typename TV, typename TS>
__global__ __launch_bounds__(kBlock) void k_lm_pass(Buffers b, Sizes z, const TV* __restrict__ vin, int vstride,
                                                    TS* __restrict__ sout, const Ctrl* ctrl) {
    if (ctrl->stopped || !ctrl->active) return;
    const int64_t tile = int64_t(blockIdx.x) * kWavesPerBlock + threadIdx.x / kWave;
    if (tile >= z.ntiles) return;
    const TS* __restrict__ Vinv = reinterpret_cast<const TS*>(b.Vinv);
    tile_landmarks<TC, 3>(
        b.lo_cam, b.tile_start, b.seg_base, tile,
        [&](int32_t i, bool valid, int32_t cam, int32_t, TC* v) {
            v[0] = v[1] = v[2] = TC(0);
            if (!valid) return;
            TC J[24];
            load_J<TJ, TC>(b.J_lo, z.npad, i, J);
            const TV* vc = vin + int64_t(cam) * vstride;
            TC q0 = TC(0), q1 = TC(0);
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                const TC xk = TC(vc[k]);
                q0 += J[k] * xk;
                q1 += J[9 + k] * xk;
            }
            v[0] = J[18] * q0 + J[21] * q1;
            v[1] = J[19] * q0 + J[22] * q1;
            v[2] = J[20] * q0 + J[23] * q1;
        },
        [&](int32_t seg, const TC* t) {
            const int64_t l = b.nel[seg];
            TC A[6], y[3];
#pragma unroll
            for (int k = 0; k < 6; ++k) A[k] = TC(Vinv[6 * l + k]);
            sym3_apply(A, t, y);
            TS* o = sout + 4 * l;
            o[0] = TS(y[0]);
            o[1] = TS(y[1]);
            o[2] = TS(y[2]);
        });
}

// Back-substitution dx_l = -V_lambda^-1 (b_l + sum_{i in l} J_l^T J_p x_c) in
// float64 with V_lambda^-1 recomputed from the float64 V.
template <typename TJ>
__global__ __launch_bounds__(kBlock) void k_backsub(Buffers b, Sizes z, int damping, const double* __restrict__ x,
                                                    double* __restrict__ dxl, const Ctrl* ctrl) {
    if (!ctrl->active) return;
    const int64_t tile = int64_t(blockIdx.x) * kWavesPerBlock + threadIdx.x / kWave;
    if (tile >= z.ntiles) return;
    const double lam = ctrl->lambda;
    tile_landmarks<double, 3>(
        b.lo_cam, b.tile_start, b.seg_base, tile,
        [&](int32_t i, bool valid, int32_t cam, int32_t, double* v) {
            v[0] = v[1] = v[2] = 0.0;
            if (!valid) return;
            double J[24];
            load_J<TJ, double>(b.J_lo, z.npad, i, J);
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
        [&](int32_t seg, const double* t) {
            const int64_t l = b.nel[seg];
            double Vd[6], inv[6], rhs[3], y[3];
#pragma unroll
            for (int k = 0; k < 6; ++k) Vd[k] = b.V[6 * l + k];
            inv3_damped(Vd, lam, damping, inv);
#pragma unroll
            for (int k = 0; k < 3; ++k) rhs[k] = b.bl[3 * l + k] + t[k];
            sym3_apply(inv, rhs, y);
#pragma unroll
            for (int k = 0; k < 3; ++k) dxl[3 * l + k] = -y[k];
        });
}

// Landmarks without observations get dx_l = -V^-1 b_l = 0.
__global__ __launch_bounds__(kBlock) void k_zero_empty(Buffers b, Sizes z, double* dxl, const Ctrl* ctrl) {
    if (!ctrl->active) return;
    const int32_t l = blockIdx.x * kBlock + threadIdx.x;
    if (l >= z.nl) return;
    if (b.lm_off[l + 1] == b.lm_off[l]) {
        dxl[3 * int64_t(l)] = 0.0;
        dxl[3 * int64_t(l) + 1] = 0.0;
        dxl[3 * int64_t(l) + 2] = 0.0;
    }
}

// -------------------------------------------------------------- camera pass --

// Partial W s of one camera piece: sum_i J_p^T (J_l s_l(i)), float64 arithmetic.
template <typename TJ, typename TSin>
__global__ __launch_bounds__(kBlock) void k_cam_pass(Buffers b, Sizes z, const TSin* __restrict__ sin,
                                                     const Ctrl* ctrl) {
    __shared__ double lds[kWavesPerBlock * 9];
    if (ctrl->stopped || !ctrl->active) return;
    const int32_t p = blockIdx.x;
    const int32_t a = b.piece_begin[p], e = b.piece_end[p];
    double acc[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) acc[k] = 0.0;
    for (int32_t i = a + threadIdx.x; i < e; i += kBlock) {
        const int64_t l = b.co_lm[i];
        const TSin* sl = sin + 4 * l;
        const double s0 = double(sl[0]), s1 = double(sl[1]), s2 = double(sl[2]);
        double J[24];
        load_J<TJ, double>(b.J_co, z.npad, i, J);
        const double z0 = J[18] * s0 + J[19] * s1 + J[20] * s2;
        const double z1 = J[21] * s0 + J[22] * s1 + J[23] * s2;
#pragma unroll
        for (int k = 0; k < 9; ++k) acc[k] += J[k] * z0 + J[9 + k] * z1;
    }
    block_sum<9>(acc, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < 9; ++k) b.part[9 * int64_t(p) + k] = acc[k];
    }
}

// Per camera: u_c = sum of its pieces, then
//   rhs:    b~_c = b_p - u_c,  v_c = -U^-1 b~_c,  x_c = v_c
//   series: v_c = U^-1 u_c,    x_c += v_c
//   apply:  vout_c = U^-1 u_c
// and the squared norms of v and x over all cameras (stop rule).
template <typename TS>
__global__ __launch_bounds__(kBlock) void k_cam_fin(Buffers b, Sizes z, int mode, int order, double eps,
                                                    double* vout, Ctrl* ctrl) {
    __shared__ double lds[kWavesPerBlock * 2];
    if (ctrl->stopped || !ctrl->active) return;
    const int32_t c = blockIdx.x * kBlock + threadIdx.x;
    double nv2 = 0.0, nx2 = 0.0;
    if (c < z.nc) {
        double u[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) u[k] = 0.0;
        for (int32_t p = b.cam_piece[c]; p < b.cam_piece[c + 1]; ++p) {
#pragma unroll
            for (int k = 0; k < 9; ++k) u[k] += b.part[9 * int64_t(p) + k];
        }
        const double* Ui = b.Uinv + 81 * int64_t(c);
        if (mode == kFinRhs) {
#pragma unroll
            for (int k = 0; k < 9; ++k) u[k] = b.bp[9 * int64_t(c) + k] - u[k];
        }
        double v[9];
#pragma unroll
        for (int r = 0; r < 9; ++r) {
            double sacc = 0.0;
#pragma unroll
            for (int k = 0; k < 9; ++k) sacc += Ui[9 * r + k] * u[k];
            v[r] = mode == kFinRhs ? -sacc : sacc;
        }
        double* xc = b.x + 9 * int64_t(c);
        if (mode == kFinApply) {
#pragma unroll
            for (int k = 0; k < 9; ++k) vout[9 * int64_t(c) + k] = v[k];
        } else {
            TS* vq = reinterpret_cast<TS*>(b.vq) + 12 * int64_t(c);
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                const double xn = mode == kFinRhs ? v[k] : xc[k] + v[k];
                xc[k] = xn;
                b.v[9 * int64_t(c) + k] = v[k];
                vq[k] = TS(v[k]);
                nv2 += v[k] * v[k];
                nx2 += xn * xn;
            }
        }
    }
    double tot[2] = {nv2, nx2};
    block_sum<2>(tot, lds);
    double out[2];
    if (grid_sum_last<2>(tot, b.red_part, &ctrl->ticket[kTicketNorm], gridDim.x, out, lds) && threadIdx.x == 0) {
        if (mode != kFinApply) {
            ctrl->norm_v2 = out[0];
            ctrl->norm_x2 = out[1];
            ctrl->stop_order = order;
            if (mode == kFinSeries && eps > 0.0 &&
                (out[1] == 0.0 || double(order + 1) * sqrt(out[0]) < eps * sqrt(out[1])))
                ctrl->stopped = 1;
        }
    }
}

// Copies x into the caller's camera step and fills the solve info.
__global__ __launch_bounds__(kBlock) void k_finish(Buffers b, Sizes z, double* dx_cams, poba_solve_info* info,
                                                   const Ctrl* ctrl) {
    if (!ctrl->active) return;
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i < int64_t(z.nc) * 9) dx_cams[i] = b.x[i];
    if (i == 0 && info) {
        info->stop_order = ctrl->stop_order;
        info->stopped = ctrl->stopped;
        info->status = ctrl->status;
        info->reserved = 0;
        info->norm_x = sqrt(ctrl->norm_x2);
        info->norm_v = sqrt(ctrl->norm_v2);
    }
}

// Camera vector into the gather copy (stride 12, storage type).
template <typename TS>
__global__ __launch_bounds__(kBlock) void k_load_v(Buffers b, Sizes z, const double* vin, const Ctrl* ctrl) {
    if (!ctrl->active) return;
    const int32_t c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= z.nc) return;
    TS* vq = reinterpret_cast<TS*>(b.vq) + 12 * int64_t(c);
#pragma unroll
    for (int k = 0; k < 9; ++k) vq[k] = TS(vin[9 * int64_t(c) + k]);
}

// --------------------------------------------------------------- host side --

template <typename TJ, typename TS, typename TCL>
poba_status run_solve(Problem* p, int m, double eps, double* dx_cams, double* dx_lms, poba_solve_info* info,
                      hipStream_t s) {
    const Buffers& b = p->b;
    const Sizes& z = p->z;
    const int damping = p->d.damping;
    const dim3 blk(kBlock);
    const dim3 g_cam(unsigned(ceil_div(z.nc, kBlock)));
    const dim3 g_lm(unsigned(ceil_div(z.nl, kBlock)));
    const dim3 g_tiles(unsigned(ceil_div(z.ntiles, kWavesPerBlock)));
    const dim3 g_pieces(unsigned(std::max<int64_t>(p->npieces, 1)));
    const bool pieces = p->npieces > 0;
    {
        ProfScope pr(p, POBA_K_INVERSE, s);
        hipLaunchKernelGGL(k_inv_cam, g_cam, blk, 0, s, b, z, damping, b.ctrl);
        hipLaunchKernelGGL(k_inv_lm<TS>, g_lm, blk, 0, s, b, z, damping, b.ctrl);
    }
    {
        ProfScope pr(p, POBA_K_OTHER, s);
        hipLaunchKernelGGL(k_rhs_lm, g_lm, blk, 0, s, b, z, damping, b.ctrl);
    }
    if (pieces) {
        ProfScope pr(p, POBA_K_CAM_PASS, s);
        hipLaunchKernelGGL((k_cam_pass<TJ, double>), g_pieces, blk, 0, s, b, z,
                           reinterpret_cast<const double*>(b.s), b.ctrl);
    }
    {
        ProfScope pr(p, POBA_K_CAM_FIN, s);
        hipLaunchKernelGGL(k_cam_fin<TS>, g_cam, blk, 0, s, b, z, int(kFinRhs), 0, eps, (double*)nullptr, b.ctrl);
    }
    for (int i = 1; i <= m; ++i) {
        {
            ProfScope pr(p, POBA_K_LM_PASS, s);
            hipLaunchKernelGGL((k_lm_pass<TJ, TCL, TS, TS>), g_tiles, blk, 0, s, b, z,
                               reinterpret_cast<const TS*>(b.vq), 12, reinterpret_cast<TS*>(b.s), b.ctrl);
        }
        if (pieces) {
            ProfScope pr(p, POBA_K_CAM_PASS, s);
            hipLaunchKernelGGL((k_cam_pass<TJ, TS>), g_pieces, blk, 0, s, b, z, reinterpret_cast<const TS*>(b.s),
                               b.ctrl);
        }
        {
            ProfScope pr(p, POBA_K_CAM_FIN, s);
            hipLaunchKernelGGL(k_cam_fin<TS>, g_cam, blk, 0, s, b, z, int(kFinSeries), i, eps, (double*)nullptr,
                               b.ctrl);
        }
    }
    {
        ProfScope pr(p, POBA_K_BACKSUB, s);
        hipLaunchKernelGGL(k_backsub<TJ>, g_tiles, blk, 0, s, b, z, damping, b.x, dx_lms, b.ctrl);
        hipLaunchKernelGGL(k_zero_empty, g_lm, blk, 0, s, b, z, dx_lms, b.ctrl);
        hipLaunchKernelGGL(k_finish, dim3(unsigned(ceil_div(int64_t(z.nc) * 9, kBlock))), blk, 0, s, b, z, dx_cams,
                           info, b.ctrl);
    }
    return hipGetLastError() == hipSuccess ? POBA_OK : POBA_ERR_HIP;
}

poba_status launch_solve(Problem* p, int m, double eps, double* dx_cams, double* dx_lms, poba_solve_info* info,
                         hipStream_t s) {
    switch (p->d.precision) {
        case POBA_F64: return run_solve<double, double, double>(p, m, eps, dx_cams, dx_lms, info, s);
        case POBA_F32: return run_solve<float, float, float>(p, m, eps, dx_cams, dx_lms, info, s);
        default: return run_solve<bf16_t, float, float>(p, m, eps, dx_cams, dx_lms, info, s);
    }
}

poba_status launch_begin_solve(Problem* p, double lam, hipStream_t s) {
    hipLaunchKernelGGL(k_begin_solve, dim3(1), dim3(64), 0, s, p->b.ctrl, lam);
    return hipGetLastError() == hipSuccess ? POBA_OK : POBA_ERR_HIP;
}

template <typename TJ, typename TS, typename TCL>
poba_status run_apply_P(Problem* p, const double* vin, double* vout, hipStream_t s) {
    const Buffers& b = p->b;
    const Sizes& z = p->z;
    const dim3 blk(kBlock);
    const dim3 g_cam(unsigned(ceil_div(z.nc, kBlock)));
    hipLaunchKernelGGL(k_load_v<TS>, g_cam, blk, 0, s, b, z, vin, b.ctrl);
    hipLaunchKernelGGL((k_lm_pass<TJ, TCL, TS, TS>), dim3(unsigned(ceil_div(z.ntiles, kWavesPerBlock))), blk, 0, s, b,
                       z, reinterpret_cast<const TS*>(b.vq), 12, reinterpret_cast<TS*>(b.s), b.ctrl);
    if (p->npieces > 0)
        hipLaunchKernelGGL((k_cam_pass<TJ, TS>), dim3(unsigned(p->npieces)), blk, 0, s, b, z,
                           reinterpret_cast<const TS*>(b.s), b.ctrl);
    hipLaunchKernelGGL(k_cam_fin<TS>, g_cam, blk, 0, s, b, z, int(kFinApply), 0, 0.0, vout, b.ctrl);
    return hipGetLastError() == hipSuccess ? POBA_OK : POBA_ERR_HIP;
}

// Widens the stored records of one order to float64 in original order.
template <typename TJ>
__global__ __launch_bounds__(kBlock) void k_get_jac(Buffers b, Sizes z, int order, double* Jp, double* Jl, double* r) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= z.N) return;
    double J[24];
    load_J<TJ, double>(order == 0 ? b.J_lo : b.J_co, z.npad, i, J);
    const int64_t o = order == 0 ? b.perm_l[i] : b.perm_c[i];
#pragma unroll
    for (int k = 0; k < 18; ++k) Jp[18 * o + k] = J[k];
#pragma unroll
    for (int k = 0; k < 6; ++k) Jl[6 * o + k] = J[18 + k];
    if (r && order == 0) {
        r[2 * o] = b.r_lo[2 * i];
        r[2 * o + 1] = b.r_lo[2 * i + 1];
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

}  // namespace poba

using namespace poba;

extern "C" {

poba_status poba_power_solve(poba_problem p, double lambda, int32_t m, double eps, double* dx_cams, double* dx_lms,
                             poba_solve_info* info, poba_stream stream) {
    if (!p || !dx_cams || !dx_lms) return POBA_ERR_INVALID_ARG;
    if (!(lambda > 0.0) || m < 0 || m > 100000 || !(eps >= 0.0)) return POBA_ERR_INVALID_ARG;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    poba_status st = launch_begin_solve(p, lambda, s);
    if (st) return st;
    return launch_solve(p, m, eps, dx_cams, dx_lms, info, s);
}

poba_status poba_apply_P(poba_problem p, const double* v_in, double* v_out, poba_stream stream) {
    if (!p || !v_in || !v_out) return POBA_ERR_INVALID_ARG;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_begin_solve, dim3(1), dim3(64), 0, s, p->b.ctrl, 0.0);
    // k_begin_solve overwrote lambda; the inverses of the last solve are kept,
    // and apply-P does not read lambda.
    switch (p->d.precision) {
        case POBA_F64: return run_apply_P<double, double, double>(p, v_in, v_out, s);
        case POBA_F32: return run_apply_P<float, float, float>(p, v_in, v_out, s);
        default: return run_apply_P<bf16_t, float, float>(p, v_in, v_out, s);
    }
}

poba_status poba_get_jacobians(poba_problem p, int32_t order, double* Jp, double* Jl, double* r, poba_stream stream) {
    if (!p || !Jp || !Jl || (order != 0 && order != 1)) return POBA_ERR_INVALID_ARG;
    if (p->z.N == 0) return POBA_OK;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const dim3 g(unsigned(ceil_div(p->z.N, kBlock)));
    switch (p->d.precision) {
        case POBA_F64: hipLaunchKernelGGL(k_get_jac<double>, g, dim3(kBlock), 0, s, p->b, p->z, order, Jp, Jl, r); break;
        case POBA_F32: hipLaunchKernelGGL(k_get_jac<float>, g, dim3(kBlock), 0, s, p->b, p->z, order, Jp, Jl, r); break;
        default: hipLaunchKernelGGL(k_get_jac<bf16_t>, g, dim3(kBlock), 0, s, p->b, p->z, order, Jp, Jl, r); break;
    }
    return hipGetLastError() == hipSuccess ? POBA_OK : POBA_ERR_HIP;
}

poba_status poba_get_blocks(poba_problem p, double* U, double* V, double* bp, double* bl, poba_stream stream) {
    if (!p) return POBA_ERR_INVALID_ARG;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int64_t n = std::max<int64_t>(int64_t(p->z.nc) * 81, int64_t(p->z.nl) * 3);
    hipLaunchKernelGGL(k_get_blocks, dim3(unsigned(ceil_div(n, kBlock))), dim3(kBlock), 0, s, p->b, p->z, U, V, bp, bl);
    return hipGetLastError() == hipSuccess ? POBA_OK : POBA_ERR_HIP;
}

}  // extern "C"
