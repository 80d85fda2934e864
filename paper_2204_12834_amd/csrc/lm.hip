// One Levenberg-Marquardt iteration on the device (Sec. 5.1 "LM loop").
//
// The accept/reject decision needs F at the trial state and the decrease of
// the undamped linear model, L(0) - L(dx) = -sum_i (r_i . e_i + e_i . e_i / 2)
// with e_i = J_p dx_c + J_l dx_l; both are float64 sums over all observations
// computed in one landmark-major pass.  Every decision (gain ratio, damping
// update, convergence) is taken by a single device thread, so a step needs no
// host synchronisation and can be captured in a graph.
#include "camera_model.hpp"
#include "device_ops.hpp"
#include "kernels.hpp"

namespace poba {

__global__ void k_lm_init(poba_lm_state* st, double lambda0) {
    if (threadIdx.x == 0) {
        st->lambda = lambda0;
        st->nu = 2.0;
        st->cost = 0.0;
        st->cost_new = 0.0;
        st->model_decrease = 0.0;
        st->gain = 0.0;
        st->iteration = 0;
        st->accepted = 0;
        st->done = 0;
        st->need_linearize = 1;
        st->stop_order = 0;
        st->status = 0;
        st->n_accepted = 0;
        st->converged = 0;
    }
}

__global__ void k_begin_step(Ctrl* ctrl, const poba_lm_state* st) {
    if (threadIdx.x == 0) {
        const int active = st->done ? 0 : 1;
        ctrl->active = active;
        ctrl->lin = active && st->need_linearize;
        ctrl->lambda = st->lambda;
        ctrl->stopped = 0;
        ctrl->stop_order = 0;
        ctrl->status = 0;
        ctrl->accepted = 0;
    }
}

// cams_new = cams + dx_p, lms_new = lms + dx_l.
__global__ __launch_bounds__(kBlock) void k_trial(Buffers b, Sizes z, const double* cams, const double* lms,
                                                  const Ctrl* ctrl) {
    if (!ctrl->active) return;
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i < int64_t(z.nc) * 9) b.cams_new[i] = cams[i] + b.dxp[i];
    if (i < int64_t(z.nl) * 3) b.lms_new[i] = lms[i] + b.dxl[i];
}

// F(x + dx) and L(0) - L(dx) over all observations, camera-major: one block
// per camera piece (the camera's record and step are the same for the block).
template <typename TJ>
__global__ __launch_bounds__(kBlock) void k_eval(Buffers b, Sizes z, int loss, double delta, Ctrl* ctrl) {
    __shared__ double lds[kWavesPerBlock * 3];
    if (!ctrl->active) return;
    double cost = 0.0, model = 0.0, bad = 0.0;
    const int32_t p = b.sched[blockIdx.x];
    if (p >= 0) {
        const int64_t c = b.piece_cam[p];
        const int32_t a = b.piece_begin[p], e = b.piece_end[p];
        const double* rec = b.cam_rec + kCamRec * c;
        const double* dp = b.dxp + 9 * c;
        for (int32_t i = a + threadIdx.x; i < e; i += kBlock) {
            const int64_t l = b.co_lm[i];
            double X[3], px[2];
#pragma unroll
            for (int k = 0; k < 3; ++k) X[k] = b.lms_new[3 * l + k];
            project_rec(rec, X, px);
            const double e0 = px[0] - b.obs_co[2 * int64_t(i)], e1 = px[1] - b.obs_co[2 * int64_t(i) + 1];
            const double s2 = e0 * e0 + e1 * e1;
            double rho = s2, wgt;
            if (loss == POBA_LOSS_HUBER) huber(s2, delta, rho, wgt);
            cost += 0.5 * rho;
            if (!isfinite(rho)) bad = 1.0;
            double J[24];
            load_J<TJ, double>(b.J_co, z.npad, i, J);
            const double* dl = b.dxl + 3 * l;
            double m0 = J[18] * dl[0] + J[19] * dl[1] + J[20] * dl[2];
            double m1 = J[21] * dl[0] + J[22] * dl[1] + J[23] * dl[2];
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                m0 += J[k] * dp[k];
                m1 += J[9 + k] * dp[k];
            }
            const double r0 = b.r_co[2 * int64_t(i)], r1 = b.r_co[2 * int64_t(i) + 1];
            model -= r0 * m0 + r1 * m1 + 0.5 * (m0 * m0 + m1 * m1);
        }
    }
    double tot[3] = {cost, model, bad};
    block_sum<3>(tot, lds);
    store_block_partial<3>(tot, b.red_part);
}

__global__ __launch_bounds__(kReduceBlock) void k_eval_final(Buffers b, uint32_t nblocks, Ctrl* ctrl) {
    __shared__ double lds[(kReduceBlock / kWave) * 3];
    if (!ctrl->active) return;
    double out[3];
    sum_partials<3>(b.red_part, nblocks, out, lds);
    if (threadIdx.x == 0) {
        ctrl->red[1] = out[2] != 0.0 ? __builtin_nan("") : out[0];
        ctrl->red[2] = out[1];
    }
}

struct LMParams {
    double func_tol, eta, lambda_min, lambda_max;
    int32_t max_iters;
};

// Gain ratio, accept / reject, damping update and termination.
__global__ void k_control(Ctrl* ctrl, poba_lm_state* st, LMParams o) {
    if (threadIdx.x != 0 || !ctrl->active) return;
    const double F = st->cost;
    const double Fn = ctrl->red[1];
    const double L = ctrl->red[2];
    const double rho = (isfinite(Fn) && L > 0.0) ? (F - Fn) / L : -__builtin_inf();
    const int accepted = rho > o.eta ? 1 : 0;
    st->iteration += 1;
    st->accepted = accepted;
    st->gain = rho;
    st->cost_new = Fn;
    st->model_decrease = L;
    st->stop_order = ctrl->stop_order;
    st->status |= ctrl->status;
    ctrl->accepted = accepted;
    double lam = st->lambda;
    if (accepted) {
        const double rel = F > 0.0 ? (F - Fn) / F : 0.0;
        const double t = 2.0 * rho - 1.0;
        lam *= fmax(1.0 / 3.0, 1.0 - t * t * t);
        st->nu = 2.0;
        st->cost = Fn;
        st->need_linearize = 1;
        st->n_accepted += 1;
        if (rel < o.func_tol) {
            st->done = 1;
            st->converged = 1;
        }
    } else {
        lam *= st->nu;
        st->nu *= 2.0;
        st->need_linearize = 0;
    }
    st->lambda = fmin(fmax(lam, o.lambda_min), o.lambda_max);
    if (st->iteration >= o.max_iters) st->done = 1;
}

// Accepted step: the trial state becomes the state.
__global__ __launch_bounds__(kBlock) void k_apply(Buffers b, Sizes z, double* cams, double* lms, const Ctrl* ctrl) {
    if (!ctrl->active || !ctrl->accepted) return;
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i < int64_t(z.nc) * 9) cams[i] = b.cams_new[i];
    if (i < int64_t(z.nl) * 3) lms[i] = b.lms_new[i];
}

}  // namespace poba

using namespace poba;

extern "C" {

poba_status poba_lm_init(poba_problem p, poba_lm_state* st, const poba_lm_options* o, poba_stream stream) {
    (void)hipGetLastError();  // report only this call's launch errors
    if (!p || !st || !o) return POBA_ERR_INVALID_ARG;
    if (!(o->lambda0 > 0.0)) return POBA_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_lm_init, dim3(1), dim3(64), 0, reinterpret_cast<hipStream_t>(stream), st, o->lambda0);
    return hipGetLastError() == hipSuccess ? POBA_OK : POBA_ERR_HIP;
}

poba_status poba_lm_step(poba_problem p, double* cams, double* lms, poba_lm_state* st, const poba_lm_options* o,
                         poba_stream stream) {
    (void)hipGetLastError();  // report only this call's launch errors
    if (!p || !cams || !lms || !st || !o) return POBA_ERR_INVALID_ARG;
    if (o->m < 0 || o->m > 100000 || !(o->eps >= 0.0) || o->max_iters < 1 || !(o->lambda_min > 0.0) ||
        !(o->lambda_max >= o->lambda_min))
        return POBA_ERR_INVALID_ARG;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const Buffers& b = p->b;
    const Sizes& z = p->z;
    hipLaunchKernelGGL(k_begin_step, dim3(1), dim3(64), 0, s, b.ctrl, st);
    poba_status rc = launch_linearize(p, cams, lms, &b.ctrl->lin, nullptr, &st->cost, s);
    if (rc) return rc;
    rc = launch_solve(p, o->m, o->eps, b.dxp, b.dxl, nullptr, s);
    if (rc) return rc;
    const int64_t nstate = std::max<int64_t>(int64_t(z.nc) * 9, int64_t(z.nl) * 3);
    const dim3 g_state(unsigned(ceil_div(nstate, kBlock)));
    {
        ProfScope pr(p, POBA_K_EVAL, s);
        hipLaunchKernelGGL(k_trial, g_state, dim3(kBlock), 0, s, b, z, cams, lms, b.ctrl);
        rc = launch_cam_prep(p, b.cams_new, &b.ctrl->active, s);
        if (rc) return rc;
        const dim3 g_tiles(unsigned(std::max<int64_t>(p->sched_len, 1)));
        switch (p->d.precision) {
            case POBA_F64: hipLaunchKernelGGL(k_eval<double>, g_tiles, dim3(kBlock), 0, s, b, z, p->d.loss, p->d.huber_delta, b.ctrl); break;
            case POBA_F32: hipLaunchKernelGGL(k_eval<float>, g_tiles, dim3(kBlock), 0, s, b, z, p->d.loss, p->d.huber_delta, b.ctrl); break;
            default: hipLaunchKernelGGL(k_eval<bf16_t>, g_tiles, dim3(kBlock), 0, s, b, z, p->d.loss, p->d.huber_delta, b.ctrl); break;
        }
        hipLaunchKernelGGL(k_eval_final, dim3(1), dim3(kReduceBlock), 0, s, b, unsigned(g_tiles.x), b.ctrl);
    }
    LMParams prm{o->func_tol, o->eta, o->lambda_min, o->lambda_max, o->max_iters};
    hipLaunchKernelGGL(k_control, dim3(1), dim3(64), 0, s, b.ctrl, st, prm);
    hipLaunchKernelGGL(k_apply, g_state, dim3(kBlock), 0, s, b, z, cams, lms, b.ctrl);
    return hipGetLastError() == hipSuccess ? POBA_OK : POBA_ERR_HIP;
}

}  // extern "C"
