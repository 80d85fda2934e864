// One Levenberg-Marquardt iteration on the device (Sec. 5.1 "LM loop") for
// every problem of a handle at once.
//
// The accept/reject decision needs F at the trial state and the decrease of
// the undamped linear model, L(0) - L(dx) = -sum_i (r_i . e_i + e_i . e_i / 2)
// with e_i = J_p dx_c + J_l dx_l; both are float64 sums over the problem's
// observations computed in one camera-major pass.  Every decision (gain
// ratio, damping update, convergence) is taken on the device by one thread
// per problem, so a step needs no host synchronisation and can be captured in
// a graph.  A problem that is done leaves its state untouched.
#include "camera_model.hpp"
#include "device_ops.hpp"
#include "kernels.hpp"

namespace poba {

__global__ void k_lm_init(poba_lm_state* states, int32_t np, double lambda0) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < np) {
        poba_lm_state* st = states + j;
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

// Per-problem flags from the LM states; one block counts the active problems
// and whether any of them needs a new linearisation.
__global__ __launch_bounds__(kReduceBlock) void k_begin_step(Ctrl* ctrl, PCtrl* pctl, const poba_lm_state* st,
                                                             int32_t np) {
    int n_active = 0, any_lin = 0;
    for (int32_t base = 0; base < np; base += blockDim.x) {
        const int32_t j = base + threadIdx.x;
        int active = 0, lin = 0;
        if (j < np) {
            active = st[j].done ? 0 : 1;
            lin = active && st[j].need_linearize;
            PCtrl& q = pctl[j];
            q.active = active;
            q.lambda = st[j].lambda;
            q.stopped = 0;
            q.stop_order = 0;
            q.status = 0;
            q.accepted = 0;
        }
        n_active += __syncthreads_count(active);
        any_lin |= __syncthreads_or(lin);
    }
    if (threadIdx.x == 0) {
        ctrl->active = n_active;
        ctrl->running = n_active;
        ctrl->lin = any_lin ? 1 : 0;
    }
}

// cams_new = cams + dx_p; per landmark the trial position lms + dx_l and the
// step dx_l side by side in one 64-byte record, so that the evaluation's
// gather of both takes one line.
__global__ __launch_bounds__(kBlock) void k_trial(Buffers b, Sizes z, const double* cams, const double* lms,
                                                  const Ctrl* ctrl) {
    if (!ctrl->active) return;
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i < int64_t(z.nc) * 9) b.cams_new[i] = cams[i] + b.dxp[i];
    if (i < int64_t(z.nl)) {
        double d[3], x[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            d[k] = b.dxl[3 * i + k];
            x[k] = lms[3 * i + k] + d[k];
        }
        double2* o = reinterpret_cast<double2*>(b.lm_trial + 8 * i);
        o[0] = make_double2(x[0], x[1]);
        o[1] = make_double2(x[2], d[0]);
        o[2] = make_double2(d[1], d[2]);
    }
}

// The trial position and step of landmark l from its record.
__device__ __forceinline__ void load_lm_trial(const double* t, int64_t l, double* X, double* dl) {
    const double2* q = reinterpret_cast<const double2*>(t + 8 * l);
    const double2 a = q[0], c = q[1], e = q[2];
    X[0] = a.x;
    X[1] = a.y;
    X[2] = c.x;
    dl[0] = c.y;
    dl[1] = e.x;
    dl[2] = e.y;
}

// Threads per piece (measured at the city size): one wavefront over point
// records, whose blocks are rebuilt in float64 (10% faster than four); four
// over stored blocks (one was 3% slower).
constexpr int eval_threads(bool point) { return point ? kWave : kBlock; }

// F(x + dx) and L(0) - L(dx) over all observations, camera-major: one block
// per camera piece (the camera's record and step are the same for the block);
// the piece's partial sums go to its slot of piece_red.  Over stored blocks
// each thread takes U observations at a time, all their loads (landmark
// index, then the trial landmark and its step) issued before any of them is
// evaluated, so the dependent gathers of U observations overlap.
template <typename TJ, bool PT, int NT>
__global__ __launch_bounds__(NT) void k_eval(Buffers b, Sizes z, int loss, double delta, const Ctrl* ctrl) {
    __shared__ double lds[(NT / kWave) * 3];
    if (!ctrl->active) return;
    double cost = 0.0, model = 0.0, bad = 0.0;
    const PieceRec pr = b.sched_rec[blockIdx.x];  // piece, its range, camera and problem in one load
    // the same for the whole block: wave-uniform values, so the camera's
    // record and step come through the scalar cache
    const int32_t p = __builtin_amdgcn_readfirstlane(pr.p);
    if (p < 0 || !b.pctl[__builtin_amdgcn_readfirstlane(pr.prob)].active) return;
    {
        const int64_t c = __builtin_amdgcn_readfirstlane(pr.cam);
        const int32_t a = __builtin_amdgcn_readfirstlane(pr.begin), e = __builtin_amdgcn_readfirstlane(pr.end);
        const double* rec = b.cam_rec + kCamRec * c;
        const double* dp = b.dxp + 9 * c;
        // one observation's terms from its loaded data (added only where `use`)
        auto term = [&](bool use, const double* X, const double* dl, const double* o, const double* r,
                        const double* J) {
            double px[2];
            project_rec(rec, X, px);
            const double e0 = px[0] - o[0], e1 = px[1] - o[1];
            const double s2 = e0 * e0 + e1 * e1;
            double rho = s2, wgt;
            if (loss == POBA_LOSS_HUBER) huber(s2, delta, rho, wgt);
            double m0 = J[18] * dl[0] + J[19] * dl[1] + J[20] * dl[2];
            double m1 = J[21] * dl[0] + J[22] * dl[1] + J[23] * dl[2];
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                m0 += J[k] * dp[k];
                m1 += J[9 + k] * dp[k];
            }
            const double md = r[0] * m0 + r[1] * m1 + 0.5 * (m0 * m0 + m1 * m1);
            cost += use ? 0.5 * rho : 0.0;
            model -= use ? md : 0.0;
            if (use && !isfinite(rho)) bad = 1.0;
        };
        if constexpr (PT) {
            for (int32_t i = a + threadIdx.x; i < e; i += NT) {
                const int64_t l = b.co_lm[i];
                double X[3], dl[3], J[24];
                load_lm_trial(b.lm_trial, l, X, dl);
                Rec<TJ, PT>::template jac<double>(b, z, b.J_co, i, c, J);
                const double o[2] = {b.obs_co[2 * int64_t(i)], b.obs_co[2 * int64_t(i) + 1]};
                const double r[2] = {b.r_co[2 * int64_t(i)], b.r_co[2 * int64_t(i) + 1]};
                term(true, X, dl, o, r, J);
            }
        } else {
            constexpr int U = sizeof(TJ) == 8 ? 1 : 2;  // float64 records: one (registers)
            for (int32_t base = a + threadIdx.x; base < e; base += U * NT) {
                int32_t ii[U];
                bool ok[U];
                int64_t l[U];
                RawRec<TJ> raw[U];
                double X[U][3], dl[U][3], o[U][2], r[U][2];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    ok[u] = base + u * NT < e;
                    ii[u] = ok[u] ? base + u * NT : a;  // lanes past the piece read its first position
                    l[u] = b.co_lm[ii[u]];
                    load_raw<TJ>(b.J_co, z.npad, ii[u], raw[u]);
                    o[u][0] = b.obs_co[2 * int64_t(ii[u])];
                    o[u][1] = b.obs_co[2 * int64_t(ii[u]) + 1];
                    r[u][0] = b.r_co[2 * int64_t(ii[u])];
                    r[u][1] = b.r_co[2 * int64_t(ii[u]) + 1];
                }
#pragma unroll
                for (int u = 0; u < U; ++u) load_lm_trial(b.lm_trial, l[u], X[u], dl[u]);
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    double J[24];
                    unpack<double>(raw[u], J);
                    term(ok[u], X[u], dl[u], o[u], r[u], J);
                }
            }
        }
    }
    double tot[3] = {cost, model, bad};
    block_sum<3>(tot, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) b.piece_red[3 * int64_t(p) + k] = tot[k];
    }
}

// Per problem (one block each): F(x + dx) and the model decrease from its
// pieces in piece order.
__global__ __launch_bounds__(kBlock) void k_eval_final(Buffers b, const Ctrl* ctrl) {
    __shared__ double lds[kWavesPerBlock * 3];
    if (!ctrl->active) return;
    PCtrl& q = b.pctl[blockIdx.x];
    if (!q.active) return;
    const int32_t a = b.prob_piece_off[blockIdx.x], e = b.prob_piece_off[blockIdx.x + 1];
    double out[3];
    sum_partials<3>(b.piece_red + 3 * int64_t(a), uint32_t(e - a), out, lds);
    if (threadIdx.x == 0) {
        q.cost_new = out[2] != 0.0 ? __builtin_nan("") : out[0];
        q.model = out[1];
    }
}

struct LMParams {
    double func_tol, eta, lambda_min, lambda_max;
    int32_t max_iters;
};

// Gain ratio, accept / reject, damping update and termination, one thread
// per problem.
__global__ void k_control(Buffers b, int32_t np, poba_lm_state* states, LMParams o) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= np) return;
    PCtrl& q = b.pctl[j];
    if (!q.active) return;
    poba_lm_state* st = states + j;
    const double F = st->cost;
    const double Fn = q.cost_new;
    const double L = q.model;
    const double rho = (isfinite(Fn) && L > 0.0) ? (F - Fn) / L : -__builtin_inf();
    const int accepted = rho > o.eta ? 1 : 0;
    st->iteration += 1;
    st->accepted = accepted;
    st->gain = rho;
    st->cost_new = Fn;
    st->model_decrease = L;
    st->stop_order = q.stop_order;
    st->status |= q.status;
    q.accepted = accepted;
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

// Accepted step: the trial state becomes the state (problem by problem).
__global__ __launch_bounds__(kBlock) void k_apply(Buffers b, Sizes z, double* cams, double* lms, const Ctrl* ctrl) {
    if (!ctrl->active) return;
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i < int64_t(z.nc) * 9) {
        const PCtrl& q = b.pctl[b.cam_prob[i / 9]];
        if (q.active && q.accepted) cams[i] = b.cams_new[i];
    }
    if (i < int64_t(z.nl) * 3) {
        const PCtrl& q = b.pctl[b.lm_prob[i / 3]];
        if (q.active && q.accepted) lms[i] = b.lm_trial[8 * (i / 3) + i % 3];
    }
}

}  // namespace poba

using namespace poba;

extern "C" {

poba_status poba_lm_init(poba_problem p, poba_lm_state* st, const poba_lm_options* o, poba_stream stream) {
    (void)hipGetLastError();  // report only this call's launch errors
    if (!p || !st || !o) return POBA_ERR_INVALID_ARG;
    if (!(o->lambda0 > 0.0)) return POBA_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_lm_init, dim3(unsigned(ceil_div(p->z.np, kBlock))), dim3(kBlock), 0,
                       reinterpret_cast<hipStream_t>(stream), st, p->z.np, o->lambda0);
    return hipGetLastError() == hipSuccess ? POBA_OK : POBA_ERR_HIP;
}

}  // extern "C"

namespace {

bool bad_options(const poba_lm_options* o) {
    return o->m < 0 || o->m > 100000 || !(o->eps >= 0.0) || o->max_iters < 1 || !(o->lambda_min > 0.0) ||
           !(o->lambda_max >= o->lambda_min);
}

// Problem flags from the LM states, and the linearisation where a step asks for it.
poba_status lm_begin(Problem* p, double* cams, double* lms, poba_lm_state* st, hipStream_t s) {
    const Buffers& b = p->b;
    hipLaunchKernelGGL(k_begin_step, dim3(1), dim3(kReduceBlock), 0, s, b.ctrl, b.pctl, st, p->z.np);
    return launch_linearize(p, cams, lms, &b.ctrl->lin, nullptr, st, s);
}

__global__ __launch_bounds__(kBlock) void k_take_step(Buffers b, Sizes z, const double* __restrict__ dxp,
                                                      const double* __restrict__ dxl) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i < int64_t(z.nc) * 9) b.dxp[i] = dxp[i];
    if (i < int64_t(z.nl) * 3) b.dxl[i] = dxl[i];
}

// Trial state, F there and the model decrease, the decision and the damping
// update for the step in b.dxp, b.dxl.
poba_status lm_finish(Problem* p, double* cams, double* lms, poba_lm_state* st, const poba_lm_options* o,
                      hipStream_t s) {
    const Buffers& b = p->b;
    const Sizes& z = p->z;
    poba_status rc = POBA_OK;
    const int64_t nstate = std::max<int64_t>(int64_t(z.nc) * 9, int64_t(z.nl) * 3);
    const dim3 g_state(unsigned(ceil_div(nstate, kBlock)));
    {
        ProfScope pr(p, POBA_K_EVAL, s);
        hipLaunchKernelGGL(k_trial, g_state, dim3(kBlock), 0, s, b, z, cams, lms, b.ctrl);
        rc = launch_cam_prep(p, b.cams_new, &b.ctrl->active, b.cam_rec, s);
        if (rc) return rc;
        const dim3 g_tiles(unsigned(std::max<int64_t>(p->sched_len, 1)));
        const int loss = p->d.loss;
        const double delta = p->d.huber_delta;
        if (z.point) {
            if (p->d.precision == POBA_F64)
                hipLaunchKernelGGL((k_eval<double, true, eval_threads(true)>), g_tiles, dim3(eval_threads(true)), 0, s, b, z, loss, delta, b.ctrl);
            else
                hipLaunchKernelGGL((k_eval<float, true, eval_threads(true)>), g_tiles, dim3(eval_threads(true)), 0, s, b, z, loss, delta, b.ctrl);
        } else {
            auto eval = [&](auto tj) {
                using TJ = decltype(tj);
                if (small_pieces(p))
                    hipLaunchKernelGGL((k_eval<TJ, false, kWave>), g_tiles, dim3(kWave), 0, s, b, z, loss, delta, b.ctrl);
                else
                    hipLaunchKernelGGL((k_eval<TJ, false, eval_threads(false)>), g_tiles, dim3(eval_threads(false)), 0, s,
                                       b, z, loss, delta, b.ctrl);
            };
            switch (p->d.precision) {
                case POBA_F64: eval(double()); break;
                case POBA_F32: eval(float()); break;
                default: eval(bf16_t()); break;
            }
        }
        hipLaunchKernelGGL(k_eval_final, dim3(unsigned(z.np)), dim3(kBlock), 0, s, b, b.ctrl);
    }
    LMParams prm{o->func_tol, o->eta, o->lambda_min, o->lambda_max, o->max_iters};
    hipLaunchKernelGGL(k_control, dim3(unsigned(ceil_div(z.np, kBlock))), dim3(kBlock), 0, s, b, z.np, st, prm);
    hipLaunchKernelGGL(k_apply, g_state, dim3(kBlock), 0, s, b, z, cams, lms, b.ctrl);
    return hipGetLastError() == hipSuccess ? POBA_OK : POBA_ERR_HIP;
}

}  // namespace

extern "C" {

poba_status poba_lm_step(poba_problem p, double* cams, double* lms, poba_lm_state* st, const poba_lm_options* o,
                         poba_stream stream) {
    (void)hipGetLastError();  // report only this call's launch errors
    if (!p || !cams || !lms || !st || !o || bad_options(o)) return POBA_ERR_INVALID_ARG;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    poba_status rc = lm_begin(p, cams, lms, st, s);
    if (rc) return rc;
    rc = launch_solve(p, o->m, o->eps, p->b.dxp, p->b.dxl, nullptr, s);
    if (rc) return rc;
    return lm_finish(p, cams, lms, st, o, s);
}

poba_status poba_lm_begin(poba_problem p, double* cams, double* lms, poba_lm_state* st, poba_stream stream) {
    (void)hipGetLastError();  // report only this call's launch errors
    if (!p || !cams || !lms || !st) return POBA_ERR_INVALID_ARG;
    return lm_begin(p, cams, lms, st, reinterpret_cast<hipStream_t>(stream));
}

poba_status poba_lm_finish(poba_problem p, double* cams, double* lms, poba_lm_state* st, const poba_lm_options* o,
                           const double* dx_cams, const double* dx_lms, poba_stream stream) {
    (void)hipGetLastError();  // report only this call's launch errors
    if (!p || !cams || !lms || !st || !o || !dx_cams || !dx_lms || bad_options(o)) return POBA_ERR_INVALID_ARG;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const Buffers& b = p->b;
    const Sizes& z = p->z;
    // the flags again (calls between begin and finish may have changed them)
    hipLaunchKernelGGL(k_begin_step, dim3(1), dim3(kReduceBlock), 0, s, b.ctrl, b.pctl, st, z.np);
    const int64_t nstate = std::max<int64_t>(int64_t(z.nc) * 9, int64_t(z.nl) * 3);
    hipLaunchKernelGGL(k_take_step, dim3(unsigned(ceil_div(nstate, kBlock))), dim3(kBlock), 0, s, b, z, dx_cams,
                       dx_lms);
    if (hipGetLastError() != hipSuccess) return POBA_ERR_HIP;
    return lm_finish(p, cams, lms, st, o, s);
}

}  // extern "C"
