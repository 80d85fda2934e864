// Preconditioned conjugate gradients (Hestenes and Stiefel) on the reduced
// camera system S dx_p = -b~ of Sec. 4.2 (eqs. Schur, Sx), the solver the
// paper compares the power series against in Sec. 2 (Fig. 2):
//
//   x = 0, r = -b~, z = M^-1 r, p = z
//   per iteration: q = S p, alpha = (r.z) / (p.q), x += alpha p,
//                  r -= alpha q, stop when |r| <= tol |b~|,
//                  z = M^-1 r, beta = (r.z)_new / (r.z)_old, p = z + beta p
//
// with S p = U_lambda p - W V_lambda^-1 W^T p evaluated matrix-free in float64
// (the landmark and camera passes over the stored records, blocks widened,
// V^-1 recomputed in float64), and one of three preconditioners M^-1:
//   none:          the identity;
//   Schur-Jacobi:  the inverted 9x9 diagonal blocks of S,
//                  S_cc = U_lambda,c - sum_l W_cl V_l^-1 W_cl^T;
//   power series:  S~(m) = sum_{i<=m} P^i U^-1 (eq. S_approx), i.e. the series
//                  of the power solve run on the right-hand side r, in the
//                  handle's storage precision (4m products per application).
// Every problem of a batch runs its own recursion; a problem leaves the
// iteration (inactive) when it converges.  The host reads how many remain
// every few iterations and stops when none does.
#include "device_ops.hpp"
#include "kernels.hpp"

namespace poba {

namespace {

constexpr int kCheckEvery = 4;  // iterations between host reads of the active count

enum PcgPrecond { kPcNone = 0, kPcJacobi = 1, kPcPower = 2 };

__device__ __forceinline__ double* cg_vec(const Buffers& b, const Sizes& z, int k) {
    return b.cg + int64_t(k) * 9 * z.nc;
}
enum { kX = 0, kR = 1, kZ = 2, kP = 3, kQ = 4 };

// A problem leaves the iteration: skipped by every later kernel of the call.
__device__ __forceinline__ void pcg_leave(PCtrl& q, Ctrl* ctrl) {
    q.active = 0;
    atomicSub(&ctrl->active, 1);
    atomicSub(&ctrl->running, 1);
}

// ------------------------------------------------- Schur-Jacobi blocks --
//
// One wavefront per camera c over its camera-major observations; the observation
// of landmark l contributes W_cl V_l^-1 W_cl^T with W_cl = J_p^T J_l.  When
// the handle has repeated (camera, landmark) pairs (DUPS), W_cl sums J_p^T J_l
// over every observation of l by camera c (found in the landmark-major
// segment of l) and only the first of them in that segment contributes, so a
// repeated pair enters once with its summed block.  The 45 upper entries are
// summed over the lanes in a fixed order (through LDS); lanes 0..44 write
// S_cc = U_c + lambda D_c - sum (inverted by k_sj_invert).
template <typename TJ, bool PT, bool DUPS>
__global__ __launch_bounds__(kWave) void k_sj_blocks(Buffers b, Sizes z, const Ctrl* ctrl) {
    __shared__ double lds[45][kWave];
    if (!ctrl->active) return;
    const int32_t c = blockIdx.x;
    PCtrl& q = b.pctl[b.cam_prob[c]];
    if (!q.active) return;
    const double lam = q.lambda;
    double acc[45];
#pragma unroll
    for (int k = 0; k < 45; ++k) acc[k] = 0.0;
    const int32_t i0 = b.cam_off[c], i1 = b.cam_off[c + 1];
    for (int32_t i = i0 + threadIdx.x; i < i1; i += kWave) {
        const int32_t l = b.co_lm[i];
        const int32_t seg = b.co_seg[i];
        double W[27];  // W_cl, 9x3 row-major
#pragma unroll
        for (int k = 0; k < 27; ++k) W[k] = 0.0;
        auto add_w = [&](const void* base, int64_t pos) {
            double J[24];
            Rec<TJ, PT>::template jac<double>(b, z, base, pos, c, J);
#pragma unroll
            for (int r = 0; r < 9; ++r)
#pragma unroll
                for (int k = 0; k < 3; ++k) W[3 * r + k] += J[r] * J[18 + k] + J[9 + r] * J[21 + k];
        };
        int32_t first = -1, count = 1;
        const int32_t j1 = DUPS ? b.lm_off[l + 1] : 0;
        if (DUPS) {
            count = 0;
            for (int32_t j = b.lm_off[l]; j < j1; ++j) {
                if (int32_t(b.lo_cam[j] & kIndexMask) == c) {
                    if (first < 0) first = j;
                    ++count;
                }
            }
        }
        if (count <= 1) {
            add_w(b.J_co, i);
        } else {
            if (b.perm_l[first] != b.perm_c[i]) continue;
            for (int32_t j = first; j < j1; ++j)
                if (int32_t(b.lo_cam[j] & kIndexMask) == c) add_w(b.J_lo, j);
        }
        double Vd[6], dd[3], inv[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) Vd[k] = b.V[6 * int64_t(l) + k];
#pragma unroll
        for (int k = 0; k < 3; ++k) dd[k] = b.Dl[3 * int64_t(seg) + k];
        inv3_damped(Vd, lam, dd, inv);
        int e = 0;
#pragma unroll
        for (int r = 0; r < 9; ++r) {
            double y[3];  // row r of W V^-1
            sym3_apply(inv, W + 3 * r, y);
#pragma unroll
            for (int k = r; k < 9; ++k, ++e) acc[e] += y[0] * W[3 * k] + y[1] * W[3 * k + 1] + y[2] * W[3 * k + 2];
        }
    }
    // lane e < 45 sums entry e over the lanes in lane order
#pragma unroll
    for (int k = 0; k < 45; ++k) lds[k][threadIdx.x] = acc[k];
    __syncthreads();
    const int e = threadIdx.x;
    if (e >= 45) return;
    double sum = 0.0;
    for (int k = 0; k < kWave; ++k) sum += lds[e][k];
    int r = 0, base = 0;  // entry e is (r, k) of the upper triangle, row-major
    while (e >= base + 9 - r) {
        base += 9 - r;
        ++r;
    }
    const int k = r + (e - base);
    double v = b.U[81 * int64_t(c) + 9 * r + k] - sum;
    if (k == r) v += lam * b.Dp[9 * int64_t(c) + r];
    double* out = b.sj + 81 * int64_t(c);
    out[9 * r + k] = v;
    out[9 * k + r] = v;
}

// S_cc^-1 in place, one thread per camera.
__global__ __launch_bounds__(kBlock) void k_sj_invert(Buffers b, Sizes z, const Ctrl* ctrl) {
    if (!ctrl->active) return;
    const int32_t c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= z.nc) return;
    PCtrl& q = b.pctl[b.cam_prob[c]];
    if (!q.active) return;
    double* out = b.sj + 81 * int64_t(c);
    double L[81];
#pragma unroll
    for (int k = 0; k < 81; ++k) L[k] = out[k];
    if (!spd_inverse9(L, out)) {
        // not invertible: the preconditioner falls back to the identity here
#pragma unroll
        for (int k = 0; k < 81; ++k) out[k] = (k % 10 == 0) ? 1.0 : 0.0;
        atomicOr(&q.status, POBA_ERR_NOT_SPD);
    }
}

__global__ __launch_bounds__(kBlock) void k_clear_flag(int32_t* flag) {
    if (threadIdx.x == 0) *flag = 0;
}

// flag = 1 if some camera observes some landmark more than once: every
// landmark-major position compares its camera with the earlier positions of
// its segment (back to the segment's head).
__global__ __launch_bounds__(kBlock) void k_find_repeats(Buffers b, Sizes z, int32_t* flag) {
    const int64_t j = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (j >= z.N) return;
    const uint32_t w = b.lo_cam[j];
    if (w & kHeadBit) return;
    const uint32_t c = w & kIndexMask;
    for (int64_t k = j - 1; k >= 0; --k) {
        const uint32_t v = b.lo_cam[k];
        if ((v & kIndexMask) == c) {
            *flag = 1;  // every writer stores the same value
            return;
        }
        if (v & kHeadBit) return;
    }
}

// ------------------------------------------------------ per-camera steps --

// q = S p = U_lambda p - (W V^-1 W^T p), the second term summed over the
// camera's pieces; p.q per camera to cam_red.
__global__ __launch_bounds__(kBlock) void k_pcg_q(Buffers b, Sizes z, const Ctrl* ctrl) {
    if (!ctrl->active) return;
    const int32_t c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= z.nc) return;
    const PCtrl& qc = b.pctl[b.cam_prob[c]];
    if (!qc.active) return;
    const double* pv = cg_vec(b, z, kP) + 9 * int64_t(c);
    double* qv = cg_vec(b, z, kQ) + 9 * int64_t(c);
    double p[9], u[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        p[k] = pv[k];
        u[k] = 0.0;
    }
    for (int32_t pc = b.cam_piece[c]; pc < b.cam_piece[c + 1]; ++pc) {
#pragma unroll
        for (int k = 0; k < 9; ++k) u[k] += b.part[9 * int64_t(pc) + k];
    }
    const double* U = b.U + 81 * int64_t(c);
    double pq = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        double a = qc.lambda * b.Dp[9 * int64_t(c) + k] * p[k];
#pragma unroll
        for (int j = 0; j < 9; ++j) a += U[9 * k + j] * p[j];
        a -= u[k];
        qv[k] = a;
        pq += p[k] * a;
    }
    b.cam_red[2 * int64_t(c)] = pq;
    b.cam_red[2 * int64_t(c) + 1] = 0.0;
}

// init: x = 0, r = -bt (b~, or b_p for a handle without observations); else
// x += alpha p, r -= alpha q.  Then the
// preconditioner where it is per camera (none: z = r; Schur-Jacobi:
// z = S_cc^-1 r) with r.z and r.r to cam_red, or for the power series its
// order 0, v = U^-1 r, into the series' term and sum.
template <int PC>
__global__ __launch_bounds__(kBlock) void k_pcg_update(Buffers b, Sizes z, int init, const double* __restrict__ bt,
                                                       const Ctrl* ctrl) {
    if (!ctrl->active) return;
    const int32_t c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= z.nc) return;
    const int32_t prob = b.cam_prob[c];
    if (!b.pctl[prob].active) return;
    const int64_t o = 9 * int64_t(c);
    double* xv = cg_vec(b, z, kX) + o;
    double* rv = cg_vec(b, z, kR) + o;
    double r[9];
    if (init) {
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            xv[k] = 0.0;
            r[k] = -bt[o + k];
            rv[k] = r[k];
        }
    } else {
        const double alpha = b.pcg_ctl[prob].alpha;
        const double* pv = cg_vec(b, z, kP) + o;
        const double* qv = cg_vec(b, z, kQ) + o;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            xv[k] += alpha * pv[k];
            r[k] = rv[k] - alpha * qv[k];
            rv[k] = r[k];
        }
    }
    if (PC == kPcPower) {
        const double* Ui = b.Uinv + 81 * int64_t(c);
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            double v = 0.0;
#pragma unroll
            for (int j = 0; j < 9; ++j) v += Ui[9 * k + j] * r[j];
            b.v[o + k] = v;
            b.x[o + k] = v;
        }
        return;
    }
    double zc[9];
    if (PC == kPcJacobi) {
        const double* Si = b.sj + 81 * int64_t(c);
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            double v = 0.0;
#pragma unroll
            for (int j = 0; j < 9; ++j) v += Si[9 * k + j] * r[j];
            zc[k] = v;
        }
    } else {
#pragma unroll
        for (int k = 0; k < 9; ++k) zc[k] = r[k];
    }
    double* zv = cg_vec(b, z, kZ) + o;
    double rz = 0.0, rr = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        zv[k] = zc[k];
        rz += r[k] * zc[k];
        rr += r[k] * r[k];
    }
    b.cam_red[2 * int64_t(c)] = rz;
    b.cam_red[2 * int64_t(c) + 1] = rr;
}

// Power-series preconditioner: z = the series sum; r.z and r.r to cam_red.
__global__ __launch_bounds__(kBlock) void k_pcg_take_series(Buffers b, Sizes z, const Ctrl* ctrl) {
    if (!ctrl->active) return;
    const int32_t c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= z.nc) return;
    if (!b.pctl[b.cam_prob[c]].active) return;
    const int64_t o = 9 * int64_t(c);
    const double* rv = cg_vec(b, z, kR) + o;
    double* zv = cg_vec(b, z, kZ) + o;
    double rz = 0.0, rr = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const double zk = b.x[o + k], rk = rv[k];
        zv[k] = zk;
        rz += rk * zk;
        rr += rk * rk;
    }
    b.cam_red[2 * int64_t(c)] = rz;
    b.cam_red[2 * int64_t(c) + 1] = rr;
}

// p = z + beta p (beta = 0 at the start).
__global__ __launch_bounds__(kBlock) void k_pcg_dir(Buffers b, Sizes z, const Ctrl* ctrl) {
    if (!ctrl->active) return;
    const int32_t c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= z.nc) return;
    const int32_t prob = b.cam_prob[c];
    if (!b.pctl[prob].active) return;
    const double beta = b.pcg_ctl[prob].beta;
    const int64_t o = 9 * int64_t(c);
    const double* zv = cg_vec(b, z, kZ) + o;
    double* pv = cg_vec(b, z, kP) + o;
#pragma unroll
    for (int k = 0; k < 9; ++k) pv[k] = zv[k] + beta * pv[k];
}

// --------------------------------------------------- per-problem scalars --

// alpha = (r.z) / (p.q) of iteration `it` (one block per problem); a
// non-positive or non-finite p.q ends the problem's iteration (status bit).
__global__ __launch_bounds__(kBlock) void k_pcg_alpha(Buffers b, int32_t np, int32_t it, double* coeffs,
                                                      Ctrl* ctrl) {
    __shared__ double lds[kWavesPerBlock];
    if (!ctrl->active) return;
    const int32_t j = blockIdx.x;
    PCtrl& q = b.pctl[j];
    if (!q.active) return;
    const int32_t c0 = b.prob_cam_off[j], c1 = b.prob_cam_off[j + 1];
    double pq;
    sum_partials<1>(b.cam_red + 2 * int64_t(c0), uint32_t(c1 - c0), &pq, lds, 2);
    if (threadIdx.x != 0) return;
    PcgCtl& g = b.pcg_ctl[j];
    g.iterations = it;
    if (!(pq > 0.0) || !isfinite(pq)) {
        g.alpha = 0.0;
        atomicOr(&q.status, isfinite(pq) ? POBA_ERR_NOT_SPD : POBA_ERR_NONFINITE);
        pcg_leave(q, ctrl);
        return;
    }
    g.alpha = g.rz / pq;
    if (coeffs) coeffs[2 * (int64_t(it - 1) * np + j)] = g.alpha;
}

// After the residual update of iteration `it` (0: the start): |r| against
// tol |b|, then beta = (r.z)_new / (r.z)_old (one block per problem).
__global__ __launch_bounds__(kBlock) void k_pcg_beta(Buffers b, int32_t np, int32_t it, double tol, double* coeffs,
                                                     Ctrl* ctrl) {
    __shared__ double lds[kWavesPerBlock * 2];
    if (!ctrl->active) return;
    const int32_t j = blockIdx.x;
    PCtrl& q = b.pctl[j];
    if (!q.active) return;
    const int32_t c0 = b.prob_cam_off[j], c1 = b.prob_cam_off[j + 1];
    double tot[2];
    sum_partials<2>(b.cam_red + 2 * int64_t(c0), uint32_t(c1 - c0), tot, lds);
    if (threadIdx.x != 0) return;
    PcgCtl& g = b.pcg_ctl[j];
    const double rz = tot[0], rr = tot[1];
    g.r2 = rr;
    if (it == 0) {
        g.b2 = rr;
        g.iterations = 0;
        g.converged = 0;
        g.alpha = 0.0;
        g.beta = 0.0;
        g.rz = rz;
        if (rr == 0.0) {
            g.converged = 1;
            pcg_leave(q, ctrl);
            return;
        }
    } else {
        if (!isfinite(rr)) {
            atomicOr(&q.status, POBA_ERR_NONFINITE);
            pcg_leave(q, ctrl);
            return;
        }
        if (sqrt(rr) <= tol * sqrt(g.b2)) {
            g.converged = 1;
            pcg_leave(q, ctrl);
            return;
        }
        g.beta = rz / g.rz;
        g.rz = rz;
        if (coeffs) coeffs[2 * (int64_t(it - 1) * np + j) + 1] = g.beta;
    }
    if (!(rz > 0.0) || !isfinite(rz)) {
        // M^-1 not positive definite on r (or r.z lost to rounding)
        atomicOr(&q.status, isfinite(rz) ? POBA_ERR_NOT_SPD : POBA_ERR_NONFINITE);
        pcg_leave(q, ctrl);
    }
}

// The camera step into the series sum (read by the back-substitution).
__global__ __launch_bounds__(kBlock) void k_pcg_x_out(Buffers b, Sizes z) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i < int64_t(z.nc) * 9) b.x[i] = cg_vec(b, z, kX)[i];
}

// Info of every problem, which become active again for the back-substitution.
__global__ __launch_bounds__(kReduceBlock) void k_pcg_end(Buffers b, int32_t np, poba_pcg_info* info, Ctrl* ctrl) {
    for (int32_t j = threadIdx.x; j < np; j += blockDim.x) {
        PCtrl& q = b.pctl[j];
        const PcgCtl& g = b.pcg_ctl[j];
        if (info) {
            poba_pcg_info& o = info[j];
            o.iterations = g.iterations;
            o.converged = g.converged;
            o.status = q.status;
            o.reserved = 0;
            o.rel_residual = g.b2 > 0.0 ? sqrt(g.r2 / g.b2) : 0.0;
            o.rz = g.rz;
        }
        q.active = 1;
        q.stopped = 0;
    }
    if (threadIdx.x == 0) {
        ctrl->active = np;
        ctrl->running = np;
    }
}

template <typename TJ, bool PT>
void launch_sj_blocks(Problem* p, hipStream_t s) {
    const dim3 g(unsigned(p->z.nc)), wave(kWave);
    if (p->repeats)
        hipLaunchKernelGGL((k_sj_blocks<TJ, PT, true>), g, wave, 0, s, p->b, p->z, p->b.ctrl);
    else
        hipLaunchKernelGGL((k_sj_blocks<TJ, PT, false>), g, wave, 0, s, p->b, p->z, p->b.ctrl);
    hipLaunchKernelGGL(k_sj_invert, dim3(unsigned(ceil_div(p->z.nc, kBlock))), dim3(kBlock), 0, s, p->b, p->z,
                       p->b.ctrl);
}

poba_status sj_blocks(Problem* p, hipStream_t s) {
    if (p->repeats < 0) {
        // once per handle: does any (camera, landmark) pair repeat?
        int32_t* flag = p->b.scratch_i;
        hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(kBlock), 0, s, flag);
        if (p->z.N > 0)
            hipLaunchKernelGGL(k_find_repeats, dim3(unsigned(ceil_div(p->z.N, kBlock))), dim3(kBlock), 0, s, p->b,
                               p->z, flag);
        int32_t h = 0;
        if (hipMemcpyAsync(&h, flag, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return POBA_ERR_HIP;
        p->repeats = h ? 1 : 0;
    }
    ProfScope pr(p, POBA_K_INVERSE, s);
    if (p->z.point) {
        if (p->d.precision == POBA_F64) launch_sj_blocks<double, true>(p, s);
        else launch_sj_blocks<float, true>(p, s);
    } else {
        switch (p->d.precision) {
            case POBA_F64: launch_sj_blocks<double, false>(p, s); break;
            case POBA_F32: launch_sj_blocks<float, false>(p, s); break;
            default: launch_sj_blocks<bf16_t, false>(p, s); break;
        }
    }
    return hipGetLastError() == hipSuccess ? POBA_OK : POBA_ERR_HIP;
}

// z = M^-1 r after the residual update (init: from x = 0, r = -b~), with
// r.z and r.r per camera in cam_red.
poba_status precondition(Problem* p, int precond, int m, int init, hipStream_t s) {
    const Sizes& z = p->z;
    const dim3 g_cam(unsigned(ceil_div(z.nc, kBlock))), blk(kBlock);
    poba_status st = POBA_OK;
    // without observations b~ = b_p (and no pass writes b~)
    const double* bt = p->npieces > 0 ? p->b.bt : p->b.bp;
    {
        ProfScope pr(p, POBA_K_OTHER, s);
        switch (precond) {
            case kPcNone:
                hipLaunchKernelGGL(k_pcg_update<kPcNone>, g_cam, blk, 0, s, p->b, z, init, bt, p->b.ctrl);
                break;
            case kPcJacobi:
                hipLaunchKernelGGL(k_pcg_update<kPcJacobi>, g_cam, blk, 0, s, p->b, z, init, bt, p->b.ctrl);
                break;
            default:
                hipLaunchKernelGGL(k_pcg_update<kPcPower>, g_cam, blk, 0, s, p->b, z, init, bt, p->b.ctrl);
                break;
        }
    }
    if (precond != kPcPower) return hipGetLastError() == hipSuccess ? POBA_OK : POBA_ERR_HIP;
    {
        ProfScope pr(p, POBA_K_OTHER, s);
        if ((st = launch_load_v(p, p->b.v, s))) return st;
    }
    if ((st = launch_series_orders(p, m, s))) return st;
    ProfScope pr(p, POBA_K_OTHER, s);
    hipLaunchKernelGGL(k_pcg_take_series, g_cam, blk, 0, s, p->b, z, p->b.ctrl);
    return hipGetLastError() == hipSuccess ? POBA_OK : POBA_ERR_HIP;
}

}  // namespace

}  // namespace poba

using namespace poba;

extern "C" {

poba_status poba_pcg_solve(poba_problem p, double lambda, int32_t precond, int32_t m, double tol, int32_t max_iters,
                           double* dx_cams, double* dx_lms, poba_pcg_info* info, double* coeffs,
                           poba_stream stream) {
    (void)hipGetLastError();  // report only this call's launch errors
    if (!p || !dx_cams || !dx_lms) return POBA_ERR_INVALID_ARG;
    if (!(lambda > 0.0) || !(tol >= 0.0) || max_iters < 0 || max_iters > 1000000) return POBA_ERR_INVALID_ARG;
    if (precond < POBA_PRECOND_NONE || precond > POBA_PRECOND_POWER) return POBA_ERR_INVALID_ARG;
    if (precond == POBA_PRECOND_POWER && (m < 0 || m > 100000)) return POBA_ERR_INVALID_ARG;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const Sizes& z = p->z;
    const Buffers& b = p->b;
    const int32_t np = z.np;
    const dim3 g_cam(unsigned(ceil_div(z.nc, kBlock))), blk(kBlock);
    poba_status st;
    if ((st = launch_begin_solve(p, lambda, s))) return st;
    if ((st = launch_solve_prepare(p, s))) return st;
    if (precond == POBA_PRECOND_SCHUR_JACOBI && (st = sj_blocks(p, s))) return st;
    if ((st = precondition(p, precond, m, 1, s))) return st;
    {
        ProfScope pr(p, POBA_K_OTHER, s);
        hipLaunchKernelGGL(k_pcg_beta, dim3(unsigned(np)), blk, 0, s, b, np, 0, tol, coeffs, b.ctrl);
        hipLaunchKernelGGL(k_pcg_dir, g_cam, blk, 0, s, b, z, b.ctrl);
    }
    for (int32_t it = 1; it <= max_iters; ++it) {
        if ((st = launch_schur_part64(p, b.cg + 3 * 9 * int64_t(z.nc), s))) return st;
        {
            ProfScope pr(p, POBA_K_OTHER, s);
            hipLaunchKernelGGL(k_pcg_q, g_cam, blk, 0, s, b, z, b.ctrl);
            hipLaunchKernelGGL(k_pcg_alpha, dim3(unsigned(np)), blk, 0, s, b, np, it, coeffs, b.ctrl);
        }
        if ((st = precondition(p, precond, m, 0, s))) return st;
        {
            ProfScope pr(p, POBA_K_OTHER, s);
            hipLaunchKernelGGL(k_pcg_beta, dim3(unsigned(np)), blk, 0, s, b, np, it, tol, coeffs, b.ctrl);
            hipLaunchKernelGGL(k_pcg_dir, g_cam, blk, 0, s, b, z, b.ctrl);
        }
        if (it % kCheckEvery == 0 && it < max_iters) {
            int32_t left = 0;
            if (hipMemcpyAsync(&left, &b.ctrl->active, sizeof(left), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                return POBA_ERR_HIP;
            if (left == 0) break;
        }
    }
    {
        ProfScope pr(p, POBA_K_OTHER, s);
        hipLaunchKernelGGL(k_pcg_x_out, dim3(unsigned(ceil_div(int64_t(z.nc) * 9, kBlock))), blk, 0, s, b, z);
        hipLaunchKernelGGL(k_pcg_end, dim3(1), dim3(kReduceBlock), 0, s, b, np, info, b.ctrl);
    }
    if (hipGetLastError() != hipSuccess) return POBA_ERR_HIP;
    return launch_backsub_from_x(p, dx_cams, dx_lms, s);
}

}  // extern "C"
