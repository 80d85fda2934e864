/*
 * poba.h - C ABI of the MI355X (gfx950) power-series bundle-adjustment library.
 *
 * The library computes one Levenberg-Marquardt (LM) iteration of bundle
 * adjustment the way Power Bundle Adjustment does (Weber, Demmel, Chan,
 * Cremers, arXiv 2204.12834): residuals and Jacobian blocks of every
 * observation, the block-diagonal damped normal-equation blocks, the Schur
 * complement system for the cameras solved by the power series of the inverse
 * Schur complement, back-substitution for the landmarks, and the accept/reject
 * decision with the damping update.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Cameras are float64 [n_cams][9]: angle-axis rotation (3), translation (3),
 *    focal length, radial k1, radial k2 (the BAL camera layout; the camera
 *    looks down its -z axis; a point projects to f (1 + k1 |p|^2 + k2 |p|^4) p
 *    with p = -P_xy / P_z, P = R(omega) X + t).  Landmarks are float64
 *    [n_lms][3].  Observations are float64 [n_obs][2] pixel positions with
 *    int32 camera and landmark indices.  The residual is model minus
 *    observation; the cost is F = 1/2 sum_i rho(|r_i|^2) (Sec. 4 of the
 *    paper; rho is the identity for the squared loss).
 *  - Pointers documented [dev] are device pointers on the current HIP device;
 *    [host] pointers are host memory.  The caller owns every buffer.  The
 *    library never allocates device memory: all scratch lives in a caller
 *    workspace whose size poba_workspace_bytes returns.
 *  - Every call is asynchronous on the given stream (a hipStream_t passed as
 *    void*; NULL is the default stream) unless stated otherwise.  Errors that
 *    the host can detect are returned at once.  Errors that only the device
 *    can see are OR-ed into a device status word (poba_solve_info.status,
 *    poba_lm_state.status) so that calls stay free of host synchronisation.
 *  - A handle may be used by one stream at a time; distinct handles are
 *    independent.  Results are bitwise reproducible for the same inputs,
 *    device and launch configuration: no floating-point atomics are used.
 */
#ifndef POBA_H
#define POBA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t poba_status;

enum {
    POBA_OK = 0,
    POBA_ERR_INVALID_ARG = 1,  /* null pointer, negative size, bad enum value   */
    POBA_ERR_INDEX_RANGE = 2,  /* an observation index is outside its range      */
    POBA_ERR_NOT_SPD = 4,      /* a damped block had a non-positive pivot (bit)  */
    POBA_ERR_NONFINITE = 8,    /* a residual or cost was not finite (bit)        */
    POBA_ERR_HIP = 16,         /* a HIP runtime call or kernel launch failed     */
    POBA_ERR_WORKSPACE = 32,   /* workspace missing, misaligned or too small     */
    POBA_ERR_STATE = 64        /* call not valid in the handle's current state   */
};

/* Storage precision of the per-observation Jacobian blocks and of the
 * landmark-side vectors of the series (Sec. 5 implements single- and
 * double-precision solvers).  Camera-side vectors, U^-1, accumulations, the
 * cost and the LM decision are float64 in every mode. */
enum { POBA_F64 = 0, POBA_F32 = 1, POBA_F32_BF16J = 2 };

/* What the passes read per observation (both orders).  JACOBIAN: the 24
 * scalars of J_p (2x9) and J_l (2x3) in the storage precision.  POINT: the
 * camera-frame point P = R X + t and the square root of the IRLS weight
 * (4 scalars, float32 or float64); every pass rebuilds the blocks from them
 * and the camera's parameters (Sec. 4: J depends on the observation only
 * through P), moving about a sixth of the bytes.  POINT is available with
 * POBA_F64 and POBA_F32. */
enum { POBA_RECORDS_JACOBIAN = 0, POBA_RECORDS_POINT = 1 };

/* D^T D of Sec. 4.1: Marquardt = diag(J^T J) clamped to [1e-6, 1e32]; identity = I. */
enum { POBA_DAMP_MARQUARDT = 0, POBA_DAMP_IDENTITY = 1 };

/* Loss on |r_i|^2: squared (Sec. 4) or Huber with IRLS reweighting. */
enum { POBA_LOSS_L2 = 0, POBA_LOSS_HUBER = 1 };

typedef void *poba_stream; /* hipStream_t */
typedef struct poba_problem_s *poba_problem;

/* [host] Problem description. */
typedef struct {
    int32_t n_cams;     /* >= 1 */
    int32_t n_lms;      /* >= 1 */
    int64_t n_obs;      /* >= 0, < 2^31 */
    int32_t precision;  /* POBA_F64 / POBA_F32 / POBA_F32_BF16J */
    int32_t damping;    /* POBA_DAMP_* */
    int32_t loss;       /* POBA_LOSS_* */
    int32_t piece_size; /* observations per camera-pass work item; 0 = default (1024) */
    int32_t lm_ranges;  /* landmark ranges of the camera-major order (XCD-local gathers,
                           and with point records the slices staged in LDS by the
                           camera pass); 0 = automatic, 1 = none, else a multiple of 8 */
    int32_t records;    /* POBA_RECORDS_*: what is stored per observation      */
    double huber_delta; /* pixels; used when loss == POBA_LOSS_HUBER, must be > 0 */
} poba_desc;

/* [dev] Written by poba_power_solve, one per problem of the handle. */
typedef struct {
    int32_t stop_order; /* highest power of P in the result (Sec. 4.3, x(m))  */
    int32_t stopped;    /* 1 if the stop rule (eq. qcriterion) ended the series early */
    int32_t status;     /* OR of POBA_ERR_* bits seen on the device            */
    int32_t reserved;
    double norm_x;      /* |x(stop_order)|_2 over all camera parameters        */
    double norm_v;      /* |x(stop_order) - x(stop_order - 1)|_2               */
} poba_solve_info;

/* [dev] LM state carried between poba_lm_step calls, one per problem of the
 * handle; set up by poba_lm_init. */
typedef struct {
    double lambda;         /* damping for the next step                          */
    double nu;             /* growth factor applied on the next rejection        */
    double cost;           /* F at the current state                             */
    double cost_new;       /* F at state + step of the last iteration            */
    double model_decrease; /* L(0) - L(dx) of the last iteration                 */
    double gain;           /* (F - F_new) / (L(0) - L(dx)) of the last iteration */
    int32_t iteration;     /* LM iterations taken (accepted or not)              */
    int32_t accepted;      /* last step accepted                                 */
    int32_t done;          /* 1 once converged or out of iterations              */
    int32_t need_linearize;/* 1 if the next step must re-evaluate J and r        */
    int32_t stop_order;    /* series order used by the last step                 */
    int32_t status;        /* OR of POBA_ERR_* bits seen on the device           */
    int32_t n_accepted;    /* accepted steps so far                              */
    int32_t converged;     /* 1 if the relative function tolerance was met       */
} poba_lm_state;

/* [host] LM settings; poba_lm_default_options fills the values of Sec. 5.1. */
typedef struct {
    double lambda0;    /* initial damping (1e-4)                               */
    double func_tol;   /* stop when (F_old - F_new) / F_old < func_tol (1e-6)  */
    double eps;        /* series stop threshold of eq. qcriterion (0.01); 0 = fixed order */
    double eta;        /* accept iff gain ratio > eta (1e-3)                   */
    double lambda_min; /* damping clamp (1e-16)                                */
    double lambda_max; /* damping clamp (1e16)                                 */
    int32_t m;         /* maximal series order, number of P applications (20)  */
    int32_t max_iters; /* maximal LM iterations (50)                           */
} poba_lm_options;

/* Library version (major * 10000 + minor * 100 + patch). */
int32_t poba_version(void);

/* Human-readable name of a status value (or of its lowest set bit). */
const char *poba_status_string(poba_status s);

/* Fills *o with the LM settings of Sec. 5.1. */
void poba_lm_default_options(poba_lm_options *o);

/* Bytes of device workspace a problem needs (pure host computation; 0 if the
 * description is invalid).  The workspace holds the observation orders, the
 * Jacobian blocks in both orders, all per-camera and per-landmark blocks and
 * vectors, and the scratch of every call.  Rough size per observation:
 * 2 x 24 Jacobian scalars + 60 bytes; per landmark about 200 bytes. */
size_t poba_workspace_bytes(const poba_desc *d);

/* Builds a problem: validates the indices, sorts the observations into a
 * landmark-major order (stable by landmark) and a camera-major order (stable
 * by camera, then by landmark range: the observed landmarks are cut into
 * lm_ranges contiguous ranges so that each of the GPU's eight dies gathers
 * from a slice that fits its L2), and lays out the work tiles of both passes.  obs_cam, obs_lm [dev] int32
 * [n_obs]; obs_xy [dev] float64 [n_obs][2]; workspace [dev], 256-byte
 * aligned, at least poba_workspace_bytes(d) bytes, owned by the caller and
 * used by the handle until poba_destroy.  The inputs are copied and may be
 * freed after the call returns.  Synchronises the stream (set-up only).
 * Returns POBA_ERR_INDEX_RANGE if an index is out of range. */
poba_status poba_create(const poba_desc *d, const int32_t *obs_cam, const int32_t *obs_lm,
                        const double *obs_xy, void *workspace, size_t workspace_bytes,
                        poba_stream stream, poba_problem *out);

/* Batched problems: n_problems independent bundle-adjustment problems held in
 * one handle and solved together, every call covering all of them.  Problem j
 * owns the cameras [prob_cam_off[j], prob_cam_off[j+1]) and the landmarks
 * [prob_lm_off[j], prob_lm_off[j+1]) of the concatenated state (both [host]
 * int32 [n_problems + 1], starting at 0, strictly increasing, ending at
 * n_cams / n_lms); each observation must pair a camera and a landmark of the
 * same problem (else POBA_ERR_INDEX_RANGE).  Each problem keeps its own
 * damping, series stop rule and LM decision: poba_power_solve fills
 * info[n_problems], poba_linearize cost[n_problems], and poba_lm_init /
 * poba_lm_step take st[n_problems].  The kernels of every call cover all
 * problems in one launch each (a landmark segment or camera piece never
 * mixes two problems, so each problem's results match a handle of its own
 * up to the floating-point summation order).  poba_create is the case
 * n_problems = 1. */
size_t poba_batch_workspace_bytes(const poba_desc *d, int32_t n_problems);
poba_status poba_batch_create(const poba_desc *d, int32_t n_problems, const int32_t *prob_cam_off,
                              const int32_t *prob_lm_off, const int32_t *obs_cam,
                              const int32_t *obs_lm, const double *obs_xy, void *workspace,
                              size_t workspace_bytes, poba_stream stream, poba_problem *out);

/* Releases the host-side handle (the workspace stays the caller's). */
poba_status poba_destroy(poba_problem p);

/* Bytes of the library-held workspace of poba_create_static, per GPU. */
#define POBA_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): poba_create
 * with the workspace taken from a device array of POBA_STATIC_WORKSPACE_BYTES
 * that the library holds on every GPU it runs on until the process ends.  It
 * calls no hipMalloc, hipFree or allocating library routine; the scratch of
 * its radix sorts and scans is sized exactly for the problem.  Arguments,
 * results and errors as poba_create (one problem), except: a problem whose
 * workspace would exceed the array returns POBA_ERR_WORKSPACE before any
 * device work (in float32 storage about 150,000 observations fit, in float64
 * about 100,000).  Every handle made by this call on one GPU uses that GPU's
 * one array: a new call makes the handle of the previous call on the same
 * GPU invalid (poba_destroy still releases it), and calls on two such handles
 * that overlap in time race.  The array keeps the contents of the last
 * handle; creation clears the part it lays out before use. */
poba_status poba_create_static(const poba_desc *d, const int32_t *obs_cam, const int32_t *obs_lm,
                               const double *obs_xy, poba_stream stream, poba_problem *out);

/* Sec. 4 and 4.1: evaluates residuals r_i and Jacobian blocks J_p (2x9),
 * J_l (2x3) at cams [dev] float64 [n_cams][9], lms [dev] float64 [n_lms][3];
 * applies the Huber reweighting if configured; stores the blocks (rounded to
 * the storage precision) in both observation orders; accumulates the
 * undamped blocks U = J_p^T J_p, V = J_l^T J_l and b_p = J_p^T r,
 * b_l = J_l^T r in float64 from the rounded blocks; writes F of every problem
 * to cost [dev] (float64 [n_problems]; may be NULL). */
poba_status poba_linearize(poba_problem p, const double *cams, const double *lms, double *cost,
                           poba_stream stream);

/* Sec. 4.2-4.3: with the blocks of the last poba_linearize, forms
 * U_lambda = U + lambda D_p^T D_p and V_lambda likewise (eq. normal), inverts
 * every block in float64, forms b~ = b_p - W V^-1 b_l (eq. Schur), sums the
 * power series x(m) = -sum_{i=0..m} (U^-1 W V^-1 W^T)^i U^-1 b~ (eqs.
 * S_approx, x_approx) matrix-free, stopping early when
 * (i+1) |x(i) - x(i-1)| / |x(i)| < eps (eq. qcriterion; eps = 0 gives the
 * fixed order m), and back-substitutes dx_l = -V^-1 (b_l + W^T dx_p) (the
 * sign that solves eq. normal; the paper prints -b_l).
 * dx_cams [dev] float64 [n_cams][9], dx_lms [dev] float64 [n_lms][3],
 * info [dev] [n_problems] (may be NULL).  Every problem of a batch is
 * solved with the same lambda and stops by its own rule.  lambda > 0,
 * 0 <= m <= 100000, eps >= 0. */
poba_status poba_power_solve(poba_problem p, double lambda, int32_t m, double eps, double *dx_cams,
                             double *dx_lms, poba_solve_info *info, poba_stream stream);

/* ---- preconditioned conjugate gradients (the comparison of Sec. 2) ----- */

/* Preconditioners M^-1 of poba_pcg_solve (Sec. 2, Fig. 2). */
enum {
    POBA_PRECOND_NONE = 0,          /* the identity                                    */
    POBA_PRECOND_SCHUR_JACOBI = 1,  /* inverted 9x9 diagonal blocks of S               */
    POBA_PRECOND_POWER = 2          /* S~(m) = sum_{i<=m} P^i U^-1 (eq. S_approx)      */
};

/* [dev] Written by poba_pcg_solve, one per problem of the handle. */
typedef struct {
    int32_t iterations;   /* CG iterations taken                                    */
    int32_t converged;    /* 1 if |r| <= tol |b~| was reached                       */
    int32_t status;       /* OR of POBA_ERR_* bits seen on the device               */
    int32_t reserved;
    double rel_residual;  /* |r| / |b~| of the recursion at the last iterate        */
    double rz;            /* r . M^-1 r at the last iterate                         */
} poba_pcg_info;

/* The damped step of poba_power_solve with the camera step from conjugate
 * gradients (Hestenes-Stiefel, x_0 = 0) on the reduced camera system
 * S dx_p = -b~ (eqs. Schur, Sx), S = U_lambda - W V_lambda^-1 W^T applied
 * matrix-free in float64 (stored blocks widened, V^-1 recomputed in float64),
 * preconditioned by `precond` (POBA_PRECOND_*; the power series runs order
 * m in the storage precision, as poba_power_solve does, costing m
 * applications of P per iteration).  Each problem iterates until
 * |r_k| <= tol |b~| or max_iters; then dx_l = -V^-1 (b_l + W^T dx_p).
 * dx_cams [dev] float64 [n_cams][9], dx_lms [dev] float64 [n_lms][3],
 * info [dev] [n_problems] (may be NULL), coeffs [dev] float64
 * [max_iters][n_problems][2] (may be NULL): alpha_k and beta_k of iteration
 * k + 1 per problem (the Lanczos coefficients behind a condition-number
 * estimate of M^-1 S; entries of iterations not taken, and the beta of the
 * last one, are left as they were).  lambda > 0, tol >= 0,
 * 0 <= max_iters <= 1000000, 0 <= m <= 100000 for the power series.
 * Synchronises the stream every four iterations to end the loop once every
 * problem has converged; not for graph capture.  A non-positive p.q or r.z
 * ends that problem's iteration with POBA_ERR_NOT_SPD in its status. */
poba_status poba_pcg_solve(poba_problem p, double lambda, int32_t precond, int32_t m, double tol,
                           int32_t max_iters, double *dx_cams, double *dx_lms, poba_pcg_info *info,
                           double *coeffs, poba_stream stream);

/* Resets the LM states st [dev] [n_problems]: lambda = lambda0, nu = 2,
 * iteration 0, needs a linearisation, not done. */
poba_status poba_lm_init(poba_problem p, poba_lm_state *st, const poba_lm_options *o,
                         poba_stream stream);

/* One LM iteration (Sec. 5.1 "LM loop") of every problem that is not done,
 * on the state cams, lms [dev] (a problem's part updated in place when its
 * step is accepted) and st [dev] [n_problems]: linearises if a last step was
 * accepted (or on the first call), solves with st[j].lambda as
 * poba_power_solve does (order o->m, threshold o->eps), evaluates F at the
 * trial state and the undamped linear-model decrease L(0) - L(dx), accepts
 * iff F_new is finite, L(0) - L(dx) > 0 and the gain ratio exceeds o->eta,
 * and updates lambda (success: lambda *= max(1/3, 1 - (2 rho - 1)^3), nu = 2;
 * failure: lambda *= nu, nu *= 2).  Once st[j].done is set, further calls
 * leave problem j alone.  No host synchronisation and no memory set or copy:
 * the call can be captured in a graph (poba_lm_graph_create). */
poba_status poba_lm_step(poba_problem p, double *cams, double *lms, poba_lm_state *st,
                         const poba_lm_options *o, poba_stream stream);

/* ---- LM with a step computed elsewhere --------------------------------- */

/* The two halves of poba_lm_step around its solve, for a caller that computes
 * the step itself (e.g. by the clustered solve of Sec. 5.3):
 * poba_lm_begin sets up the problems that are not done and linearises where
 * st[j].need_linearize is set (writing st[j].cost); poba_lm_finish takes the
 * step dx_cams [dev] float64 [n_cams][9], dx_lms [dev] float64 [n_lms][3] and
 * evaluates, accepts or rejects it and updates lambda exactly as
 * poba_lm_step does (o->m and o->eps are not used).  Between the two calls
 * the handle may be used for other calls at st[j].lambda. */
poba_status poba_lm_begin(poba_problem p, double *cams, double *lms, poba_lm_state *st, poba_stream stream);
poba_status poba_lm_finish(poba_problem p, double *cams, double *lms, poba_lm_state *st,
                           const poba_lm_options *o, const double *dx_cams, const double *dx_lms,
                           poba_stream stream);

/* Sec. 4.2, eq. (back_substitution) for a given camera step: with the blocks
 * of the last poba_linearize and damping lambda > 0, dx_lms [dev] float64
 * [n_lms][3] = -V_lambda^-1 (b_l + W^T dx_cams), dx_cams [dev] float64
 * [n_cams][9].  (Every problem of a batch uses the same lambda.) */
poba_status poba_back_substitute(poba_problem p, double lambda, const double *dx_cams, double *dx_lms,
                                 poba_stream stream);

/* ---- camera clusters (Sec. 5.3, PoST) --------------------------------- */

/* [host] The camera graph of a problem: an edge between two cameras that
 * observe a common landmark, weighted by the number of such landmarks (each
 * landmark counted once per camera pair).  obs_cam, obs_lm [host] int32
 * [n_obs].  Returns POBA_ERR_INDEX_RANGE for an index out of range.  The
 * host calls on a graph return POBA_ERR_WORKSPACE when host memory runs out. */
typedef struct poba_camera_graph_s *poba_camera_graph;
poba_status poba_camera_graph_create(int64_t n_obs, const int32_t *obs_cam, const int32_t *obs_lm,
                                     int32_t n_cams, int32_t n_lms, poba_camera_graph *out);
poba_status poba_camera_graph_destroy(poba_camera_graph g);

/* [host] The edges (a < b, ordered by (a, b)) and weights; with a, b, w NULL
 * only their number. */
poba_status poba_camera_graph_edges(poba_camera_graph g, int64_t *n_edges, int32_t *a, int32_t *b, int32_t *w);

/* [host] Greedy clustering of the cameras: edges are visited by decreasing
 * key (ties: the edge order), where the key is the weight, or for seed >= 0
 * the weight times a uniform number in [0, 1) drawn per edge by the SplitMix64
 * finaliser of seed ^ (a << 32 | b) (top 53 bits); the two clusters of an edge
 * merge when the result has at most max_size cameras.  cluster [host] int32
 * [n_cams] receives cluster indices numbered in the order of each cluster's
 * smallest camera, *n_clusters their number (may be NULL). */
poba_status poba_camera_graph_cluster(poba_camera_graph g, int32_t max_size, int64_t seed, int32_t *cluster,
                                      int32_t *n_clusters);

/* [host] The graph's observation order: order [n_obs] lists the original
 * observation indices by landmark (stable within a landmark). */
poba_status poba_camera_graph_order(poba_camera_graph g, int32_t *order);

/* [host] The batched layout of the graph's problem clustered by `cluster`
 * (Sec. 5.3): problem k is cluster k.  cam_pos [n_cams]: the camera's index
 * in cluster order (clusters in turn, cameras ascending); the landmarks are
 * the (cluster, landmark) pairs that have observations, numbered by cluster
 * then landmark, plus one unobserved pair (landmark 0) for a cluster without
 * observations: obs_vlm [n_obs] the pair of each observation taken in the
 * graph's observation order (poba_camera_graph_order), vlm_src
 * [n_obs + n_clusters] the landmark of each pair, *n_vlm their number;
 * prob_cam_off, prob_lm_off [n_clusters + 1] the ranges for
 * poba_batch_create.  All host memory; cluster values must lie in
 * [0, n_clusters) (else POBA_ERR_INDEX_RANGE) and use every index (else
 * POBA_ERR_INVALID_ARG). */
poba_status poba_camera_graph_layout(poba_camera_graph g, const int32_t *cluster, int32_t n_clusters,
                                     int32_t *cam_pos, int32_t *obs_vlm, int32_t *vlm_src, int32_t *n_vlm,
                                     int32_t *prob_cam_off, int32_t *prob_lm_off);

/* Replaces the undamped landmark blocks of the last poba_linearize: V [dev]
 * float64 [n_lms][3][3] (the upper triangle is read) and b_l [dev] float64
 * [n_lms][3].  With the V and b_l of a whole problem gathered onto the
 * (cluster, landmark) pairs of its clustered layout, the clustered handle's
 * reduced system is the block diagonal of the whole one over the clusters
 * (Sec. 5.3).  Valid until the next poba_linearize. */
poba_status poba_set_landmark_blocks(poba_problem p, const double *V, const double *bl, poba_stream stream);

/* ---- differentiation of the damped step (an extension) ------------------ */

/* Replaces the observed pixel positions of the handle: obs_xy [dev] float64
 * [n_obs][2] in the original observation order (as given to poba_create).
 * Takes effect at the next poba_linearize. */
poba_status poba_set_observations(poba_problem p, const double *obs_xy, poba_stream stream);

/* frozen = 1: later solves reuse the damping diagonal D (Sec. 4.1 D^T D) of
 * the last solve made with frozen = 0 instead of taking it from the current
 * blocks, so D is a constant of the step (the setting in which
 * poba_step_adjoint differentiates it).  frozen = 0 (default) restores the
 * normal behaviour.  D is zero until a first unfrozen solve has run. */
poba_status poba_set_damping_frozen(poba_problem p, int32_t frozen);

/* Adjoint of the damped step dx = -H^-1 g of eq. normal (Sec. 4.1) at fixed
 * lambda and fixed D, H = J^T J + lambda D, g = J^T r, r = pi - o, by implicit
 * differentiation.  The handle must hold the linearisation at cams, lms [dev]
 * (poba_linearize at that state, squared loss only), and dx_cams, dx_lms
 * [dev] must be the step that poba_power_solve(lambda, m, eps = 0) returned
 * there.  For the upstream gradient grad_dx_cams [dev] [n_cams][9],
 * grad_dx_lms [dev] [n_lms][3]:
 *   z = H~^-1 gbar, the same power solve of order m run on gbar (the
 *       truncated inverse H~ of eqs. S_approx, x_approx is symmetric), into
 *       z_cams [n_cams][9], z_lms [n_lms][3] [dev];
 *   grad_obs [dev] [n_obs][2], original observation order: J_i z_i, the
 *       exact gradient of <gbar, dx> with respect to o_i for the step as
 *       computed (dx is linear in o);
 *   grad_intrinsics [dev] [n_cams][3] (f, k1, k2): -z^T d(H dx + g)/d theta
 *       at fixed dx, from the mixed second derivatives of the projection.
 * All float64.  Overwrites the series work buffers (the state used by
 * poba_lm_step is not kept across this call: call poba_lm_init again before
 * further LM iterations).  info [dev] may be NULL.  Returns
 * POBA_ERR_INVALID_ARG for the Huber loss (its weights depend on o). */
poba_status poba_step_adjoint(poba_problem p, double lambda, int32_t m, const double *cams,
                              const double *lms, const double *dx_cams, const double *dx_lms,
                              const double *grad_dx_cams, const double *grad_dx_lms, double *z_cams,
                              double *z_lms, double *grad_obs, double *grad_intrinsics,
                              poba_solve_info *info, poba_stream stream);

/* A HIP graph of n_steps consecutive poba_lm_step calls with these
 * arguments (device pointers, options copied), captured on a private
 * stream; one poba_lm_graph_launch then runs the n_steps iterations of every
 * problem with a single launch on the caller's stream.  Steps after a
 * problem is done leave it untouched, so a graph of max_iters steps runs an
 * LM solve to its end.  Event timing (poba_profile_enable) is not recorded
 * inside the graph.  1 <= n_steps <= 1000. */
typedef struct poba_lm_graph_s *poba_lm_graph;
poba_status poba_lm_graph_create(poba_problem p, double *cams, double *lms, poba_lm_state *st,
                                 const poba_lm_options *o, int32_t n_steps, poba_lm_graph *out);
poba_status poba_lm_graph_launch(poba_lm_graph g, poba_stream stream);
poba_status poba_lm_graph_destroy(poba_lm_graph g);

/* Model pixel positions out_xy [dev] float64 [n_obs][2] of observations
 * (obs_cam, obs_lm [dev] int32 [n_obs]) at cams, lms [dev].  Needs no handle;
 * indices must be in range (they are not checked). */
poba_status poba_project(int64_t n_obs, const int32_t *obs_cam, const int32_t *obs_lm,
                         const double *cams, const double *lms, double *out_xy,
                         poba_stream stream);

/* Residual check of the reduced camera system (Sec. 4.2, eq. Schur) for a
 * camera step dx_cams [dev] float64 [n_cams][9] of the last poba_power_solve
 * (its lambda, damping diagonal and b~): rel_residual[j] = |S x + b~|_2 /
 * |b~|_2 per problem [dev] float64 [n_problems], with S x = U_lambda x -
 * W V_lambda^-1 W^T x evaluated in float64 (V^-1 recomputed in float64, the
 * stored Jacobian blocks widened, norms summed with TwoSum compensation).
 * For the series x(m) it equals |U P^{m+1} U^-1 b~| / |b~|. */
poba_status poba_solve_residual(poba_problem p, const double *dx_cams, double *rel_residual,
                                poba_stream stream);

/* ---- inspection (tests, diagnostics) ---------------------------------- */

/* Copies the undamped blocks of the last linearisation: U [dev] float64
 * [n_cams][9][9], V [dev] float64 [n_lms][3][3], b_p [n_cams][9],
 * b_l [n_lms][3].  Any pointer may be NULL. */
poba_status poba_get_blocks(poba_problem p, double *U, double *V, double *bp, double *bl,
                            poba_stream stream);

/* Copies the stored Jacobian blocks of one order (0 = landmark-major,
 * 1 = camera-major), widened to float64 and put back in original
 * observation order: Jp [dev] [n_obs][2][9], Jl [dev] [n_obs][2][3].
 * r [dev] [n_obs][2] receives the (reweighted) residual; it may be NULL. */
poba_status poba_get_jacobians(poba_problem p, int32_t order, double *Jp, double *Jl, double *r,
                               poba_stream stream);

/* The observation orders: perm_lm, perm_cam [dev] int32 [n_obs] (original
 * index of each position), lm_off [dev] int32 [n_lms + 1], cam_off [dev]
 * int32 [n_cams + 1].  Any pointer may be NULL. */
poba_status poba_get_orders(poba_problem p, int32_t *perm_lm, int32_t *perm_cam, int32_t *lm_off,
                            int32_t *cam_off, poba_stream stream);

/* One application of P = U^-1 W V^-1 W^T (Sec. 4.3) with the damped
 * inverses of the last poba_power_solve: v_out = P v_in, both [dev] float64
 * [n_cams][9]. */
poba_status poba_apply_P(poba_problem p, const double *v_in, double *v_out, poba_stream stream);

/* ---- launch tuning ------------------------------------------------------ */

enum {
    POBA_TUNE_TILES_PER_WAVE = 0, /* 64-observation landmark tiles per wavefront in the
                                     landmark pass that gathers the camera vector
                                     from global memory (1..64, default 4); the LDS
                                     variants split the tiles evenly instead     */
    POBA_TUNE_LM_RANGES = 1,      /* landmark ranges chosen at creation (read only) */
    POBA_TUNE_LDS_CAMERA = 2,     /* 1: landmark pass reads the camera vector from LDS when
                                     it fits in 64 KB (default); 0: from global memory */
    POBA_TUNE_RANGE_LDS = 3       /* point records: 1 (default where possible): the series
                                     camera pass stages each landmark range's slice of the
                                     landmark vector in LDS; possible when the handle was
                                     created with ranges of at most 80 KB of that vector
                                     (automatic ranges are); 0: gathers from L2 per piece */
};

/* Sets a launch parameter of the handle's kernels (results do not depend on
 * it beyond floating-point summation order).  Returns POBA_ERR_INVALID_ARG for
 * an unknown key or a value out of range. */
poba_status poba_set_tuning(poba_problem p, int32_t key, int32_t value);

/* Reads a launch parameter into *value [host]. */
poba_status poba_get_tuning(poba_problem p, int32_t key, int32_t *value);

/* ---- timing (benchmarks) ---------------------------------------------- */

/* Kernel classes timed with events when profiling is on. */
enum {
    POBA_K_LINEARIZE = 0, /* both linearisation passes                   */
    POBA_K_INVERSE = 1,   /* damped block inversions                      */
    POBA_K_LM_PASS = 2,   /* landmark pass of a series order: t_l = W^T v,
                             s_l = V^-1 t_l                               */
    POBA_K_CAM_PASS = 3,  /* camera pass of a series order: partial W s   */
    POBA_K_CAM_FIN = 4,   /* camera finish of a series order: U^-1,
                             series sum, norms, stop rule                 */
    POBA_K_BACKSUB = 5,   /* back-substitution                            */
    POBA_K_EVAL = 6,      /* trial cost and model decrease                */
    POBA_K_OTHER = 7,     /* the rest, among it the reduced right-hand
                             side b~ (its camera pass and finish)         */
    POBA_K_COUNT = 8
};

/* Turns per-launch event timing on (1) or off (0).  While on, every launch
 * is bracketed by hipEventRecord on its stream; timings accumulate until
 * read.  At most 65536 timed launches between reads. */
poba_status poba_profile_enable(poba_problem p, int32_t enable);

/* Synchronises on the recorded events and returns, per kernel class, the
 * summed milliseconds ms[POBA_K_COUNT] and launch counts n[POBA_K_COUNT]
 * [host] since the last read; then clears them. */
poba_status poba_profile_read(poba_problem p, double *ms, int64_t *n);

/* ---- bandwidth probe ---------------------------------------------------- */

/* Streams `bytes` (a multiple of 16; src 16-byte aligned) from src [dev].
 * kind 0 only reads (dst [dev]: `blocks` floats of sink, written only for a
 * value that ordinary data never sums to); kind 1 copies src to dst [dev];
 * kind 2 only writes `bytes` of zeros to dst [dev] (src is not read).
 * blocks <= 0 selects 4096 blocks.  Used to measure the achievable HBM
 * bandwidth and to calibrate byte counters with a transfer of known size. */
poba_status poba_probe(int32_t kind, const void *src, void *dst, size_t bytes, int32_t blocks,
                       poba_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* POBA_H */
