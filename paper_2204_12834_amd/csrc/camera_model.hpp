// Residual and Jacobian blocks of one observation (float64).
//
// Camera (BAL layout): omega (angle-axis), t, f, k1, k2.  With
// theta^2 = omega.omega, A = sin(theta)/theta, B = (1 - cos(theta))/theta^2:
//
//   R X = X + A (omega x X) + B (omega x (omega x X))          (Rodrigues)
//   P   = R X + t,   p = -P_xy / P_z,   d = 1 + k1 |p|^2 + k2 |p|^4
//   pi  = f d p,     r = pi - o
//
// d(R X)/d omega_j follows from the product rule on the three terms, with
// dA/domega_j = C omega_j and dB/domega_j = D omega_j where
// C = A'(theta)/theta = (theta cos(theta) - sin(theta)) / theta^3 and
// D = B'(theta)/theta = (theta sin(theta) - 2 (1 - cos(theta))) / theta^4;
// A, B, C, D switch to their Taylor series below theta^2 = 1e-3.
//
// Floating-point contraction is off inside these functions so that the
// landmark-major and camera-major passes, which both call them, produce
// bit-identical blocks wherever the compiler inlines them.
#pragma once

#include <hip/hip_runtime.h>

namespace poba {

struct ObsEval {
    double r[2];
    double J[24];  // J_p row 0 (9), J_p row 1 (9), J_l row 0 (3), J_l row 1 (3)
};

__device__ __forceinline__ void rodrigues_coeffs(double th2, double& A, double& B, double& C, double& D) {
#pragma clang fp contract(off)
    if (th2 < 1e-3) {
        const double t4 = th2 * th2, t6 = t4 * th2;
        A = 1.0 - th2 / 6.0 + t4 / 120.0 - t6 / 5040.0;
        B = 0.5 - th2 / 24.0 + t4 / 720.0 - t6 / 40320.0;
        C = -1.0 / 3.0 + th2 / 30.0 - t4 / 840.0 + t6 / 45360.0;
        D = -1.0 / 12.0 + th2 / 180.0 - t4 / 6720.0 + t6 / 453600.0;
    } else {
        const double th = sqrt(th2);
        double s, c;
        sincos(th, &s, &c);
        const double omc = 2.0 * sin(0.5 * th) * sin(0.5 * th);
        A = s / th;
        B = omc / th2;
        C = (th * c - s) / (th2 * th);
        D = (th * s - 2.0 * omc) / (th2 * th2);
    }
}

__device__ __forceinline__ void cross3(const double* a, const double* b, double* o) {
#pragma clang fp contract(off)
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

// dRX[k][j] = d(R X)_k / d omega_j
//   = C w_j (w x X)_k + A (e_j x X)_k + D w_j (w x (w x X))_k
//     + B ( (e_j x (w x X))_k + (w x (e_j x X))_k )
__device__ __forceinline__ void rotation_derivative(const double* w, const double* X, const double* wx,
                                                    const double* wwx, double A, double B, double C, double D,
                                                    double (*dRX)[3]) {
#pragma clang fp contract(off)
    for (int j = 0; j < 3; ++j) {
        double ej[3] = {0.0, 0.0, 0.0};
        ej[j] = 1.0;
        double ejX[3], ejwx[3], wejX[3];
        cross3(ej, X, ejX);
        cross3(ej, wx, ejwx);
        cross3(w, ejX, wejX);
        for (int k = 0; k < 3; ++k)
            dRX[k][j] = C * w[j] * wx[k] + A * ejX[k] + D * w[j] * wwx[k] + B * (ejwx[k] + wejX[k]);
    }
}

// Camera-frame point of landmark X (no derivatives).
__device__ __forceinline__ void transform_point(const double* cam, const double* X, double* P) {
#pragma clang fp contract(off)
    const double* w = cam;
    const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    double A, B, C, D;
    rodrigues_coeffs(th2, A, B, C, D);
    double wx[3], wwx[3];
    cross3(w, X, wx);
    cross3(w, wx, wwx);
    for (int k = 0; k < 3; ++k) P[k] = X[k] + A * wx[k] + B * wwx[k] + cam[3 + k];
}

__device__ __forceinline__ void project_point(const double* cam, const double* X, double* px) {
#pragma clang fp contract(off)
    double P[3];
    transform_point(cam, X, P);
    const double iz = 1.0 / P[2];
    const double p0 = -P[0] * iz, p1 = -P[1] * iz;
    const double r2 = p0 * p0 + p1 * p1;
    const double d = 1.0 + cam[7] * r2 + cam[8] * r2 * r2;
    px[0] = cam[6] * d * p0;
    px[1] = cam[6] * d * p1;
}

__device__ __forceinline__ void evaluate_obs(const double* cam, const double* X, double ox, double oy, ObsEval& e) {
#pragma clang fp contract(off)
    const double* w = cam;
    const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    double A, B, C, D;
    rodrigues_coeffs(th2, A, B, C, D);
    double wx[3], wwx[3];
    cross3(w, X, wx);
    cross3(w, wx, wwx);
    double P[3];
    for (int k = 0; k < 3; ++k) P[k] = X[k] + A * wx[k] + B * wwx[k] + cam[3 + k];

    // rotation matrix R = I + A [w]x + B [w]x^2, [w]x^2 = w w^T - th2 I
    double R[3][3];
    R[0][0] = 1.0 + B * (w[0] * w[0] - th2);
    R[1][1] = 1.0 + B * (w[1] * w[1] - th2);
    R[2][2] = 1.0 + B * (w[2] * w[2] - th2);
    R[0][1] = -A * w[2] + B * w[0] * w[1];
    R[1][0] = A * w[2] + B * w[0] * w[1];
    R[0][2] = A * w[1] + B * w[0] * w[2];
    R[2][0] = -A * w[1] + B * w[0] * w[2];
    R[1][2] = -A * w[0] + B * w[1] * w[2];
    R[2][1] = A * w[0] + B * w[1] * w[2];

    double dRX[3][3];
    rotation_derivative(w, X, wx, wwx, A, B, C, D, dRX);

    const double iz = 1.0 / P[2];
    const double p[2] = {-P[0] * iz, -P[1] * iz};
    const double r2 = p[0] * p[0] + p[1] * p[1];
    const double f = cam[6], k1 = cam[7], k2 = cam[8];
    const double d = 1.0 + k1 * r2 + k2 * r2 * r2;
    const double dd = 2.0 * (k1 + 2.0 * k2 * r2);  // d(d)/dp = dd * p^T

    e.r[0] = f * d * p[0] - ox;
    e.r[1] = f * d * p[1] - oy;

    // dpi/dp = f (d I + p dd p^T);  dp/dP = [[-iz, 0, P0 iz^2], [0, -iz, P1 iz^2]]
    double dpi_dp[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) dpi_dp[a][b] = f * ((a == b ? d : 0.0) + p[a] * dd * p[b]);
    const double dp_dP[2][3] = {{-iz, 0.0, P[0] * iz * iz}, {0.0, -iz, P[1] * iz * iz}};
    double JP[2][3];
    for (int a = 0; a < 2; ++a)
        for (int c = 0; c < 3; ++c) JP[a][c] = dpi_dp[a][0] * dp_dP[0][c] + dpi_dp[a][1] * dp_dP[1][c];

    for (int a = 0; a < 2; ++a) {
        double* Jp = e.J + 9 * a;
        for (int j = 0; j < 3; ++j) Jp[j] = JP[a][0] * dRX[0][j] + JP[a][1] * dRX[1][j] + JP[a][2] * dRX[2][j];
        for (int j = 0; j < 3; ++j) Jp[3 + j] = JP[a][j];
        Jp[6] = d * p[a];
        Jp[7] = f * r2 * p[a];
        Jp[8] = f * r2 * r2 * p[a];
        double* Jl = e.J + 18 + 3 * a;
        for (int j = 0; j < 3; ++j) Jl[j] = JP[a][0] * R[0][j] + JP[a][1] * R[1][j] + JP[a][2] * R[2][j];
    }
}

// Coefficient of [w]x^2 in the left Jacobian of SO(3),
// E = (1 - sin(theta)/theta) / theta^2 (Taylor series below theta^2 = 1e-3).
__device__ __forceinline__ double left_jacobian_coeff(double th2, double A) {
#pragma clang fp contract(off)
    if (th2 < 1e-3) {
        const double t4 = th2 * th2;
        return 1.0 / 6.0 - th2 / 120.0 + t4 / 5040.0 - t4 * th2 / 362880.0;
    }
    return (1.0 - A) / th2;
}

// Per-camera data shared by all of its observations: the nine parameters,
// the Rodrigues coefficients A, B, C, D, the rotation matrix R and the
// coefficient E of the left Jacobian J_l(w) = I + B [w]x + E [w]x^2.
// Layout: [0..8] parameters, [9..12] A B C D, [13..21] R row-major, [22] E, 1 pad.
constexpr int kCamRec = 24;  // doubles per record

__device__ __forceinline__ void make_cam_record(const double* cam, double* rec) {
#pragma clang fp contract(off)
    const double* w = cam;
    const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    double A, B, C, D;
    rodrigues_coeffs(th2, A, B, C, D);
    for (int k = 0; k < 9; ++k) rec[k] = cam[k];
    rec[9] = A;
    rec[10] = B;
    rec[11] = C;
    rec[12] = D;
    double* R = rec + 13;
    R[0] = 1.0 + B * (w[0] * w[0] - th2);
    R[4] = 1.0 + B * (w[1] * w[1] - th2);
    R[8] = 1.0 + B * (w[2] * w[2] - th2);
    R[1] = -A * w[2] + B * w[0] * w[1];
    R[3] = A * w[2] + B * w[0] * w[1];
    R[2] = A * w[1] + B * w[0] * w[2];
    R[6] = -A * w[1] + B * w[0] * w[2];
    R[5] = -A * w[0] + B * w[1] * w[2];
    R[7] = A * w[0] + B * w[1] * w[2];
    rec[22] = left_jacobian_coeff(th2, A);
    rec[23] = 0.0;
}

// Model pixel of X from a camera record: P = R X + t.
__device__ __forceinline__ void project_rec(const double* rec, const double* X, double* px) {
#pragma clang fp contract(off)
    const double* R = rec + 13;
    double P[3];
    for (int k = 0; k < 3; ++k) P[k] = R[3 * k] * X[0] + R[3 * k + 1] * X[1] + R[3 * k + 2] * X[2] + rec[3 + k];
    const double iz = 1.0 / P[2];
    const double p0 = -P[0] * iz, p1 = -P[1] * iz;
    const double r2 = p0 * p0 + p1 * p1;
    const double d = 1.0 + rec[7] * r2 + rec[8] * r2 * r2;
    px[0] = rec[6] * d * p0;
    px[1] = rec[6] * d * p1;
}

// Residual and Jacobian blocks from a camera record (same formulas as
// evaluate_obs with the per-camera factors hoisted).
__device__ __forceinline__ void evaluate_obs_rec(const double* rec, const double* X, double ox, double oy, ObsEval& e) {
#pragma clang fp contract(off)
    const double* w = rec;
    const double A = rec[9], B = rec[10], C = rec[11], D = rec[12];
    const double* Rm = rec + 13;
    double wx[3], wwx[3];
    cross3(w, X, wx);
    cross3(w, wx, wwx);
    double P[3];
    for (int k = 0; k < 3; ++k) P[k] = Rm[3 * k] * X[0] + Rm[3 * k + 1] * X[1] + Rm[3 * k + 2] * X[2] + rec[3 + k];
    double dRX[3][3];
    rotation_derivative(w, X, wx, wwx, A, B, C, D, dRX);
    const double iz = 1.0 / P[2];
    const double p[2] = {-P[0] * iz, -P[1] * iz};
    const double r2 = p[0] * p[0] + p[1] * p[1];
    const double f = rec[6], k1 = rec[7], k2 = rec[8];
    const double d = 1.0 + k1 * r2 + k2 * r2 * r2;
    const double dd = 2.0 * (k1 + 2.0 * k2 * r2);
    e.r[0] = f * d * p[0] - ox;
    e.r[1] = f * d * p[1] - oy;
    double dpi_dp[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) dpi_dp[a][b] = f * ((a == b ? d : 0.0) + p[a] * dd * p[b]);
    const double dp_dP[2][3] = {{-iz, 0.0, P[0] * iz * iz}, {0.0, -iz, P[1] * iz * iz}};
    double JP[2][3];
    for (int a = 0; a < 2; ++a)
        for (int c = 0; c < 3; ++c) JP[a][c] = dpi_dp[a][0] * dp_dP[0][c] + dpi_dp[a][1] * dp_dP[1][c];
    for (int a = 0; a < 2; ++a) {
        double* Jp = e.J + 9 * a;
        for (int j = 0; j < 3; ++j) Jp[j] = JP[a][0] * dRX[0][j] + JP[a][1] * dRX[1][j] + JP[a][2] * dRX[2][j];
        for (int j = 0; j < 3; ++j) Jp[3 + j] = JP[a][j];
        Jp[6] = d * p[a];
        Jp[7] = f * r2 * p[a];
        Jp[8] = f * r2 * r2 * p[a];
        double* Jl = e.J + 18 + 3 * a;
        for (int j = 0; j < 3; ++j) Jl[j] = JP[a][0] * Rm[j] + JP[a][1] * Rm[3 + j] + JP[a][2] * Rm[6 + j];
    }
}

// Normalised image point of an observation and its derivatives, for the
// second-order terms of the adjoint: p = -P_xy / P_z, n = |p|^2 and
// dp[a][j] = d p_a / d y_j for y = (omega, t, X).  The intrinsics enter only
// through pi = f (1 + k1 n + k2 n^2) p.
struct ObsGeom {
    double p[2];
    double n;
    double dp[2][9];
};

__device__ __forceinline__ void observation_geometry(const double* rec, const double* X, ObsGeom& g) {
    const double* w = rec;
    const double A = rec[9], B = rec[10], C = rec[11], D = rec[12];
    const double* Rm = rec + 13;
    double wx[3], wwx[3];
    cross3(w, X, wx);
    cross3(w, wx, wwx);
    double P[3];
    for (int k = 0; k < 3; ++k) P[k] = Rm[3 * k] * X[0] + Rm[3 * k + 1] * X[1] + Rm[3 * k + 2] * X[2] + rec[3 + k];
    double dRX[3][3];
    rotation_derivative(w, X, wx, wwx, A, B, C, D, dRX);
    const double iz = 1.0 / P[2];
    g.p[0] = -P[0] * iz;
    g.p[1] = -P[1] * iz;
    g.n = g.p[0] * g.p[0] + g.p[1] * g.p[1];
    const double dp_dP[2][3] = {{-iz, 0.0, P[0] * iz * iz}, {0.0, -iz, P[1] * iz * iz}};
    for (int a = 0; a < 2; ++a) {
        for (int j = 0; j < 3; ++j) {
            g.dp[a][j] = dp_dP[a][0] * dRX[0][j] + dp_dP[a][1] * dRX[1][j] + dp_dP[a][2] * dRX[2][j];
            g.dp[a][3 + j] = dp_dP[a][j];
            g.dp[a][6 + j] = dp_dP[a][0] * Rm[j] + dp_dP[a][1] * Rm[3 + j] + dp_dP[a][2] * Rm[6 + j];
        }
    }
}

// ------------------------------------------------------------ point records --
//
// The blocks of an observation depend on it only through its camera-frame
// point P = R X + t: with p = -P_xy / P_z, n = |p|^2, d = 1 + k1 n + k2 n^2,
// A = dpi/dp = f (d I + 2 (k1 + 2 k2 n) p p^T) (symmetric 2x2) and
// dp/dP = -1/P_z [[1, 0, p_0], [0, 1, p_1]],
//   J_P   = dpi/dP = -1/P_z [A_0, A_1, A p]            (2x3)
//   J_p   = [J_P dRX, J_P, d p, f n p, f n^2 p]      dRX = -[P - t]x J_l(w)
//   J_l   = J_P R
// A point record keeps (P, sqrt(w)); the blocks are rebuilt from it and the
// camera record, scaled by sqrt(w) like the stored blocks of the IRLS step.

// Camera-frame point and residual of an observation from the camera record.
__device__ __forceinline__ void camera_point(const double* rec, const double* X, double ox, double oy, double* P,
                                             double* r) {
#pragma clang fp contract(off)
    const double* Rm = rec + 13;
    for (int k = 0; k < 3; ++k) P[k] = Rm[3 * k] * X[0] + Rm[3 * k + 1] * X[1] + Rm[3 * k + 2] * X[2] + rec[3 + k];
    const double iz = 1.0 / P[2];
    const double p0 = -P[0] * iz, p1 = -P[1] * iz;
    const double n = p0 * p0 + p1 * p1;
    const double d = 1.0 + rec[7] * n + rec[8] * n * n;
    r[0] = rec[6] * d * p0 - ox;
    r[1] = rec[6] * d * p1 - oy;
}

// The 24 block scalars (J_p row 0, row 1, J_l row 0, row 1) of a point record,
// times sw, in arithmetic T.
template <typename T>
__device__ __forceinline__ void point_jacobian(const double* rec, const T* P, T sw, T* J) {
#pragma clang fp contract(off)
    const T f = T(rec[6]), k1 = T(rec[7]), k2 = T(rec[8]);
    const T iz = T(1) / P[2];
    const T p0 = -P[0] * iz, p1 = -P[1] * iz;
    const T n = p0 * p0 + p1 * p1;
    const T d = T(1) + k1 * n + k2 * n * n;
    const T dd = T(2) * (k1 + T(2) * k2 * n);
    const T A00 = f * (d + dd * p0 * p0), A01 = f * dd * p0 * p1, A11 = f * (d + dd * p1 * p1);
    T JP[2][3];
    JP[0][0] = -iz * A00;
    JP[0][1] = -iz * A01;
    JP[0][2] = -iz * (A00 * p0 + A01 * p1);
    JP[1][0] = -iz * A01;
    JP[1][1] = -iz * A11;
    JP[1][2] = -iz * (A01 * p0 + A11 * p1);
    // dRX = -[RX]x J_l(w), RX = P - t
    const T w0 = T(rec[0]), w1 = T(rec[1]), w2 = T(rec[2]);
    const T B = T(rec[10]), E = T(rec[22]);
    const T th2 = w0 * w0 + w1 * w1 + w2 * w2;
    const T W[3][3] = {{T(0), -w2, w1}, {w2, T(0), -w0}, {-w1, w0, T(0)}};
    T Jl[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const T ww = (i == j ? -th2 : T(0)) + (i == 0 ? w0 : (i == 1 ? w1 : w2)) * (j == 0 ? w0 : (j == 1 ? w1 : w2));
            Jl[i][j] = (i == j ? T(1) : T(0)) + B * W[i][j] + E * ww;
        }
    const T X0 = P[0] - T(rec[3]), X1 = P[1] - T(rec[4]), X2 = P[2] - T(rec[5]);
    const T S[3][3] = {{T(0), X2, -X1}, {-X2, T(0), X0}, {X1, -X0, T(0)}};  // -[RX]x
    T dRX[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) dRX[i][j] = S[i][0] * Jl[0][j] + S[i][1] * Jl[1][j] + S[i][2] * Jl[2][j];
    const T pp[2] = {p0, p1};
    for (int a = 0; a < 2; ++a) {
        T* Jp = J + 9 * a;
        for (int j = 0; j < 3; ++j) Jp[j] = sw * (JP[a][0] * dRX[0][j] + JP[a][1] * dRX[1][j] + JP[a][2] * dRX[2][j]);
        for (int j = 0; j < 3; ++j) Jp[3 + j] = sw * JP[a][j];
        Jp[6] = sw * (d * pp[a]);
        Jp[7] = sw * (f * n * pp[a]);
        Jp[8] = sw * (f * n * n * pp[a]);
        T* Jl_ = J + 18 + 3 * a;
        for (int j = 0; j < 3; ++j)
            Jl_[j] = sw * (JP[a][0] * T(rec[13 + j]) + JP[a][1] * T(rec[16 + j]) + JP[a][2] * T(rec[19 + j]));
    }
}

// Residual in float64 and the blocks in float32 arithmetic, for float32
// storage: the camera-frame point, the projection and the
// residual in float64 exactly as evaluate_obs_rec forms them (the cost and
// the gain ratio need them), then J_P = dpi/dP, J_p = [J_P dRX, J_P, d p,
// f n p, f n^2 p] with dRX = -[R X]x J_l(w), and J_l = J_P R in float32 from
// R X, 1/P_z, p, n and d rounded to float32 (no cancellation is left to the
// float32 part).  J is unweighted.
__device__ __forceinline__ void evaluate_obs_f32(const double* rec, const double* X, double ox, double oy, double* r,
                                                 float* J) {
#pragma clang fp contract(off)
    const double* Rm = rec + 13;
    double RX[3], P[3];
    for (int k = 0; k < 3; ++k) {
        RX[k] = Rm[3 * k] * X[0] + Rm[3 * k + 1] * X[1] + Rm[3 * k + 2] * X[2];
        P[k] = RX[k] + rec[3 + k];
    }
    const double iz = 1.0 / P[2];
    const double p0 = -P[0] * iz, p1 = -P[1] * iz;
    const double n = p0 * p0 + p1 * p1;
    const double d = 1.0 + rec[7] * n + rec[8] * n * n;
    r[0] = rec[6] * d * p0 - ox;
    r[1] = rec[6] * d * p1 - oy;
    const float fz = float(iz), q0 = float(p0), q1 = float(p1), fn = float(n), fd = float(d);
    const float f = float(rec[6]), k1 = float(rec[7]), k2 = float(rec[8]);
    const float dd = 2.0f * (k1 + 2.0f * k2 * fn);
    const float A00 = f * (fd + dd * q0 * q0), A01 = f * dd * q0 * q1, A11 = f * (fd + dd * q1 * q1);
    float JP[2][3];
    JP[0][0] = -fz * A00;
    JP[0][1] = -fz * A01;
    JP[0][2] = -fz * (A00 * q0 + A01 * q1);
    JP[1][0] = -fz * A01;
    JP[1][1] = -fz * A11;
    JP[1][2] = -fz * (A01 * q0 + A11 * q1);
    const float w0 = float(rec[0]), w1 = float(rec[1]), w2 = float(rec[2]);
    const float B = float(rec[10]), E = float(rec[22]);
    const float th2 = w0 * w0 + w1 * w1 + w2 * w2;
    const float wv[3] = {w0, w1, w2};
    const float W[3][3] = {{0.0f, -w2, w1}, {w2, 0.0f, -w0}, {-w1, w0, 0.0f}};
    float Jw[3][3];  // J_l(w) = I + B [w]x + E (w w^T - th2 I)
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            Jw[i][j] = (i == j ? 1.0f : 0.0f) + B * W[i][j] + E * (wv[i] * wv[j] - (i == j ? th2 : 0.0f));
    const float X0 = float(RX[0]), X1 = float(RX[1]), X2 = float(RX[2]);
    const float S[3][3] = {{0.0f, X2, -X1}, {-X2, 0.0f, X0}, {X1, -X0, 0.0f}};  // -[R X]x
    float dRX[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) dRX[i][j] = S[i][0] * Jw[0][j] + S[i][1] * Jw[1][j] + S[i][2] * Jw[2][j];
    const float qq[2] = {q0, q1};
    for (int a = 0; a < 2; ++a) {
        float* Jp = J + 9 * a;
        for (int j = 0; j < 3; ++j) Jp[j] = JP[a][0] * dRX[0][j] + JP[a][1] * dRX[1][j] + JP[a][2] * dRX[2][j];
        for (int j = 0; j < 3; ++j) Jp[3 + j] = JP[a][j];
        Jp[6] = fd * qq[a];
        Jp[7] = f * fn * qq[a];
        Jp[8] = f * fn * fn * qq[a];
        float* Jl = J + 18 + 3 * a;
        for (int j = 0; j < 3; ++j)
            Jl[j] = JP[a][0] * float(Rm[j]) + JP[a][1] * float(Rm[3 + j]) + JP[a][2] * float(Rm[6 + j]);
    }
}

// Huber on s = |r|^2: rho(s) = s (s <= delta^2), 2 delta sqrt(s) - delta^2 otherwise;
// IRLS weight w = rho'(s) = min(1, delta / sqrt(s)).
__device__ __forceinline__ void huber(double s, double delta, double& rho, double& w) {
    if (s <= delta * delta) {
        rho = s;
        w = 1.0;
    } else {
        const double rs = sqrt(s);
        rho = 2.0 * delta * rs - delta * delta;
        w = delta / rs;
    }
}

}  // namespace poba
