"""Camera model, residuals and Jacobian blocks (oracle; test infrastructure).

The paper fixes the state layout (Sec. 4: d_p = 9 parameters per camera for
the BAL problems, 3 per landmark) and the residual as the discrepancy between
model and observation, but does not write the projection out.  Reading used
here: the public BAL camera convention,

    P  = R(omega) X + t                (R by the Rodrigues formula)
    p  = -P_xy / P_z                   (the camera looks down its -z axis)
    pi = f * (1 + k1 |p|^2 + k2 |p|^4) * p
    r  = pi - o                        (model minus observation)

with camera parameters ordered (omega_x, omega_y, omega_z, t_x, t_y, t_z, f,
k1, k2) and an additive update on all nine (Sec. 4.1: the LM step is an
additive Delta x).

All functions are vectorised over observations and accept complex input, so
the Jacobians can be checked by the complex-step method.
"""
from __future__ import annotations

import numpy as np

SMALL_ANGLE2 = 1e-20


def _cross(a, b):
    return np.stack([
        a[..., 1] * b[..., 2] - a[..., 2] * b[..., 1],
        a[..., 2] * b[..., 0] - a[..., 0] * b[..., 2],
        a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0],
    ], axis=-1)


def _skew(v):
    z = np.zeros_like(v[..., 0])
    return np.stack([
        np.stack([z, -v[..., 2], v[..., 1]], axis=-1),
        np.stack([v[..., 2], z, -v[..., 0]], axis=-1),
        np.stack([-v[..., 1], v[..., 0], z], axis=-1),
    ], axis=-2)


def rotate(omega, X):
    """R(omega) X with the axis-angle form of the Rodrigues formula,
    X cos(th) + (k x X) sin(th) + k (k.X)(1 - cos(th)),  k = omega / th,
    with 1 - cos(th) taken as 2 sin^2(th/2).
    Near th = 0 the first-order form X + omega x X + (omega x (omega x X))/2
    is used (its error is O(th^3 |X|))."""
    omega = np.asarray(omega)
    X = np.asarray(X)
    th2 = np.sum(omega * omega, axis=-1)
    small = np.real(th2) < SMALL_ANGLE2
    th2_safe = np.where(small, 1.0, th2)
    th = np.sqrt(th2_safe)
    k = omega / th[..., None]
    c = np.cos(th)[..., None]
    s = np.sin(th)[..., None]
    kx = _cross(k, X)
    kdx = np.sum(k * X, axis=-1)[..., None]
    omc = 2.0 * np.sin(0.5 * th)[..., None] ** 2  # 1 - cos(th) without cancellation
    gen = X * c + kx * s + k * kdx * omc
    wx = _cross(omega, X)
    approx = X + wx + 0.5 * _cross(omega, wx)
    return np.where(small[..., None], approx, gen)


def camera_points(cams, lms, obs_cam, obs_lm):
    """Landmarks in camera coordinates, P_i = R(omega_c) X_l + t_c  [N,3]."""
    C = np.asarray(cams)[obs_cam]
    X = np.asarray(lms)[obs_lm]
    return rotate(C[:, 0:3], X) + C[:, 3:6]


def project(cams, lms, obs_cam, obs_lm):
    """Model pixel positions pi_i [N,2]."""
    C = np.asarray(cams)[obs_cam]
    P = camera_points(cams, lms, obs_cam, obs_lm)
    p = -P[:, 0:2] / P[:, 2:3]
    r2 = np.sum(p * p, axis=1)
    d = 1.0 + C[:, 7] * r2 + C[:, 8] * r2 * r2
    return (C[:, 6] * d)[:, None] * p


def residuals(cams, lms, obs_cam, obs_lm, obs_xy):
    """r_i = pi_i - o_i  [N,2]  (Sec. 4: residuals are model minus observation)."""
    return project(cams, lms, obs_cam, obs_lm) - np.asarray(obs_xy)


def left_jacobian_so3(omega):
    """Left Jacobian of SO(3): I + (1-cos th)/th^2 [w]x + (th - sin th)/th^3 [w]x^2.
    d/d omega of R(omega) X equals -[R X]x J_l(omega) (first-order expansion
    R(omega + d) = exp([J_l d]x) R(omega))."""
    th2 = np.sum(omega * omega, axis=-1)
    small = np.real(th2) < 1e-12
    th2s = np.where(small, 1.0, th2)
    th = np.sqrt(th2s)
    a = np.where(small, 0.5 - th2 / 24.0, 2.0 * np.sin(0.5 * th) ** 2 / th2s)
    b = np.where(small, 1.0 / 6.0 - th2 / 120.0, (th - np.sin(th)) / (th2s * th))
    K = _skew(omega)
    eye = np.broadcast_to(np.eye(3), K.shape)
    return eye + a[..., None, None] * K + b[..., None, None] * (K @ K)


def jacobians(cams, lms, obs_cam, obs_lm):
    """Analytic Jacobian blocks of r_i: J_p = dr_i/dcam (N,2,9), J_l = dr_i/dX (N,2,3).

    Chain rule through P -> p -> pi:
      dp/dP   = [[-1/Pz, 0, Px/Pz^2], [0, -1/Pz, Py/Pz^2]]
      dpi/dp  = f (d I + p (2 (k1 + 2 k2 |p|^2) p)^T)
      dpi/df  = d p,  dpi/dk1 = f |p|^2 p,  dpi/dk2 = f |p|^4 p
      dP/dX   = R,    dP/dt = I,  dP/domega = -[P - t]x J_l(omega)
    """
    C = np.asarray(cams)[obs_cam]
    X = np.asarray(lms)[obs_lm]
    omega = C[:, 0:3]
    RX = rotate(omega, X)
    P = RX + C[:, 3:6]
    f, k1, k2 = C[:, 6], C[:, 7], C[:, 8]
    iz = 1.0 / P[:, 2]
    p = -P[:, 0:2] * iz[:, None]
    r2 = np.sum(p * p, axis=1)
    d = 1.0 + k1 * r2 + k2 * r2 * r2
    n = P.shape[0]
    dp_dP = np.zeros((n, 2, 3), dtype=P.dtype)
    dp_dP[:, 0, 0] = -iz
    dp_dP[:, 1, 1] = -iz
    dp_dP[:, 0, 2] = P[:, 0] * iz * iz
    dp_dP[:, 1, 2] = P[:, 1] * iz * iz
    dd_dp = 2.0 * (k1 + 2.0 * k2 * r2)[:, None] * p
    dpi_dp = f[:, None, None] * (d[:, None, None] * np.eye(2)[None] + p[:, :, None] * dd_dp[:, None, :])
    dpi_dP = dpi_dp @ dp_dP
    R_cols = rotate(np.repeat(omega[:, None, :], 3, axis=1),
                    np.broadcast_to(np.eye(3), (n, 3, 3)))  # rows: R e_j
    R = np.swapaxes(R_cols, 1, 2)
    dP_dw = -_skew(RX) @ left_jacobian_so3(omega)
    Jp = np.zeros((n, 2, 9), dtype=P.dtype)
    Jp[:, :, 0:3] = dpi_dP @ dP_dw
    Jp[:, :, 3:6] = dpi_dP
    Jp[:, :, 6] = d[:, None] * p
    Jp[:, :, 7] = (f * r2)[:, None] * p
    Jp[:, :, 8] = (f * r2 * r2)[:, None] * p
    Jl = dpi_dP @ R
    return Jp, Jl


def complex_step_jacobians(cams, lms, obs_cam, obs_lm, h=1e-30):
    """Jacobian blocks by the complex-step method (Squire and Trapp 1998):
    df/dx = Im f(x + i h) / h, exact to rounding for real-analytic f."""
    cams = np.asarray(cams, dtype=np.complex128)
    lms = np.asarray(lms, dtype=np.complex128)
    n = len(obs_cam)
    Jp = np.zeros((n, 2, 9))
    Jl = np.zeros((n, 2, 3))
    C = cams[obs_cam]
    X = lms[obs_lm]
    cam_idx = np.arange(n)
    for j in range(9):
        Cj = C.copy()
        Cj[:, j] += 1j * h
        out = project(Cj, X, cam_idx, cam_idx)
        Jp[:, :, j] = np.imag(out) / h
    for j in range(3):
        Xj = X.copy()
        Xj[:, j] += 1j * h
        out = project(C, Xj, cam_idx, cam_idx)
        Jl[:, :, j] = np.imag(out) / h
    return Jp, Jl


def central_difference_jacobians(cams, lms, obs_cam, obs_lm, rel_h=1e-6):
    """Jacobian blocks by central differences, step h = rel_h * max(1, |x|)."""
    cams = np.asarray(cams, dtype=np.float64)
    lms = np.asarray(lms, dtype=np.float64)
    n = len(obs_cam)
    C = cams[obs_cam]
    X = lms[obs_lm]
    idx = np.arange(n)
    Jp = np.zeros((n, 2, 9))
    Jl = np.zeros((n, 2, 3))
    for j in range(9):
        h = rel_h * np.maximum(1.0, np.abs(C[:, j]))
        Cp, Cm = C.copy(), C.copy()
        Cp[:, j] += h
        Cm[:, j] -= h
        Jp[:, :, j] = (project(Cp, X, idx, idx) - project(Cm, X, idx, idx)) / (2.0 * h[:, None])
    for j in range(3):
        h = rel_h * np.maximum(1.0, np.abs(X[:, j]))
        Xp, Xm = X.copy(), X.copy()
        Xp[:, j] += h
        Xm[:, j] -= h
        Jl[:, :, j] = (project(C, Xp, idx, idx) - project(C, Xm, idx, idx)) / (2.0 * h[:, None])
    return Jp, Jl
