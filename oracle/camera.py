"""Camera model, rotation parameterization and analytic Jacobians (FP64).

Energy (Sec. 4, eq. ba_energy): E = sum over observations of |r_ij|^2, no 1/2.
Camera model (Sec. 6.2, "Snavely" model with one focal length and two radial
distortion terms), read as the BAL model:
    P = R X + t,   p = -P_xy / P_z,   pi = f (1 + k1 |p|^2 + k2 |p|^4) p,
    r = pi - uv.
Pose dimensionality d_p = 9 (Sec. 4): rotation increment (3), translation (3),
focal length, k1, k2.  The rotation is stored as a matrix and updated on the
left, R <- Exp(dw) R, so dP/d(dw) = -[R X]_x (analytic Jacobians, Sec. 6.1).
The angle-axis vector is produced only when reading cameras back out.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def hat(w: np.ndarray) -> np.ndarray:
    """Skew-symmetric matrices [w]_x for w of shape (..., 3)."""
    z = np.zeros(w.shape[:-1])
    return np.stack([
        np.stack([z, -w[..., 2], w[..., 1]], axis=-1),
        np.stack([w[..., 2], z, -w[..., 0]], axis=-1),
        np.stack([-w[..., 1], w[..., 0], z], axis=-1),
    ], axis=-2)


def so3_exp(w: np.ndarray) -> np.ndarray:
    """Rodrigues' formula in half-angle form, I + (sin t / t) W + (2 sin^2(t/2) / t^2) W^2.

    For t < 1e-8 the second-order series I + W + W^2 / 2 is used.
    """
    w = np.asarray(w, dtype=np.float64)
    th = np.linalg.norm(w, axis=-1)
    W = hat(w)
    W2 = W @ W
    small = th < 1e-8
    ths = np.where(small, 1.0, th)
    a = np.where(small, 1.0, np.sin(ths) / ths)
    b = np.where(small, 0.5, 2.0 * np.sin(0.5 * ths) ** 2 / (ths * ths))
    eye = np.broadcast_to(np.eye(3), W.shape)
    return eye + a[..., None, None] * W + b[..., None, None] * W2


def so3_log(R: np.ndarray) -> np.ndarray:
    """Angle-axis vector of rotation matrices (..., 3, 3), valid up to and at angle pi.

    The angle is atan2(|v| / 2, (tr R - 1) / 2), v the antisymmetric part
    (acos of the trace alone is ill-conditioned near pi).  Above pi/2 the axis
    is taken from the symmetric part cos(t) I + (1 - cos(t)) a a^T, signed by v.
    """
    R = np.asarray(R, dtype=np.float64)
    flat = R.reshape(-1, 3, 3)
    out = np.zeros((flat.shape[0], 3))
    for n, M in enumerate(flat):
        c = 0.5 * (np.trace(M) - 1.0)
        v = np.array([M[2, 1] - M[1, 2], M[0, 2] - M[2, 0], M[1, 0] - M[0, 1]])
        s = 0.5 * np.linalg.norm(v)
        th = np.arctan2(s, c)
        if th < 1e-8:
            out[n] = 0.5 * v
        elif c >= 0.0:
            out[n] = th * v / (2.0 * s)
        else:
            B = (0.5 * (M + M.T) - c * np.eye(3)) / (1.0 - c)
            i = int(np.argmax(np.diag(B)))
            a = B[:, i] / np.sqrt(max(B[i, i], 1e-300))
            a /= np.linalg.norm(a)
            if np.dot(a, v) < 0:
                a = -a
            out[n] = th * a
    return out.reshape(R.shape[:-2] + (3,))


@dataclass
class CameraState:
    R: np.ndarray  # (n_p, 3, 3)
    t: np.ndarray  # (n_p, 3)
    intr: np.ndarray  # (n_p, 3): f, k1, k2
    X: np.ndarray  # (n_l, 3)

    def copy(self) -> "CameraState":
        return CameraState(self.R.copy(), self.t.copy(), self.intr.copy(), self.X.copy())


def state_from_bal(cameras: np.ndarray, points: np.ndarray) -> CameraState:
    cams = np.asarray(cameras, dtype=np.float64)
    return CameraState(so3_exp(cams[:, 0:3]), cams[:, 3:6].copy(), cams[:, 6:9].copy(),
                       np.asarray(points, dtype=np.float64).copy())


def bal_from_state(s: CameraState) -> np.ndarray:
    return np.concatenate([so3_log(s.R), s.t, s.intr], axis=1)


def project_residuals(s: CameraState, ci: np.ndarray, pi: np.ndarray, uv: np.ndarray) -> np.ndarray:
    """r = pi(camera, X) - uv for each observation, shape (n_o, 2)."""
    P = np.einsum("nij,nj->ni", s.R[ci], s.X[pi]) + s.t[ci]
    p = -P[:, 0:2] / P[:, 2:3]
    n2 = np.sum(p * p, axis=1)
    f, k1, k2 = s.intr[ci, 0], s.intr[ci, 1], s.intr[ci, 2]
    d = 1.0 + k1 * n2 + k2 * n2 * n2
    return (f * d)[:, None] * p - uv


def linearize_observations(s: CameraState, ci: np.ndarray, pi: np.ndarray, uv: np.ndarray):
    """Residuals r (n,2), pose Jacobians Jp (n,2,9) and landmark Jacobians Jl (n,2,3)."""
    RX = np.einsum("nij,nj->ni", s.R[ci], s.X[pi])
    P = RX + s.t[ci]
    Px, Py, Pz = P[:, 0], P[:, 1], P[:, 2]
    p = np.stack([-Px / Pz, -Py / Pz], axis=1)
    n2 = np.sum(p * p, axis=1)
    f, k1, k2 = s.intr[ci, 0], s.intr[ci, 1], s.intr[ci, 2]
    d = 1.0 + k1 * n2 + k2 * n2 * n2
    r = (f * d)[:, None] * p - uv

    n = ci.shape[0]
    # dp/dP (2x3)
    dp_dP = np.zeros((n, 2, 3))
    dp_dP[:, 0, 0] = -1.0 / Pz
    dp_dP[:, 0, 2] = Px / (Pz * Pz)
    dp_dP[:, 1, 1] = -1.0 / Pz
    dp_dP[:, 1, 2] = Py / (Pz * Pz)
    # dpi/dp = f (d I + 2 (k1 + 2 k2 |p|^2) p p^T)
    g = 2.0 * (k1 + 2.0 * k2 * n2)
    dpi_dp = (f * d)[:, None, None] * np.eye(2)[None] + (f * g)[:, None, None] * np.einsum("ni,nj->nij", p, p)
    dpi_dP = dpi_dp @ dp_dP  # (n,2,3)

    Jp = np.zeros((n, 2, 9))
    Jp[:, :, 0:3] = dpi_dP @ (-hat(RX))  # left rotation increment
    Jp[:, :, 3:6] = dpi_dP
    Jp[:, :, 6] = d[:, None] * p
    Jp[:, :, 7] = (f * n2)[:, None] * p
    Jp[:, :, 8] = (f * n2 * n2)[:, None] * p
    Jl = dpi_dP @ s.R[ci]
    return r, Jp, Jl


def apply_update(s: CameraState, dxp: np.ndarray, dxl: np.ndarray) -> CameraState:
    """x (+) dx: R <- Exp(dw) R, t, f, k1, k2 and X additive.  dxp (n_p,9), dxl (n_l,3)."""
    return CameraState(
        so3_exp(dxp[:, 0:3]) @ s.R,
        s.t + dxp[:, 3:6],
        s.intr + dxp[:, 6:9],
        s.X + dxl,
    )
