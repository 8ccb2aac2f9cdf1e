"""Pins of the oracle's camera model, rotations and Jacobians (CPU only).

None of these re-types the oracle's formulas: rotations are checked against
scipy's independent Rotation class, Jacobians against central finite
differences, the projection against a hand-evaluated example and against the
input generator's independent renderer, and the Jacobian against the exact
scale/translation gauge directions of bundle adjustment.
"""

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
from oracle.camera import CameraState, hat, linearize_observations, project_residuals
from bal_synth import make_config


def test_so3_exp_matches_scipy():
    rng = np.random.default_rng(0)
    w = rng.normal(size=(200, 3)) * rng.uniform(0, 3.1, size=(200, 1))
    w = np.concatenate([w, [[0, 0, 0], [1e-12, 0, 0], [0, -np.pi, 0], [np.pi, 0, 0], [1e-9, 2e-9, -1e-9]]])
    np.testing.assert_allclose(oracle.so3_exp(w), Rotation.from_rotvec(w).as_matrix(), atol=1e-14)


def test_so3_log_roundtrip_including_pi():
    rng = np.random.default_rng(1)
    w = rng.normal(size=(100, 3))
    w = w / np.linalg.norm(w, axis=1, keepdims=True) * rng.uniform(0, np.pi - 1e-3, size=(100, 1))
    np.testing.assert_allclose(oracle.so3_log(oracle.so3_exp(w)), w, atol=1e-10)
    # angle pi (and within 1e-6 of it): the rotation is recovered even if the sign of w flips
    for axis in [np.array([0.0, 1.0, 0.0]), np.array([1.0, 2.0, -2.0]) / 3.0]:
        for th in [np.pi, np.pi - 1e-6]:
            R = Rotation.from_rotvec(th * axis).as_matrix()
            np.testing.assert_allclose(oracle.so3_exp(oracle.so3_log(R)), R, atol=1e-9)


def test_projection_hand_example():
    # R = I, t = (0,0,-10), X = (1,2,0): P = (1,2,-10), p = (0.1, 0.2), |p|^2 = 0.05,
    # f = 500, k1 = 0.1, k2 = 0.01: d = 1 + 0.005 + 0.000025 = 1.005025,
    # pixel = 500 * 1.005025 * (0.1, 0.2) = (50.25125, 100.5025)
    s = CameraState(np.eye(3)[None], np.array([[0.0, 0.0, -10.0]]), np.array([[500.0, 0.1, 0.01]]),
                    np.array([[1.0, 2.0, 0.0]]))
    r = project_residuals(s, np.array([0]), np.array([0]), np.zeros((1, 2)))
    np.testing.assert_allclose(r[0], [50.25125, 100.5025], rtol=1e-14)


def test_generator_renderer_agrees_with_oracle_projection():
    # the generator renders with scipy rotations; at ground truth and zero pixel noise the
    # oracle's independent projection must reproduce its pixels
    p = make_config(0, noise_px=0.0)
    s = oracle.state_from_bal(p.gt_cameras, p.gt_points)
    r = project_residuals(s, p.obs_cam.astype(np.int64), p.obs_pt.astype(np.int64),
                          p.obs_uv.astype(np.float64))
    assert np.max(np.abs(r)) < 1e-4  # float32 rounding of pixels of magnitude ~1e2


def _random_state(rng, n_cams=4, n_pts=6):
    w = rng.normal(size=(n_cams, 3))
    R = oracle.so3_exp(w)
    X = rng.uniform(-1, 1, size=(n_pts, 3))
    # put every camera 6..9 units from the origin looking roughly at it
    centre = rng.normal(size=(n_cams, 3))
    centre = centre / np.linalg.norm(centre, axis=1, keepdims=True) * rng.uniform(6, 9, size=(n_cams, 1))
    # choose R so that the camera's -z axis points at the origin
    Rs = []
    for c in centre:
        zc = c / np.linalg.norm(c)
        up = np.array([0.0, 1.0, 0.0]) if abs(zc[1]) < 0.9 else np.array([1.0, 0.0, 0.0])
        xc = np.cross(up, zc)
        xc /= np.linalg.norm(xc)
        yc = np.cross(zc, xc)
        Rs.append(np.stack([xc, yc, zc]))
    R = np.stack(Rs) @ oracle.so3_exp(0.05 * w)
    t = -np.einsum("nij,nj->ni", R, centre)
    intr = np.stack([rng.uniform(400, 600, n_cams), rng.normal(0, 0.05, n_cams), rng.normal(0, 0.05, n_cams)], 1)
    return CameraState(R, t, intr, X)


def test_jacobians_match_central_differences():
    rng = np.random.default_rng(2)
    s = _random_state(rng)
    ci = np.repeat(np.arange(4), 6)
    pi = np.tile(np.arange(6), 4)
    uv = rng.normal(size=(24, 2))
    r, Jp, Jl = linearize_observations(s, ci, pi, uv)
    h = 1e-6
    fd_p = np.zeros_like(Jp)
    for j in range(9):
        def shifted(sign):
            d = np.zeros((4, 9))
            d[:, j] = sign * h
            s2 = oracle.apply_update(s, d, np.zeros((6, 3)))
            return project_residuals(s2, ci, pi, uv)
        fd_p[:, :, j] = (shifted(1) - shifted(-1)) / (2 * h)
    fd_l = np.zeros_like(Jl)
    for j in range(3):
        def shifted_l(sign):
            d = np.zeros((6, 3))
            d[:, j] = sign * h
            return project_residuals(oracle.apply_update(s, np.zeros((4, 9)), d), ci, pi, uv)
        fd_l[:, :, j] = (shifted_l(1) - shifted_l(-1)) / (2 * h)
    np.testing.assert_allclose(Jp, fd_p, rtol=1e-6, atol=1e-7 * np.abs(Jp).max())
    np.testing.assert_allclose(Jl, fd_l, rtol=1e-6, atol=1e-7 * np.abs(Jl).max())


def test_jacobian_annihilates_gauge_directions():
    # a global translation d (X += d, t -= R d) and a global scale (X, t scaled together)
    # leave every projection unchanged, so J maps both directions to zero
    rng = np.random.default_rng(3)
    s = _random_state(rng)
    ci = np.repeat(np.arange(4), 6)
    pi = np.tile(np.arange(6), 4)
    _, Jp, Jl = linearize_observations(s, ci, pi, np.zeros((24, 2)))
    for d in np.eye(3):
        dxp = np.zeros((4, 9))
        dxp[:, 3:6] = -s.R @ d
        dxl = np.tile(d, (6, 1))
        u = np.einsum("nij,nj->ni", Jp, dxp[ci]) + np.einsum("nij,nj->ni", Jl, dxl[pi])
        assert np.abs(u).max() < 1e-9 * np.abs(Jp).max()
    dxp = np.zeros((4, 9))
    dxp[:, 3:6] = s.t
    u = np.einsum("nij,nj->ni", Jp, dxp[ci]) + np.einsum("nij,nj->ni", Jl, s.X[pi])
    assert np.abs(u).max() < 1e-9 * np.abs(Jp).max() * 10


def test_rotation_jacobian_is_left_increment():
    # for the left update R <- Exp(dw) R, dP/d(dw) = -[R X]_x; check on P directly
    rng = np.random.default_rng(4)
    R = oracle.so3_exp(rng.normal(size=3))
    X = rng.normal(size=3)
    h = 1e-6
    fd = np.stack([((oracle.so3_exp(h * e) @ R - oracle.so3_exp(-h * e) @ R) @ X) / (2 * h)
                   for e in np.eye(3)], axis=1)
    np.testing.assert_allclose(fd, -hat(R @ X), atol=1e-9)
