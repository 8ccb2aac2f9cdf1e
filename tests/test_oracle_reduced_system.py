"""Pins of the oracle's explicit Schur complement through independent routes (CPU only).

* Nullspace marginalization computed with numpy's LAPACK QR (Sec. 4.3) must
  reproduce the Schur complement (Sec. 4.4, eq. red_H and red_b), undamped and
  damped (the damped remark closing Sec. 4.4, landmark damping rows Sec. 5.3).
* The QR facts of Sec. 3 (eq. q_orth, qqt) hold for those factors.
* A dense Cholesky of the whole damped system over all unknowns must equal
  the reduced solve followed by back-substitution (Sec. 4.2 / 4.3).
* The NM back-substitution (eq. backsub_nm) equals the SC one (eq. backsub_sc).
* Column scaling gives unit columns.
"""

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from oracle.normal_equations import scaled_jacobian_sparse
from bal_synth import make_ring_problem


def _tiny(seed=0, n_cams=6, n_pts=40):
    rng = np.random.default_rng(seed)
    p = make_ring_problem(rng, n_cams, n_pts, lambda r, n: r.integers(2, 6, size=n))
    bk = oracle.build_bookkeeping(p.n_cams, p.n_points, p.obs_cam, p.obs_pt, p.obs_uv)
    st = oracle.state_from_bal(p.cameras, p.points)
    lin = oracle.linearize(st, bk, p.obs_uv)
    return p, bk, st, lin


def _landmark_rows(lin):
    """Per landmark: scaled J_p restricted to its cameras (2k x 9k), J_l (2k x 3), r (2k), cams."""
    out = []
    for l in range(lin.n_points):
        idx = np.nonzero(lin.pi == l)[0]
        if idx.size == 0:
            continue
        k = idx.size
        cams = lin.ci[idx]
        Jp = np.zeros((2 * k, 9 * k))
        for a, o in enumerate(idx):
            Jp[2 * a:2 * a + 2, 9 * a:9 * a + 9] = lin.Jp[o] * lin.sp[lin.ci[o]]
        Jl = (lin.Jl[idx] * lin.sl[l]).reshape(2 * k, 3)
        out.append((l, cams, Jp, Jl, lin.r[idx].reshape(-1)))
    return out


def _scatter(H, b, cams, Bp, rr):
    k = len(cams)
    G = Bp.T @ Bp
    g = Bp.T @ rr
    for a in range(k):
        ia = slice(9 * cams[a], 9 * cams[a] + 9)
        b[ia] += g[9 * a:9 * a + 9]
        for c in range(k):
            H[ia, 9 * cams[c]:9 * cams[c] + 9] += G[9 * a:9 * a + 9, 9 * c:9 * c + 9]


@pytest.mark.parametrize("lam", [0.0, 1e-4, 0.3])
def test_nullspace_marginalization_equals_schur_complement(lam):
    p, bk, st, lin = _tiny()
    rs = oracle.reduced_camera_system(lin, lam)
    N = 9 * lin.n_cams
    H = lam * np.eye(N)
    b = np.zeros(N)
    for l, cams, Jp, Jl, r in _landmark_rows(lin):
        k = len(cams)
        # damped landmark block: append [0 | sqrt(lam) I | 0] rows (Sec. 5.3)
        A = np.vstack([Jl, np.sqrt(lam) * np.eye(3)]) if lam > 0 else Jl
        P = np.vstack([Jp, np.zeros((3, 9 * k))]) if lam > 0 else Jp
        rr = np.concatenate([r, np.zeros(3)]) if lam > 0 else r
        Q, R = np.linalg.qr(A, mode="complete")
        Q2 = Q[:, 3:]
        # Sec. 3 facts
        np.testing.assert_allclose(Q.T @ Q, np.eye(Q.shape[0]), atol=1e-12)
        assert np.abs(Q2.T @ A).max() < 1e-12 * max(1.0, np.abs(A).max())
        np.testing.assert_allclose(Q[:, :3] @ Q[:, :3].T, np.eye(Q.shape[0]) - Q2 @ Q2.T, atol=1e-12)
        np.testing.assert_allclose(R[:3].T @ R[:3], A.T @ A, atol=1e-12)
        _scatter(H, b, cams, Q2.T @ P, Q2.T @ rr)
    scale = np.abs(rs.H).max()
    np.testing.assert_allclose(H, rs.H, atol=1e-11 * scale)
    np.testing.assert_allclose(b, rs.b, atol=1e-11 * np.abs(rs.b).max())


def test_full_damped_system_equals_reduced_solve_and_back_substitution():
    p, bk, st, lin = _tiny(seed=1)
    lam = 1e-3
    Jp_m, Jl_m, r = scaled_jacobian_sparse(lin)
    J = np.hstack([Jp_m.toarray(), Jl_m.toarray()])
    # drop columns of landmarks/cameras that have no rows (none here, but keep it general)
    H = J.T @ J + lam * np.eye(J.shape[1])
    full = sla.cho_solve(sla.cho_factor(H), -J.T @ r)
    rs = oracle.reduced_camera_system(lin, lam)
    dxp = oracle.dense_spd_solve(rs.H, -rs.b)
    dxl = oracle.back_substitute(rs, dxp)
    np.testing.assert_allclose(dxp, full[: dxp.size], rtol=1e-9, atol=1e-9 * np.abs(full).max())
    np.testing.assert_allclose(dxl, full[dxp.size:], rtol=1e-9, atol=1e-9 * np.abs(full).max())


def test_nm_back_substitution_equals_sc_back_substitution():
    p, bk, st, lin = _tiny(seed=2)
    lam = 1e-2
    rs = oracle.reduced_camera_system(lin, lam)
    dxp = oracle.dense_spd_solve(rs.H, -rs.b)
    dxl = oracle.back_substitute(rs, dxp).reshape(lin.n_points, 3)
    for l, cams, Jp, Jl, r in _landmark_rows(lin):
        k = len(cams)
        A = np.vstack([Jl, np.sqrt(lam) * np.eye(3)])
        Q, R = np.linalg.qr(A, mode="complete")
        Q1 = Q[:, :3]
        P = np.vstack([Jp, np.zeros((3, 9 * k))])
        rr = np.concatenate([r, np.zeros(3)])
        v = np.concatenate([dxp[9 * c: 9 * c + 9] for c in cams])
        nm = -np.linalg.solve(R[:3], Q1.T @ rr + Q1.T @ P @ v)  # eq. backsub_nm
        np.testing.assert_allclose(nm, dxl[l], rtol=1e-8, atol=1e-10)


def test_column_scaling_unit_norm():
    p, bk, st, lin = _tiny(seed=3)
    Jp_m, Jl_m, _ = scaled_jacobian_sparse(lin)
    cn = np.sqrt(np.asarray(Jp_m.multiply(Jp_m).sum(axis=0))).ravel()
    ln = np.sqrt(np.asarray(Jl_m.multiply(Jl_m).sum(axis=0))).ravel()
    np.testing.assert_allclose(cn, 1.0, atol=1e-12)
    np.testing.assert_allclose(ln, 1.0, atol=1e-12)


def test_reduced_system_gauge_nullity_undamped():
    # BA has a 7-DoF similarity gauge (rotation, translation, scale), so the undamped
    # reduced matrix of a well-observed scene has exactly 7 near-zero eigenvalues
    p, bk, st, lin = _tiny(seed=4, n_cams=8, n_pts=120)
    ev = np.linalg.eigvalsh(oracle.reduced_camera_system(lin, 0.0).H)
    ev = ev / ev.max()
    assert np.sum(ev < 1e-9) == 7
    assert ev[7] > 1e-8


def test_model_decrease_equals_direct_model_evaluation():
    p, bk, st, lin = _tiny(seed=5)
    rs = oracle.reduced_camera_system(lin, 1e-4)
    dxp = oracle.dense_spd_solve(rs.H, -rs.b)
    dxl = oracle.back_substitute(rs, dxp)
    Jp_m, Jl_m, r = scaled_jacobian_sparse(lin)
    model = np.sum((r + Jp_m @ dxp + Jl_m @ dxl) ** 2)
    pred = oracle.model_decrease(lin, dxp, dxl)
    assert pred > 0
    np.testing.assert_allclose(pred, lin.cost - model, rtol=1e-9)


def _with_inactive(p):
    """Add a landmark seen once (inactive: no rows) and a camera without observations."""
    from bal_synth import Problem
    cams = np.vstack([p.cameras, p.cameras[0:1]]).astype(np.float32)
    cams[-1, 3:6] += 50.0
    pts = np.vstack([p.points, [[0.1, 0.2, 0.3]]]).astype(np.float32)
    oc = np.concatenate([p.obs_cam, [1]]).astype(np.int32)
    op = np.concatenate([p.obs_pt, [p.n_points]]).astype(np.int32)
    uv = np.vstack([p.obs_uv, [[2.0, -1.0]]]).astype(np.float32)
    return Problem("inactive", cams, pts, oc, op, uv, p.gt_cameras, p.gt_points)


@pytest.mark.parametrize("lam", [1e-6, 1e-4, 0.3])
def test_operator_equals_dense_schur_complement_of_the_full_system(lam):
    """The operator form (Sec. 4.2 applied to vectors) against the Schur complement of
    the full damped matrix J~^T J~ + lam I formed densely over all unknowns and reduced
    with a dense inverse of its landmark part (brute force, tiny problem)."""
    p, _, _, _ = _tiny(seed=7)
    p = _with_inactive(p)
    bk = oracle.build_bookkeeping(p.n_cams, p.n_points, p.obs_cam, p.obs_pt, p.obs_uv)
    lin = oracle.linearize(oracle.state_from_bal(p.cameras, p.points), bk, p.obs_uv)
    op = oracle.reduced_system_operator(lin, lam)
    Jp_m, Jl_m, r = scaled_jacobian_sparse(lin)
    Jp, Jl = Jp_m.toarray(), Jl_m.toarray()
    used = np.abs(Jl).sum(axis=0) > 0  # landmark columns with rows
    Jl = Jl[:, used]
    N = Jp.shape[1]
    App = Jp.T @ Jp + lam * np.eye(N)
    Apl = Jp.T @ Jl
    All = Jl.T @ Jl + lam * np.eye(Jl.shape[1])
    H = App - Apl @ np.linalg.inv(All) @ Apl.T
    b = Jp.T @ r - Apl @ np.linalg.solve(All, Jl.T @ r)
    Hop = np.stack([op.matvec(e) for e in np.eye(N)], axis=1)
    scale = np.abs(H).max()
    np.testing.assert_allclose(Hop, H, atol=1e-10 * scale)
    np.testing.assert_allclose(op.b, b, atol=1e-10 * np.abs(b).max())
    for i in range(lin.n_cams):
        np.testing.assert_allclose(op.blocks[i], H[9 * i:9 * i + 9, 9 * i:9 * i + 9], atol=1e-10 * scale)
    # back-substitution: the landmark rows of the full damped solve
    Hf = np.block([[App, Apl], [Apl.T, All]])
    full = np.linalg.solve(Hf, -np.concatenate([Jp.T @ r, Jl.T @ r]))
    dxl = oracle.back_substitute(op, full[:N]).reshape(-1, 3)
    np.testing.assert_allclose(dxl[used.reshape(-1, 3).all(axis=1)].ravel(), full[N:],
                               atol=1e-9 * np.abs(full).max())
    # the unused camera's column block is lam I
    np.testing.assert_allclose(op.blocks[-1], lam * np.eye(9), atol=1e-300)


def test_operator_equals_assembled_schur_complement():
    """Operator and assembled forms give the same reduced system, preconditioner blocks,
    back-substitution and LM trajectory (ring problem with every landmark size 3..8)."""
    p, bk, st, lin = _tiny(seed=8, n_cams=10, n_pts=150)
    for lam in (1e-4, 2.0):
        rs = oracle.reduced_camera_system(lin, lam)
        op = oracle.reduced_system_operator(lin, lam)
        rng = np.random.default_rng(0)
        for _ in range(4):
            v = rng.normal(size=rs.b.shape)
            np.testing.assert_allclose(op.matvec(v), rs.H @ v, rtol=1e-10, atol=1e-12 * np.abs(rs.H @ v).max())
        np.testing.assert_allclose(op.b, rs.b, atol=1e-12 * np.abs(rs.b).max())
        np.testing.assert_allclose(op.blocks, oracle.block_jacobi_blocks(rs.H), atol=1e-12 * np.abs(rs.H).max())
        x = rng.normal(size=rs.b.shape)
        np.testing.assert_allclose(oracle.back_substitute(op, x), oracle.back_substitute(rs, x), rtol=1e-10,
                                   atol=1e-12)
    a = oracle.lm_solve(p.cameras, p.points, p.obs_cam, p.obs_pt, p.obs_uv, oracle.LMOptions(max_iters=8))
    b = oracle.lm_solve(p.cameras, p.points, p.obs_cam, p.obs_pt, p.obs_uv,
                        oracle.LMOptions(max_iters=8, solver="pcg_operator"))
    assert [h["accepted"] for h in a.history] == [h["accepted"] for h in b.history]
    assert [h["pcg_iters"] for h in a.history] == [h["pcg_iters"] for h in b.history]
    assert b.final_cost == pytest.approx(a.final_cost, rel=1e-9)
