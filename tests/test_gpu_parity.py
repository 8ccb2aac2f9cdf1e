"""GPU path (through the C ABI) against the FP64 oracle, step by step.

Tolerances: index bookkeeping bit-exact; FP32 per-observation residuals within
1e-4 px and Jacobians within 1e-4 relative per observation; the
reduced camera system (matrix and right-hand side) within 1e-4 relative in
Frobenius norm; per-landmark invariants within 1e-4 relative; LM final cost
within 1e-3 relative.  Landmark blocks themselves are not unique (Q2 is unique
only up to an orthogonal factor), so blocks are compared only through
invariants.
"""

import numpy as np
import pytest

import oracle
from bal_synth import make_config, make_ring_problem, concat_problems, make_batch

from gpu_util import CLASS_EDGES, check_precond_blocks, gpu_context, landmark_sc_contribution, mixed_problem, oracle_lin

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", params=["tiny", "mixed"])
def case(request):
    p = make_config(0) if request.param == "tiny" else mixed_problem()
    bk, st, lin = oracle_lin(p)
    ctx = gpu_context(p)
    yield p, bk, st, lin, ctx
    ctx.close()


def test_bookkeeping_bit_exact(case):
    p, bk, st, lin, ctx = case
    g = ctx.debug_bookkeeping()
    assert np.array_equal(g["obs_perm"], bk.obs_perm)
    assert np.array_equal(g["lm_off"], bk.lm_off)
    assert np.array_equal(g["lm_active"], bk.lm_active)
    assert np.array_equal(g["cam_active"], bk.cam_active)


def test_linearization_per_observation(case):
    p, bk, st, lin, ctx = case
    r, Jp, Jl = ctx.debug_linearization()
    # FP32 rounding of R (the GPU stores it in FP32) and of the projection chain moves the
    # normalized point p by ~eps32 (|RX| + |t|) / |P_z| ~ 1e-7, i.e. ~f 1e-7 = 5e-5 px for
    # f ~ 500: the residuals must agree to 1e-4 px absolute
    err = np.abs(r - lin.r).max()
    assert err <= 1e-4, f"residual error {err:.3g} px"
    ep = np.linalg.norm((Jp - lin.Jp).reshape(len(r), -1), axis=1) / np.linalg.norm(lin.Jp.reshape(len(r), -1), axis=1)
    el = np.linalg.norm((Jl - lin.Jl).reshape(len(r), -1), axis=1) / np.linalg.norm(lin.Jl.reshape(len(r), -1), axis=1)
    assert ep.max() < 1e-4 and el.max() < 1e-4


def test_cost_and_scales(case):
    p, bk, st, lin, ctx = case
    cost = ctx.linearize()[0]
    assert abs(cost - lin.cost) <= 1e-5 * lin.cost
    ctx.marginalize()
    sc, sp = ctx.debug_scales()
    np.testing.assert_allclose(sc, lin.sp, rtol=1e-5)
    act = bk.lm_active
    np.testing.assert_allclose(sp[act], lin.sl[act], rtol=1e-5)


@pytest.mark.parametrize("lam", [0.0, 1e-4, 0.3])
def test_landmark_block_invariants(case, lam):
    """Per landmark, S B^T B S = H_pp - H_pl (H_ll + lam I)^-1 H_lp (eq. red_H, damped remark
    of Sec. 4.4) and S B^T rho = b_p - H_pl (H_ll + lam I)^-1 b_l (eq. red_b)."""
    p, bk, st, lin, ctx = case
    ctx.linearize()
    ctx.marginalize()
    if lam > 0:
        ctx.damp(lam)
    sc, _ = ctx.debug_scales()
    rng = np.random.default_rng(0)
    ls = np.nonzero(bk.lm_active)[0]
    # every landmark of the mixed case (each k class), a sample of the tiny one
    pick = ls if len(ls) <= 300 else rng.choice(ls, 120, replace=False)
    worst = 0.0
    for l in pick:
        cams, H, b, Jp, Jl, r = landmark_sc_contribution(lin, l, lam)
        k, blk, fac = ctx.debug_block(int(l))
        assert k == len(cams)
        rows = blk[3:] if lam > 0 else blk[3:3 + 2 * k - 3]
        s = np.concatenate([sc[c] for c in cams]).astype(np.float64)
        B = rows[:, :9 * k].astype(np.float64) * s[None, :]
        rho = rows[:, 9 * k + 3].astype(np.float64)
        eH = np.linalg.norm(B.T @ B - H) / max(np.linalg.norm(H), 1e-30)
        # Q2^T r can be orders of magnitude smaller than r (the landmark explains almost all of its
        # residual); an FP32 orthogonal transform leaves it an absolute error of a few eps32 |r|
        # (backward stability), so the right-hand side term gets 1e-4 |b| plus 64 eps32 |J_p| |r|
        tol_b = 1e-4 * np.linalg.norm(b) + 64 * 2.0 ** -24 * np.linalg.norm(Jp, 2) * np.linalg.norm(r)
        eb = 1e-4 * np.linalg.norm(B.T @ rho - b) / tol_b  # <= 1e-4 when within tolerance
        worst = max(worst, eH, eb)
        # the landmark columns of the B rows are exactly zero (Q2^T J_l = 0) by construction;
        # the top rows carry R1 with R1^T R1 = J_l^T J_l (scaled)
        R1 = blk[:3, 9 * k:9 * k + 3].astype(np.float64)
        np.testing.assert_allclose(R1.T @ R1, Jl.T @ Jl, atol=2e-5 * np.abs(Jl.T @ Jl).max())
        if lam > 0:
            Rh = np.zeros((3, 3))
            Rh[np.triu_indices(3)] = fac[9:15]
            np.testing.assert_allclose(Rh.T @ Rh, R1.T @ R1 + lam * np.eye(3), atol=2e-5 * (1 + lam))
    assert worst < 1e-4, worst


@pytest.mark.parametrize("lam", [0.0, 1e-4])
def test_largest_landmarks_in_row_chunks(lam):
    """Landmarks with k = 170 .. 512 observations: the QR of a block wider than one
    workgroup's chunk of rows (2 MiB) is written by several workgroups; every
    chunk must carry the same rotation.  Same invariants as above (eq. red_H /
    red_b), on every landmark, plus R1^T R1 = J_l^T J_l."""
    rng = np.random.default_rng(21)
    p = make_ring_problem(rng, 520, 8, lambda r, n: np.array([170, 171, 300, 512, 2, 5, 113, 114])[:n])
    bk, st, lin = oracle_lin(p)
    ctx = gpu_context(p)
    ctx.linearize()
    ctx.marginalize()
    if lam > 0:
        ctx.damp(lam)
    sc, _ = ctx.debug_scales()
    worst = 0.0
    for l in np.nonzero(bk.lm_active)[0]:
        cams, H, b, Jp, Jl, r = landmark_sc_contribution(lin, l, lam)
        k, blk, fac = ctx.debug_block(int(l))
        assert k == len(cams)
        rows = blk[3:] if lam > 0 else blk[3:3 + 2 * k - 3]
        s = np.concatenate([sc[c] for c in cams]).astype(np.float64)
        B = rows[:, :9 * k].astype(np.float64) * s[None, :]
        rho = rows[:, 9 * k + 3].astype(np.float64)
        eH = np.linalg.norm(B.T @ B - H) / max(np.linalg.norm(H), 1e-30)
        tol_b = 1e-4 * np.linalg.norm(b) + 64 * 2.0 ** -24 * np.linalg.norm(Jp, 2) * np.linalg.norm(r)
        eb = 1e-4 * np.linalg.norm(B.T @ rho - b) / tol_b
        worst = max(worst, eH, eb)
        R1 = blk[:3, 9 * k:9 * k + 3].astype(np.float64)
        np.testing.assert_allclose(R1.T @ R1, Jl.T @ Jl, atol=2e-5 * np.abs(Jl.T @ Jl).max())
    ctx.close()
    assert worst < 1e-4, worst


def test_orthogonal_transform_preserves_columns(case):
    """Undamped block rows are Q^T [J_p | J_l S_l | r]: column Gram matrices are preserved."""
    p, bk, st, lin, ctx = case
    ctx.linearize()
    ctx.marginalize()
    ls = np.nonzero(bk.lm_active)[0][:60]
    for l in ls:
        cams, H, b, Jp, Jl, r = landmark_sc_contribution(lin, l, 0.0)
        k, blk, fac = ctx.debug_block(int(l))
        rows = np.vstack([blk[:3], blk[3:3 + 2 * k - 3]]).astype(np.float64)
        s = np.concatenate([lin.sp[c] for c in cams])
        A = np.hstack([rows[:, :9 * k] * s[None, :], rows[:, 9 * k:9 * k + 3], rows[:, 9 * k + 3:]])
        A0 = np.hstack([Jp, Jl, r[:, None]])
        G, G0 = A.T @ A, A0.T @ A0
        assert np.linalg.norm(G - G0) <= 1e-5 * np.linalg.norm(G0)


def test_reduced_camera_system_dense(case):
    p, bk, st, lin, ctx = case
    lam = 1e-4
    ctx.linearize()
    ctx.marginalize()
    ctx.damp(lam)
    rs = oracle.reduced_camera_system(lin, lam)
    N = rs.H.shape[0]
    Hg = ctx.debug_rcs_matvec(np.eye(N, dtype=np.float32)).astype(np.float64)
    eH = np.linalg.norm(Hg - rs.H) / np.linalg.norm(rs.H)
    assert eH <= 1e-4, eH
    bg = ctx.debug_rhs().astype(np.float64)
    eb = np.linalg.norm(bg - rs.b) / np.linalg.norm(rs.b)
    assert eb <= 1e-4, eb
    # block-Jacobi: every camera's block against the oracle's 9x9 diagonal block
    check_precond_blocks(ctx, oracle.block_jacobi_blocks(rs.H))


def test_pcg_and_back_substitution(case):
    p, bk, st, lin, ctx = case
    lam = 1e-4
    ctx.linearize()
    ctx.marginalize()
    ctx.damp(lam)
    its, rel, status = ctx.solve()
    rs = oracle.reduced_camera_system(lin, lam)
    dxp, _ = ctx.debug_solution()
    assert status[0] == 0 and rel[0] <= 1e-6
    # the GPU solution solves the oracle's system to the PCG tolerance (scaled by conditioning)
    res = np.linalg.norm(rs.H @ dxp + rs.b) / np.linalg.norm(rs.b)
    assert res < 1e-3, res
    # back-substitution from the oracle's exact pose increment
    ref = oracle.dense_spd_solve(rs.H, -rs.b)
    ctx.debug_set_pose_increment(ref.astype(np.float32))
    pred = ctx.back_substitute()[0]
    _, dxl = ctx.debug_solution()
    dxl_o = (oracle.back_substitute(rs, ref).reshape(-1, 3) * lin.sl)
    act = bk.lm_active
    e = np.linalg.norm(dxl[act] - dxl_o[act]) / np.linalg.norm(dxl_o[act])
    assert e <= 1e-4, e
    pred_o = oracle.model_decrease(lin, ref, oracle.back_substitute(rs, ref))
    assert abs(pred - pred_o) <= 1e-4 * abs(pred_o), (pred, pred_o)


@pytest.mark.parametrize("lam", [1e-4, 1e-2])
def test_pcg_forcing_truncation(case, lam):
    """With the Nash-Sofer forcing test (eta = 0.1, Sec. 6.1 "forcing sequence"), the GPU
    stops within one iteration of the oracle (the GPU tracks Q by its recurrence in FP32-fed
    FP64 sums, the oracle evaluates it from its definition), and its iterate equals the
    oracle's after the same number of iterations."""
    p, bk, st, lin, ctx = case
    ctx.set_options(pcg_forcing_eta=0.1)
    try:
        ctx.linearize()
        ctx.marginalize()
        ctx.damp(lam)
        its, rel, status = ctx.solve()
    finally:
        ctx.set_options(pcg_forcing_eta=0.0)
    rs = oracle.reduced_camera_system(lin, lam)
    blocks = oracle.block_jacobi_blocks(rs.H)
    mv = lambda v: rs.H @ v  # noqa: E731
    ref = oracle.pcg(mv, rs.b, blocks, tol=1e-6, eta=0.1)
    plain = oracle.pcg(mv, rs.b, blocks, tol=1e-6)
    assert status[0] == 0
    assert abs(int(its[0]) - ref.iters) <= 1, (its[0], ref.iters)
    assert ref.iters < plain.iters  # the truncation does cut the solve short here
    same = oracle.pcg(mv, rs.b, blocks, tol=0.0, max_iters=int(its[0]))
    dxp, _ = ctx.debug_solution()
    e = np.linalg.norm(dxp - same.x) / np.linalg.norm(same.x)
    assert e <= 1e-3, e


def test_update_cost_matches_oracle(case):
    p, bk, st, lin, ctx = case
    lam = 1e-3
    ctx.linearize()
    ctx.marginalize()
    ctx.damp(lam)
    rs = oracle.reduced_camera_system(lin, lam)
    ref = oracle.dense_spd_solve(rs.H, -rs.b)
    ctx.debug_set_pose_increment(ref.astype(np.float32))
    ctx.back_substitute()
    new_cost = ctx.update()[0]
    dxl = oracle.back_substitute(rs, ref)
    ns = oracle.apply_update(st, ref.reshape(-1, 9) * lin.sp, dxl.reshape(-1, 3) * lin.sl)
    from oracle.lm import cost_of
    c_o = cost_of(ns, bk, p.obs_uv)
    assert abs(new_cost - c_o) <= 1e-4 * lin.cost, (new_cost, c_o)
    ctx.commit([0])


def test_lm_final_cost(case):
    p, bk, st, lin, ctx = case
    ref = oracle.lm_solve(p.cameras, p.points, p.obs_cam, p.obs_pt, p.obs_uv,
                          oracle.LMOptions(max_iters=10), bk)
    ctx = gpu_context(p, max_lm_iters=10)
    rep = ctx.lm_solve()[0]
    hist = ctx.history(0)
    assert rep.iterations == len(hist) <= 10
    acc = [h["new_cost"] for h in hist if h["accepted"]]
    assert all(b < a for a, b in zip([rep.initial_cost] + acc, acc))
    assert abs(rep.final_cost - ref.final_cost) <= 1e-3 * ref.final_cost, (rep.final_cost, ref.final_cost)
    # the final state's cost, evaluated by the oracle, agrees too
    cams, pts = ctx.get_cameras(), ctx.get_landmarks()
    from oracle.lm import cost_of
    c = cost_of(oracle.state_from_bal(cams, pts), bk, p.obs_uv)
    ctx.close()
    assert abs(c - rep.final_cost) <= 1e-4 * rep.final_cost


def test_deterministic_reruns():
    p = mixed_problem(seed=9, n_cams=40, n_points=120)
    out = []
    for _ in range(2):
        ctx = gpu_context(p)
        ctx.linearize()
        ctx.marginalize()
        ctx.damp(1e-3)
        its, rel, st = ctx.solve()
        pred = ctx.back_substitute()
        dxp, dxl = ctx.debug_solution()
        out.append((its.copy(), dxp.copy(), dxl.copy(), pred.copy()))
        ctx.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1]) and np.array_equal(out[0][2], out[1][2])
    assert np.array_equal(out[0][3], out[1][3])
