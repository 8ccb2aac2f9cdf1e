"""Edge cases and the batched form through the C ABI (GPU)."""

import numpy as np
import pytest

import oracle
from bal_synth import make_config, make_batch, concat_problems

from gpu_util import gpu_context, oracle_lin, with_extras

pytestmark = pytest.mark.gpu


def _ctx(**kw):
    import torch
    from paper_2103_01843_amd import Context
    return Context(stream=torch.cuda.current_stream(), **kw)


@pytest.mark.parametrize("case,code", [("dup", -1), ("cam_range", -1), ("pt_range", -1), ("nan", -5),
                                       ("too_many", -6), ("empty", -1)])
def test_invalid_input_is_rejected(case, code):
    from paper_2103_01843_amd import SqrtBAError
    n_cams = 600 if case == "too_many" else 4
    cams = np.tile(np.array([0, 0, 0, 0, 0, -10, 500, 0, 0], np.float32), (n_cams, 1))
    pts = np.zeros((3, 3), np.float32)
    oc = np.array([0, 1, 1, 2], np.int32)
    op = np.array([0, 0, 1, 1], np.int32)
    uv = np.zeros((4, 2), np.float32)
    if case == "dup":
        oc[1], op[1] = 0, 0
    elif case == "cam_range":
        oc[2] = n_cams
    elif case == "pt_range":
        op[0] = 3
    elif case == "nan":
        uv[3, 0] = np.inf
    elif case == "too_many":
        oc = np.arange(513, dtype=np.int32)
        op = np.zeros(513, np.int32)
        uv = np.zeros((513, 2), np.float32)
    elif case == "empty":
        oc, op, uv = oc[:0], op[:0], uv[:0]
    with _ctx() as ctx:
        ctx.set_cameras(cams)
        ctx.set_landmarks(pts)
        with pytest.raises(SqrtBAError) as ei:
            ctx.set_observations(oc, op, uv)
        assert ei.value.status == code
        # calls out of order are rejected too
        with pytest.raises(SqrtBAError) as ei:
            ctx.marginalize()
        assert ei.value.status in (-4,)


def test_inactive_and_degenerate_cases():
    p = with_extras(make_config(0))
    bk, st, lin = oracle_lin(p)
    assert not bk.lm_active[p.n_points - 2] and bk.lm_active[p.n_points - 1]
    assert not bk.cam_active[p.n_cams - 2]
    ctx = gpu_context(p, max_lm_iters=10)
    g = ctx.debug_bookkeeping()
    assert np.array_equal(g["obs_perm"], bk.obs_perm) and np.array_equal(g["lm_off"], bk.lm_off)
    assert np.array_equal(g["lm_active"], bk.lm_active) and np.array_equal(g["cam_active"], bk.cam_active)
    ctx.linearize()
    ctx.marginalize()
    lam = 1e-4
    ctx.damp(lam)
    # the rank-2 landmark: R1 is singular, the damped R is not; the damped invariant holds
    l = p.n_points - 1
    k, blk, fac = ctx.debug_block(l)
    assert k == 2 and np.all(np.isfinite(blk))
    Rh = np.zeros((3, 3))
    Rh[np.triu_indices(3)] = fac[9:15]
    assert abs(np.linalg.det(Rh)) > 0
    its, rel, st_ = ctx.solve()
    assert st_[0] == 0
    dxp, dxl = ctx.debug_solution()
    assert np.all(np.isfinite(dxp)) and np.all(np.isfinite(dxl))
    # the unused camera and the inactive landmark do not move
    assert np.all(dxp[9 * (p.n_cams - 2): 9 * (p.n_cams - 1)] == 0)
    ctx.close()
    ref = oracle.lm_solve(p.cameras, p.points, p.obs_cam, p.obs_pt, p.obs_uv, oracle.LMOptions(max_iters=10), bk)
    ctx = gpu_context(p, max_lm_iters=10)
    rep = ctx.lm_solve()[0]
    assert abs(rep.final_cost - ref.final_cost) <= 1e-3 * ref.final_cost
    out = ctx.get_landmarks()
    assert np.array_equal(out[p.n_points - 2], p.points[p.n_points - 2])
    outc = ctx.get_cameras()
    np.testing.assert_array_equal(outc[p.n_cams - 2, 3:], p.cameras[p.n_cams - 2, 3:])
    ctx.close()


def test_batch_matches_single_problem_runs_bitwise():
    rng = np.random.default_rng(21)
    probs = make_batch(rng, 4, cams=(5, 12), points=(40, 90), k_hi=8)
    batch = concat_problems(probs)
    ctx = gpu_context(batch, max_lm_iters=6)
    reps = ctx.lm_solve()
    cams_b, pts_b = ctx.get_cameras(), ctx.get_landmarks()
    hist_b = [ctx.history(i) for i in range(len(probs))]
    ctx.close()
    for i, p in enumerate(probs):
        c1 = gpu_context(p, max_lm_iters=6)
        r1 = c1.lm_solve()[0]
        h1 = c1.history(0)
        cams1, pts1 = c1.get_cameras(), c1.get_landmarks()
        c1.close()
        assert r1.final_cost == reps[i].final_cost
        assert [h["pcg_iters"] for h in h1] == [h["pcg_iters"] for h in hist_b[i]]
        np.testing.assert_array_equal(cams1, cams_b[batch.cam_off[i]:batch.cam_off[i + 1]])
        np.testing.assert_array_equal(pts1, pts_b[batch.pt_off[i]:batch.pt_off[i + 1]])


def test_batch_final_costs_match_oracle():
    rng = np.random.default_rng(22)
    probs = make_batch(rng, 6, cams=(5, 20), points=(50, 200), k_hi=10)
    batch = concat_problems(probs)
    ctx = gpu_context(batch, max_lm_iters=10)
    reps = ctx.lm_solve()
    ctx.close()
    for p, r in zip(probs, reps):
        ref = oracle.lm_solve(p.cameras, p.points, p.obs_cam, p.obs_pt, p.obs_uv, oracle.LMOptions(max_iters=10))
        assert abs(r.final_cost - ref.final_cost) <= 1e-3 * ref.final_cost, (r.final_cost, ref.final_cost)


def test_workspace_too_small_and_rebinding():
    import torch
    from paper_2103_01843_amd import SqrtBAError
    p = make_config(0)
    with _ctx() as ctx:
        ctx.load(p.cameras, p.points, p.obs_cam, p.obs_pt, p.obs_uv)
        n = ctx.workspace_bytes()
        ws = torch.empty(n, dtype=torch.uint8, device="cuda")
        import ctypes
        from paper_2103_01843_amd.sqrtba import lib
        st = lib().sqrtba_bind_workspace(ctx._h, ctypes.c_void_p(ws.data_ptr()), n - 256)
        assert st == -2
        ctx.bind_torch_workspace()
        c = ctx.linearize()[0]
        assert c > 0
