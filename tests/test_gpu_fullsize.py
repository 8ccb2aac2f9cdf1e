"""Parity at the full workload sizes, in the launch configuration bench.py times.

The oracle cannot form the whole reduced system of the large workloads in
seconds, so at full size the GPU path is checked on outputs the oracle computes
one at a time, and on properties that hold at any size:

* sampled landmark blocks (stratified over the size classes, plus the largest
  landmarks): S B^T B S and S B^T rho against the oracle's per-landmark Schur
  terms (eq. red_H / red_b), R^T R against R1^T R1 + lambda I;
* the product: symmetric and positive definite on seeded random vectors, and
  equal (to rounding) under the default and the autotuned launch shapes; for the
  ladybug-like workload also against the oracle's explicit reduced system;
* the LM solve (20 attempts, as benchmarked): the GPU's final cost equals the
  oracle's cost function at the GPU's final state (1e-5), and for the
  ladybug-like workload the oracle's own final cost (1e-3, stored fixture).

The ladybug-like and venice-like workloads run by default; the batch of 256
and the dense-stress workload (210 GB of HBM) run when SQRTBA_FULLSIZE_ALL=1.
"""

import json
import os

import numpy as np
import pytest

import oracle
from oracle.lm import cost_of
from bal_synth import make_config

from gpu_util import gpu_context, landmark_sc_contribution, oracle_lin, sample_landmarks

pytestmark = pytest.mark.gpu

CONFIGS = [1, 3] + ([2, 4] if os.environ.get("SQRTBA_FULLSIZE_ALL") == "1" else [])
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "oracle_lm_config{}.json")


@pytest.fixture(scope="module", params=CONFIGS)
def full(request):
    cfg = request.param
    p = make_config(cfg)
    bk, st, lin = oracle_lin(p)
    ctx = gpu_context(p, max_lm_iters=20)
    best, _ = ctx.autotune(reps=3)
    print(f"config {cfg}: autotuned shapes {best}", flush=True)
    yield cfg, p, bk, lin, ctx
    ctx.close()


def test_sampled_landmark_blocks(full):
    cfg, p, bk, lin, ctx = full
    lam = 1e-4
    ctx.linearize()
    ctx.marginalize()
    ctx.damp(lam)
    sc, _ = ctx.debug_scales()
    worst = 0.0
    for l in sample_landmarks(bk, np.random.default_rng(cfg)):
        cams, H, b, Jp, Jl, r = landmark_sc_contribution(lin, l, lam)
        k, blk, fac = ctx.debug_block(l)
        assert k == len(cams)
        s = np.concatenate([sc[c] for c in cams]).astype(np.float64)
        B = blk[3:, :9 * k].astype(np.float64) * s[None, :]
        rho = blk[3:, 9 * k + 3].astype(np.float64)
        eH = np.linalg.norm(B.T @ B - H) / max(np.linalg.norm(H), 1e-30)
        tol_b = 1e-4 * np.linalg.norm(b) + 64 * 2.0 ** -24 * np.linalg.norm(Jp, 2) * np.linalg.norm(r)
        eb = 1e-4 * np.linalg.norm(B.T @ rho - b) / tol_b
        worst = max(worst, eH, eb)
        Rh = np.zeros((3, 3))
        Rh[np.triu_indices(3)] = fac[9:15]
        np.testing.assert_allclose(Rh.T @ Rh, Jl.T @ Jl + lam * np.eye(3), atol=2e-5 * (1 + lam) * max(1.0, np.abs(Jl.T @ Jl).max()))
    assert worst < 1e-4, worst


def test_product_properties(full):
    cfg, p, bk, lin, ctx = full
    lam = 1e-4
    ctx.linearize()
    ctx.marginalize()
    ctx.damp(lam)
    n = 9 * p.n_cams
    rng = np.random.default_rng(100 + cfg)
    V = rng.normal(size=(2, n)).astype(np.float32)
    AV = ctx.debug_rcs_matvec(V).astype(np.float64)
    v, w = V.astype(np.float64)
    Av, Aw = AV
    # symmetric and positive definite (damped, so v^T A v >= lambda |v|^2)
    scale = np.linalg.norm(v) * np.linalg.norm(Aw) + np.linalg.norm(w) * np.linalg.norm(Av)
    assert abs(v @ Aw - w @ Av) <= 1e-5 * scale
    assert v @ Av >= lam * (v @ v) * (1 - 1e-4) and w @ Aw >= lam * (w @ w) * (1 - 1e-4)
    # the autotuned shapes against the default ones
    tuned = ctx.get_tuning()
    ctx.set_tuning(rows_min_k=114, huge_rows=64, huge_side=0, large_separate=0, small_rows=4, persist_wgs=0)
    AV0 = ctx.debug_rcs_matvec(V).astype(np.float64)
    ctx.set_tuning(**tuned)
    assert np.linalg.norm(AV - AV0) <= 1e-5 * np.linalg.norm(AV0)
    if cfg == 1:
        rs = oracle.reduced_camera_system(lin, lam)
        Ho = rs.H @ V.T.astype(np.float64)
        assert np.linalg.norm(AV.T - Ho) <= 1e-4 * np.linalg.norm(Ho)


def test_lm_final_cost(full):
    cfg, p, bk, lin, ctx = full
    rep = ctx.lm_solve()
    cams, pts = ctx.get_cameras(), ctx.get_landmarks()
    for i in range(p.n_problems):
        assert np.isfinite(rep[i].final_cost) and rep[i].final_cost < rep[i].initial_cost
    c = cost_of(oracle.state_from_bal(cams, pts), bk, p.obs_uv)
    total = sum(r.final_cost for r in rep)
    assert abs(c - total) <= 1e-5 * total, (c, total)
    if os.path.exists(GOLDEN.format(cfg)) and p.n_problems == 1:
        with open(GOLDEN.format(cfg)) as f:
            gold = json.load(f)
        assert abs(total - gold["final_cost"]) <= 1e-3 * gold["final_cost"], (total, gold["final_cost"])
