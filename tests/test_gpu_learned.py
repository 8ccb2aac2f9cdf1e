"""Learned block preconditioner through the C ABI (GPU) against its FP64 reference.

The paper has no learned component: parity with the paper is unpinned.  The GPU
forward/backward kernels are compared with oracle/mlp.py (FP64, same
bfloat16-rounded weights): loss to 1e-4 and each layer's gradient to 1e-3
relative; the emitted blocks must be SPD and equal block-Jacobi at
initialization; the features must match their definition evaluated on the
oracle's damped reduced system; training must lower the loss; a bad network
must fall back to block-Jacobi and still reach the tolerance.
"""

import numpy as np
import pytest

import oracle
from oracle import mlp
from bal_synth import make_config, make_ring_problem

from gpu_util import gpu_context, oracle_lin

pytestmark = pytest.mark.gpu

LAYERS = [("W1", slice(0, 64 * 128)), ("b1", slice(8192, 8320)), ("W2", slice(8320, 8320 + 16384)),
          ("b2", slice(24704, 24832)), ("W3", slice(24832, 24832 + 10368)), ("b3", slice(35200, 35281))]


def _samples(rng, n):
    x = rng.normal(size=(n, 64)).astype(np.float32)
    A = rng.normal(size=(n, 9, 9))
    P = A @ A.transpose(0, 2, 1) + 9 * np.eye(9)
    L = np.linalg.cholesky(P).astype(np.float32).astype(np.float64)
    packed = np.stack([Li[np.tril_indices(9)] for Li in L]).astype(np.float32)
    p = rng.normal(size=(n, 9)).astype(np.float32)
    q = (np.einsum("nab,nb->na", P, p) + 0.5 * rng.normal(size=(n, 9))).astype(np.float32)
    return x, L, packed, p, q


def test_forward_backward_parity_with_fp64_reference():
    p = make_config(0)
    ctx = gpu_context(p)
    rng = np.random.default_rng(0)
    theta = (mlp.init_params(3) + 0.2 * rng.normal(size=mlp.N_PARAMS)).astype(np.float32)
    ctx.mlp_set_params(theta)
    x, L, packed, pv, qv = _samples(rng, 200)
    loss, grad = ctx.mlp_eval(x, packed, pv, qv)
    th64 = mlp.bf16_round(theta)
    loss_o, grad_o = mlp.loss_and_grad(th64, x.astype(np.float64), L, pv.astype(np.float64), qv.astype(np.float64))
    assert abs(loss - loss_o) <= 1e-4 * abs(loss_o), (loss, loss_o)
    for name, sl in LAYERS:
        e = np.linalg.norm(grad[sl] - grad_o[sl]) / np.linalg.norm(grad_o[sl])
        assert e <= 1e-3, (name, e)
    # round trip of the parameters
    np.testing.assert_array_equal(ctx.mlp_get_params(), theta)
    ctx.close()


def test_blocks_identity_at_init_and_spd():
    p = make_config(0)
    ctx = gpu_context(p)
    ctx.linearize()
    ctx.marginalize()
    ctx.damp(1e-3)
    ctx.mlp_init(7)
    bj = ctx.debug_precond().astype(np.float64)
    le = ctx.debug_learned_precond().astype(np.float64)
    np.testing.assert_allclose(le, bj, rtol=2e-4, atol=2e-4 * np.abs(bj).max())
    rng = np.random.default_rng(1)
    ctx.mlp_set_params((rng.normal(size=mlp.N_PARAMS) * 2.0).astype(np.float32))
    le = ctx.debug_learned_precond().astype(np.float64)
    for m in le:
        assert np.allclose(m, m.T, rtol=1e-4, atol=1e-6 * np.abs(m).max())
        np.linalg.cholesky(0.5 * (m + m.T))
    ctx.close()


def test_features_follow_their_definition():
    p = make_config(0)
    bk, st, lin = oracle_lin(p)
    lam = 1e-3
    ctx = gpu_context(p)
    ctx.linearize()
    ctx.marginalize()
    ctx.damp(lam)
    f, lf = ctx.debug_features()
    rs = oracle.reduced_camera_system(lin, lam)
    for c in range(p.n_cams):
        P = rs.H[9 * c:9 * c + 9, 9 * c:9 * c + 9]
        d = np.diag(P)
        np.testing.assert_allclose(f[c, :9], np.log(d), atol=2e-4)
        corr = (P / np.sqrt(np.outer(d, d)))[np.triu_indices(9, 1)]
        np.testing.assert_allclose(f[c, 9:45], corr, atol=2e-4)
        np.testing.assert_allclose(f[c, 45:54], np.log(lam / d), atol=2e-4)
        assert abs(f[c, 54] - np.log(lam)) < 1e-5
        n_obs = np.sum(bk.ci == c)
        assert abs(f[c, 55] - np.log1p(n_obs)) < 1e-5
        L = np.zeros((9, 9))
        L[np.tril_indices(9)] = lf[c]
        np.testing.assert_allclose(L @ L.T, P, rtol=1e-4, atol=1e-4 * np.abs(P).max())
    ctx.close()


def test_training_lowers_loss_and_learned_solve_reaches_tolerance():
    rng = np.random.default_rng(5)
    p = make_ring_problem(rng, 30, 1500, lambda r, n: r.integers(2, 12, size=n))
    ctx = gpu_context(p, max_lm_iters=4)
    ctx.mlp_init(0)
    ctx.pcg_trace(8, 64)
    ctx.lm_solve()
    ns, nr = ctx.trace_size()
    assert ns > 0 and nr > 0
    # the loss on one fixed seeded batch (lr = 0 evaluates only) goes down
    before = ctx.mlp_train(1, batch=16384, lr=0.0, seed=99)[0]
    np.testing.assert_array_equal(ctx.mlp_train(1, batch=16384, lr=0.0, seed=99), [before])
    ctx.mlp_train(200, batch=1024, lr=5e-3, seed=1)
    after = ctx.mlp_train(1, batch=16384, lr=0.0, seed=99)[0]
    assert after < before, (before, after)
    ctx.pcg_trace(0, 0)
    # the learned mode reaches the same tolerance and final cost (fallback guarantees it)
    plain = gpu_context(p, max_lm_iters=4).lm_solve()[0]
    ctx2 = gpu_context(p, max_lm_iters=4)
    ctx2.mlp_set_params(ctx.mlp_get_params())
    ctx2.set_preconditioner("learned")
    rep = ctx2.lm_solve()[0]
    assert abs(rep.final_cost - plain.final_cost) <= 1e-3 * plain.final_cost
    assert all(h["pcg_status"] == "converged" for h in ctx2.history(0))
    ctx.close()
    ctx2.close()


def test_trained_network_gain_on_a_held_out_problem():
    """What the trained network gains over block-Jacobi, measured: trained online on
    the solver's own PCG traces of one ladybug-shaped problem, then an LM solve of a
    held-out one (another seed) with the learned blocks and with block-Jacobi, at the
    same unpreconditioned tolerance.  Measured: no gain -- the learned solve takes
    about as many PCG iterations as the plain one (within 10%; the fallback bounds a
    bad network) and reaches the same final cost (1e-3).  The CPU test
    test_block_preconditioner_bound.py shows why no 9x9 block-diagonal network can
    gain here: block-Jacobi minimizes Kaporin's condition number over such
    preconditioners, and blocks fitted freely through unrolled PCG iterations need
    no fewer iterations on right-hand sides they were not fitted to."""
    from bal_synth import make_forward_problem
    train = make_forward_problem(np.random.default_rng(301), 60, 6000, 20)
    held = make_forward_problem(np.random.default_rng(302), 60, 6000, 20)
    ctx = gpu_context(train, max_lm_iters=8)
    ctx.mlp_init(0)
    ctx.pcg_trace(8, 64)
    ctx.lm_solve()
    losses = [float(np.mean(ctx.mlp_train(50, batch=2048, lr=1e-3, seed=s))) for s in range(4)]
    theta = ctx.mlp_get_params()
    ctx.close()
    plain_ctx = gpu_context(held, max_lm_iters=8)
    plain = plain_ctx.lm_solve()[0]
    plain_ctx.close()
    lctx = gpu_context(held, max_lm_iters=8)
    lctx.mlp_set_params(theta)
    lctx.set_preconditioner("learned")
    learned = lctx.lm_solve()[0]
    stats = lctx.learned_stats()
    lctx.close()
    gain = plain.total_pcg_iters / learned.total_pcg_iters - 1.0
    print(f"training loss {losses[0]:.4f} -> {losses[-1]:.4f}; PCG iterations plain {plain.total_pcg_iters}, "
          f"learned {learned.total_pcg_iters} (gain {100 * gain:+.1f}%), fallbacks {stats['fallbacks']}; final cost "
          f"plain {plain.final_cost:.8g}, learned {learned.final_cost:.8g}", flush=True)
    assert losses[-1] < losses[0]
    assert abs(learned.final_cost - plain.final_cost) <= 1e-3 * plain.final_cost
    assert learned.total_pcg_iters <= 1.10 * plain.total_pcg_iters


def test_bad_network_falls_back_to_block_jacobi():
    p = make_config(0)
    ctx = gpu_context(p)
    ctx.linearize()
    ctx.marginalize()
    ctx.damp(1e-4)
    its_plain, rel_plain, st_plain = ctx.solve()
    dx_plain, _ = ctx.debug_solution()
    rng = np.random.default_rng(2)
    theta = np.zeros(mlp.N_PARAMS, np.float32)
    theta[24832:24832 + 10368] = rng.normal(size=10368) * 50.0  # saturated, erratic corrections
    theta[:8192] = rng.normal(size=8192)
    ctx.mlp_set_params(theta)
    ctx.set_preconditioner("learned")
    its, rel, st = ctx.solve()
    stats = ctx.learned_stats()
    assert st[0] == 0 and rel[0] <= 1e-6
    if stats["fallbacks"]:
        # after the fallback the solve is the plain one
        assert its[0] == its_plain[0]
        dx, _ = ctx.debug_solution()
        np.testing.assert_array_equal(dx, dx_plain)
    ctx.close()


def test_batch_fallback_keeps_the_other_problems_outcome():
    """A batch in learned mode where one problem falls back to block-Jacobi: the
    other problems keep the outcome of their learned solve (converged, with their
    own iteration count), and the fallback problem converges with plain blocks.
    Set-up: the untrained network emits exactly block-Jacobi (last layer zero),
    so the easy problem's learned solve equals its plain one; the hard problem's
    last plain solve is recorded under a 3-iteration limit, so the learned cap
    (1.5 x the largest last plain count) is set by the easy problem and the hard
    problem cannot reach the tolerance within it."""
    from bal_synth import concat_problems, make_forward_problem
    easy = make_ring_problem(np.random.default_rng(41), 6, 60, lambda r, n: r.integers(2, 6, size=n))
    hard = make_forward_problem(np.random.default_rng(42), 40, 2000, 20)
    batch = concat_problems([easy, hard])
    ctx = gpu_context(batch)
    ctx.mlp_init(0)
    ctx.linearize()
    ctx.marginalize()
    ctx.damp(1e-4)
    ctx.set_active([1, 0])
    its_plain, _, st_plain = ctx.solve()
    assert st_plain[0] == 0
    ctx.set_active([0, 1])
    ctx.set_options(pcg_max_iters=3)
    ctx.solve()
    ctx.set_options(pcg_max_iters=500)
    ctx.set_active([1, 1])
    ctx.set_preconditioner("learned")
    its, rel, st = ctx.solve()
    stats = ctx.learned_stats()
    ctx.close()
    assert stats["fallbacks"] == 1, stats
    assert st[0] == 0 and abs(int(its[0]) - int(its_plain[0])) <= 2 and 0 < rel[0] <= 1e-6, (st, its, rel, its_plain)
    assert st[1] == 0 and its[1] > 1.5 * its_plain[0] and 0 < rel[1] <= 1e-6, (st, its, rel)
