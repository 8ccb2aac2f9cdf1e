"""Pins of the oracle's Huber loss and its IRLS reweighting (Sec. 6.2).

* the cost terms against their closed form on both sides of delta^2, their
  continuity there, and the weight as their derivative (central differences);
* the gradient of the reweighted problem at a linearization point,
  2 sum_o J_wo^T r_wo, against central differences of the robust energy
  sum_o rho(|r_o|^2) over the state (a wrong weight power, a wrong branch or a
  missing factor fails it);
* a delta above every residual gives back the plain linearization exactly;
* the Huber LM decreases the robust cost on every accepted step, and with a
  few gross outliers planted in the pixels it stays closer to the clean
  problem's solution than the squared loss does.
"""

import numpy as np

import oracle
from oracle.lm import cost_of
from bal_synth import make_config


def test_huber_terms_closed_form_and_derivative():
    delta = 1.5
    s = np.array([0.0, 0.3, 2.25, 2.2500001, 4.0, 100.0])
    rho = oracle.huber_terms(s, delta)
    expect = np.where(s <= delta ** 2, s, 2 * delta * np.sqrt(s) - delta ** 2)
    np.testing.assert_array_equal(rho, expect)
    np.testing.assert_allclose(oracle.huber_terms(np.array([100.0]), delta), 2 * 1.5 * 10 - 2.25)
    # continuous at delta^2, never above the squared loss
    lo, hi = oracle.huber_terms(np.array([delta ** 2 * (1 - 1e-12), delta ** 2 * (1 + 1e-12)]), delta)
    assert abs(lo - hi) < 1e-9
    grid = np.linspace(0, 50, 2001)
    assert np.all(oracle.huber_terms(grid, delta) <= grid + 1e-15)
    # the weight is rho'(s), away from the kink
    pts = np.array([0.5, 1.0, 2.0, 3.0, 9.0, 40.0])
    h = 1e-6
    fd = (oracle.huber_terms(pts + h, delta) - oracle.huber_terms(pts - h, delta)) / (2 * h)
    np.testing.assert_allclose(oracle.huber_weights(pts, delta), fd, rtol=1e-7)


def _full_gradient(lin):
    """2 J^T r over (9 per camera, 3 per landmark), unscaled, from the reweighted rows."""
    gp = np.zeros((lin.n_cams, 9))
    gl = np.zeros((lin.n_points, 3))
    np.add.at(gp, lin.ci, 2 * np.einsum("nij,ni->nj", lin.Jp, lin.r))
    np.add.at(gl, lin.pi, 2 * np.einsum("nij,ni->nj", lin.Jl, lin.r))
    return gp, gl


def test_irls_gradient_equals_robust_energy_gradient():
    p = make_config(0)
    bk = oracle.build_bookkeeping(p.n_cams, p.n_points, p.obs_cam, p.obs_pt, p.obs_uv)
    st = oracle.state_from_bal(p.cameras, p.points)
    r0 = oracle.linearize(st, bk, p.obs_uv)
    delta = float(np.median(np.linalg.norm(r0.r, axis=1)))  # about half the observations beyond delta
    lin = oracle.linearize(st, bk, p.obs_uv, huber_delta=delta)
    s = np.sum(r0.r ** 2, axis=1)
    assert 0.3 < np.mean(s > delta ** 2) < 0.7
    assert abs(lin.cost - cost_of(st, bk, p.obs_uv, delta)) <= 1e-12 * lin.cost
    gp, gl = _full_gradient(lin)
    rng = np.random.default_rng(3)
    h = 1e-6
    for _ in range(24):
        dp = np.zeros((p.n_cams, 9))
        dl = np.zeros((p.n_points, 3))
        if rng.random() < 0.5:
            c, j = rng.integers(p.n_cams), rng.integers(9)
            dp[c, j] = h
            g = gp[c, j]
        else:
            l, j = rng.choice(np.nonzero(bk.lm_active)[0]), rng.integers(3)
            dl[l, j] = h
            g = gl[l, j]
        ep = cost_of(oracle.apply_update(st, dp, dl), bk, p.obs_uv, delta)
        em = cost_of(oracle.apply_update(st, -dp, -dl), bk, p.obs_uv, delta)
        fd = (ep - em) / (2 * h)
        assert abs(fd - g) <= 1e-5 * max(abs(g), 1e-3 * np.abs(gp).max()), (fd, g)


def test_delta_above_every_residual_is_the_plain_linearization():
    p = make_config(0)
    bk = oracle.build_bookkeeping(p.n_cams, p.n_points, p.obs_cam, p.obs_pt, p.obs_uv)
    st = oracle.state_from_bal(p.cameras, p.points)
    a = oracle.linearize(st, bk, p.obs_uv)
    b = oracle.linearize(st, bk, p.obs_uv, huber_delta=1e6)
    for f in ("r", "Jp", "Jl", "sp", "sl"):
        np.testing.assert_array_equal(getattr(a, f), getattr(b, f))
    assert a.cost == b.cost


def test_huber_lm_is_monotone_and_robust_to_outliers():
    p = make_config(0)
    bk = oracle.build_bookkeeping(p.n_cams, p.n_points, p.obs_cam, p.obs_pt, p.obs_uv)
    clean = oracle.lm_solve(p.cameras, p.points, p.obs_cam, p.obs_pt, p.obs_uv,
                            oracle.LMOptions(max_iters=15, solver="dense"), bk=bk)
    rng = np.random.default_rng(4)
    uv = p.obs_uv.copy()
    bad = rng.choice(len(uv), len(uv) // 50, replace=False)
    uv[bad] += rng.choice([-1.0, 1.0], size=(len(bad), 2)) * 40.0  # 40 px gross outliers
    runs = {}
    for name, delta in (("squared", None), ("huber", 1.0)):
        res = oracle.lm_solve(p.cameras, p.points, p.obs_cam, p.obs_pt, uv,
                              oracle.LMOptions(max_iters=15, solver="dense", huber_delta=delta), bk=bk)
        acc = [h for h in res.history if h["accepted"]]
        assert acc and all(h["new_cost"] < h["cost"] for h in acc)
        runs[name] = res
    # distance of the 2D projections of the clean solution's landmarks to each run's
    # (predicted pixels are invariant under the gauge, so the runs compare directly)
    rc = oracle.project_residuals(clean.state, bk.ci, bk.pi, np.zeros((len(bk.ci), 2)))
    err = {}
    for name, res in runs.items():
        ro = oracle.project_residuals(res.state, bk.ci, bk.pi, np.zeros((len(bk.ci), 2)))
        err[name] = float(np.sqrt(np.mean(np.sum((ro - rc) ** 2, axis=1))))
    assert err["huber"] < 0.5 * err["squared"], err
