"""Shared helpers of the GPU tests: contexts from generated problems, oracle views."""

from __future__ import annotations

import numpy as np

import oracle
from bal_synth import Problem, make_ring_problem


def gpu_context(p: Problem, **opts):
    import torch
    from paper_2103_01843_amd import Context

    ctx = Context(stream=torch.cuda.current_stream(), **opts)
    ctx.load(p.cameras, p.points, p.obs_cam, p.obs_pt, p.obs_uv, p.cam_off, p.pt_off)
    ctx.bind_torch_workspace()
    return ctx


def oracle_lin(p: Problem):
    bk = oracle.build_bookkeeping(p.n_cams, p.n_points, p.obs_cam, p.obs_pt, p.obs_uv, p.cam_off, p.pt_off)
    st = oracle.state_from_bal(p.cameras, p.points)
    return bk, st, oracle.linearize(st, bk, p.obs_uv)


def k_mix_sampler(ks):
    ks = np.asarray(ks)

    def f(rng, n):
        return ks[np.arange(n) % len(ks)]

    return f


# observation counts that exercise every landmark size class of the kernels,
# including both ends of each class range
CLASS_EDGES = [2, 3, 4, 7, 8, 14, 15, 28, 29, 60, 113, 114, 150]


def mixed_problem(seed: int = 5, n_cams: int = 160, n_points: int = 260) -> Problem:
    rng = np.random.default_rng(seed)
    return make_ring_problem(rng, n_cams, n_points, k_mix_sampler(CLASS_EDGES), name="mixed")


KCLASS = [(2, 3), (4, 7), (8, 14), (15, 28), (29, 113), (114, 512)]


def sample_landmarks(bk, rng, per_class=4, largest=4):
    """Active landmarks stratified over the kernels' size classes, plus the largest ones."""
    k = np.diff(bk.lm_off)
    act = np.nonzero(bk.lm_active)[0]
    pick = list(act[np.argsort(-k[act], kind="stable")[:largest]])
    for lo, hi in KCLASS:
        cand = act[(k[act] >= lo) & (k[act] <= hi)]
        if len(cand):
            pick += list(rng.choice(cand, min(per_class, len(cand)), replace=False))
    return sorted(set(int(l) for l in pick))


def landmark_sc_contribution(lin, l: int, lam: float):
    """Oracle per-landmark Schur-complement term H_pp,l - H_pl,l (H_ll,l + lam I)^-1 H_lp,l
    (scaled coordinates) and its right-hand side, restricted to the landmark's cameras."""
    idx = np.nonzero(lin.pi == l)[0]
    k = idx.size
    Jp = np.zeros((2 * k, 9 * k))
    for a, o in enumerate(idx):
        Jp[2 * a:2 * a + 2, 9 * a:9 * a + 9] = lin.Jp[o] * lin.sp[lin.ci[o]]
    Jl = (lin.Jl[idx] * lin.sl[l]).reshape(2 * k, 3)
    r = lin.r[idx].reshape(-1)
    Hll = Jl.T @ Jl + lam * np.eye(3)
    Hpl = Jp.T @ Jl
    H = Jp.T @ Jp - Hpl @ np.linalg.solve(Hll, Hpl.T)
    b = Jp.T @ r - Hpl @ np.linalg.solve(Hll, Jl.T @ r)
    return lin.ci[idx], H, b, Jp, Jl, r


def with_extras(p: Problem) -> Problem:
    """Add a camera without observations, a landmark seen once (inactive), and a
    rank-deficient landmark seen only by two cameras with the same centre."""
    cams = np.vstack([p.cameras, p.cameras[0:1] * 1.0, p.cameras[0:1]])  # cam n: unused; cam n+1 = copy of cam 0
    cams[-2, 3:6] += 100.0  # far away, unused
    n = p.n_cams
    X1 = np.array([[0.3, -0.2, 0.1]], np.float32)
    X2 = np.array([[-0.4, 0.5, 0.2]], np.float32)
    pts = np.vstack([p.points, X1, X2]).astype(np.float32)
    oc = np.concatenate([p.obs_cam, [3], [0, n + 1]]).astype(np.int32)
    op = np.concatenate([p.obs_pt, [p.n_points], [p.n_points + 1, p.n_points + 1]]).astype(np.int32)
    uv = np.vstack([p.obs_uv, [[1.0, 2.0]], [[3.0, -4.0], [3.5, -4.5]]]).astype(np.float32)
    return Problem("extras", cams.astype(np.float32), pts, oc, op, uv, p.gt_cameras, p.gt_points)


EPS32 = 2.0 ** -24


def check_precond_blocks(ctx, Bo, slack=None, tol=1e-4):
    """The block-Jacobi pin on every camera: the GPU's damped 9x9 block (L L^T from
    the Cholesky factor it exports with its features) against the oracle's diagonal
    block of H~ to `tol` relative (Frobenius), plus an optional per-block absolute
    slack derived by the caller; and the applied inverse block against the inverse
    of the GPU's own block, to the FP32 bound of a 9x9 Cholesky inverse scaled by
    the block's condition number."""
    _, lf = ctx.debug_features()
    Mi = ctx.debug_precond().astype(np.float64)
    n = Bo.shape[0]
    L = np.zeros((n, 9, 9))
    L[(slice(None),) + np.tril_indices(9)] = lf.astype(np.float64)
    P = L @ L.transpose(0, 2, 1)
    worst = 0.0
    for i in range(n):
        e = np.linalg.norm(P[i] - Bo[i])
        bound = tol * np.linalg.norm(Bo[i]) + (0.0 if slack is None else slack[i])
        assert e <= bound, (i, e / np.linalg.norm(Bo[i]), bound / np.linalg.norm(Bo[i]))
        worst = max(worst, e / np.linalg.norm(Bo[i]))
        kappa = np.linalg.cond(P[i])
        ei = np.linalg.norm(Mi[i] @ P[i] - np.eye(9))
        assert ei <= 200 * EPS32 * kappa, (i, ei, kappa)
    return worst
