"""Levenberg-Marquardt outer loop (FP64), Sec. 6.1.

Settings from Sec. 6.1: initial damping 1e-4, at most 50 iterations, stop
early at a relative function tolerance of 1e-6, CG with at most 500 iterations.
The damping update "by the ratio of actual and expected cost reduction" is
read as Nielsen's rule:
  accept iff rho > 1e-3;
  accept: lambda <- lambda * max(1/3, 1 - (2 rho - 1)^3), nu <- 2;
  reject: lambda <- lambda * nu, nu <- 2 nu;
with lambda clamped to [1e-16, 1e32] (reaching the top ends the solve).
Every attempt, accepted or rejected, counts as one iteration.  After an
accepted step the solve stops if (E_old - E_new) / E_old < func_tol.
The expected reduction is the undamped linear model's, E - |r + J dx|^2.
With a Huber loss (huber_delta, Sec. 6.2) E is the robust cost of
oracle.robust and the linear model is that of the reweighted rows (IRLS).
"""

from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from .bookkeeping import Bookkeeping, build_bookkeeping
from .camera import CameraState, apply_update, bal_from_state, project_residuals, state_from_bal
from .normal_equations import (Linearization, back_substitute, linearize, model_decrease,
                               reduced_camera_system, reduced_system_operator)
from .robust import huber_terms
from .solvers import block_jacobi_blocks, dense_spd_solve, pcg


@dataclass
class LMOptions:
    lambda0: float = 1e-4
    max_iters: int = 50
    func_tol: float = 1e-6
    pcg_tol: float = 1e-6
    pcg_max_iters: int = 500
    pcg_eta: float = 0.0  # > 0: also the Nash-Sofer forcing test of oracle.solvers.pcg
    huber_delta: Optional[float] = None  # Huber loss parameter in pixels (None: squared loss)
    # "pcg": block-Jacobi PCG on the assembled Schur complement; "pcg_operator":
    # the same PCG on the Schur complement applied to vectors (large problems);
    # "dense": Cholesky of the assembled Schur complement
    solver: str = "pcg"
    lambda_min: float = 1e-16
    lambda_max: float = 1e32
    accept_ratio: float = 1e-3


@dataclass
class LMResult:
    state: CameraState
    cost0: float
    final_cost: float
    iterations: int
    status: str
    history: List[dict] = field(default_factory=list)

    @property
    def cameras(self) -> np.ndarray:
        return bal_from_state(self.state)


def cost_of(state: CameraState, bk: Bookkeeping, obs_uv: np.ndarray,
            huber_delta: Optional[float] = None) -> float:
    uv = np.asarray(obs_uv, dtype=np.float64)[bk.obs_perm]
    r = project_residuals(state, bk.ci, bk.pi, uv)
    if huber_delta is None:
        return float(np.sum(r * r))
    return float(np.sum(huber_terms(np.sum(r * r, axis=1), huber_delta)))


def lm_attempt(state: CameraState, bk: Bookkeeping, obs_uv: np.ndarray, lin: Linearization,
               lam: float, opts: LMOptions, trace: bool = False) -> dict:
    """One damped step at fixed linearization: reduce, solve, back-substitute, evaluate."""
    if opts.solver == "pcg_operator":
        rs = reduced_system_operator(lin, lam)
        pres = pcg(rs.matvec, rs.b, rs.blocks, opts.pcg_tol, opts.pcg_max_iters, trace=trace, eta=opts.pcg_eta)
        dxp, iters, rel, status = pres.x, pres.iters, pres.rel_res, pres.status
    elif opts.solver == "dense":
        rs = reduced_camera_system(lin, lam)
        dxp = dense_spd_solve(rs.H, -rs.b)
        iters, rel, status, pres = 0, 0.0, "direct", None
    elif opts.solver == "pcg":
        rs = reduced_camera_system(lin, lam)
        pres = pcg(lambda v: rs.H @ v, rs.b, block_jacobi_blocks(rs.H), opts.pcg_tol,
                   opts.pcg_max_iters, trace=trace, eta=opts.pcg_eta)
        dxp, iters, rel, status = pres.x, pres.iters, pres.rel_res, pres.status
    else:
        raise ValueError(f"unknown solver {opts.solver!r}")
    dxl = back_substitute(rs, dxp)
    pred = model_decrease(lin, dxp, dxl)
    dp = dxp.reshape(lin.n_cams, 9) * lin.sp
    dl = dxl.reshape(lin.n_points, 3) * lin.sl
    new_state = apply_update(state, dp, dl)
    new_cost = cost_of(new_state, bk, obs_uv, opts.huber_delta)
    return {"dxp_scaled": dxp, "dxl_scaled": dxl, "dxp": dp, "dxl": dl, "pred": pred,
            "new_state": new_state, "new_cost": new_cost, "pcg_iters": iters, "rel_res": rel,
            "pcg_status": status, "rs": rs, "pcg": pres}


def lm_solve(cameras: np.ndarray, points: np.ndarray, obs_cam: np.ndarray, obs_pt: np.ndarray,
             obs_uv: np.ndarray, opts: Optional[LMOptions] = None,
             bk: Optional[Bookkeeping] = None, progress=None) -> LMResult:
    """The LM loop; `progress`, if given, is called with each attempt's history record
    and ends the loop (status "stopped") when it returns True."""
    opts = opts or LMOptions()
    if bk is None:
        bk = build_bookkeeping(cameras.shape[0], points.shape[0], obs_cam, obs_pt, obs_uv)
    state = state_from_bal(cameras, points)
    t0 = time.perf_counter()
    lin = linearize(state, bk, obs_uv, opts.huber_delta)
    E = lin.cost
    res = LMResult(state, E, E, 0, "max_iters")
    lam, nu = opts.lambda0, 2.0
    for it in range(opts.max_iters):
        a = lm_attempt(state, bk, obs_uv, lin, lam, opts)
        E_new, pred = a["new_cost"], a["pred"]
        rho = (E - E_new) / pred if pred > 0 else -np.inf
        accepted = bool(np.isfinite(E_new) and rho > opts.accept_ratio)
        res.history.append({"iter": it, "lambda": lam, "cost": E, "new_cost": E_new, "pred": pred,
                            "rho": float(rho), "accepted": accepted, "pcg_iters": a["pcg_iters"],
                            "rel_res": a["rel_res"], "t": time.perf_counter() - t0})
        res.iterations = it + 1
        if progress is not None and progress(res.history[-1]):
            if accepted:
                state, E = a["new_state"], E_new
            res.status = "stopped"
            break
        if accepted:
            rel_dec = (E - E_new) / E
            state, E = a["new_state"], E_new
            lam = lam * max(1.0 / 3.0, 1.0 - (2.0 * rho - 1.0) ** 3)
            nu = 2.0
            lam = min(max(lam, opts.lambda_min), opts.lambda_max)
            if rel_dec < opts.func_tol:
                res.status = "func_tol"
                break
            lin = linearize(state, bk, obs_uv, opts.huber_delta)
        else:
            lam = lam * nu
            nu = 2.0 * nu
            if lam >= opts.lambda_max:
                res.status = "lambda_max"
                break
            lam = max(lam, opts.lambda_min)
    res.state, res.final_cost = state, E
    return res
