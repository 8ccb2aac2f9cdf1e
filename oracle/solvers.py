"""Linear solvers for the reduced camera system (FP64).

Sec. 5.4: the reduced system is solved with conjugate gradients on the normal
equations, preconditioned with the 9x9 block diagonal of the damped reduced
matrix (block-Jacobi, the preconditioner Ceres uses as well, Sec. 6.1).  The
CG limits are at most 500 iterations and no minimum (Sec. 6.1).  The stopping
rule read here is on the unpreconditioned recurrence residual,
|r_k| / |r_0| <= tol, starting from x_0 = 0.  A dense Cholesky solve serves
tiny problems (the paper mentions direct solves for small systems, Sec. 5.4).
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np
import scipy.linalg as sla


def dense_spd_solve(H: np.ndarray, rhs: np.ndarray) -> np.ndarray:
    c = sla.cho_factor(H, lower=True)
    return sla.cho_solve(c, rhs)


def block_jacobi_blocks(H: np.ndarray, bs: int = 9) -> np.ndarray:
    n = H.shape[0] // bs
    return np.stack([H[bs * i: bs * i + bs, bs * i: bs * i + bs] for i in range(n)])


@dataclass
class PCGResult:
    x: np.ndarray
    iters: int
    rel_res: float
    status: str  # "converged", "max_iters", "breakdown", "zero_rhs"
    trace_p: List[np.ndarray] = field(default_factory=list)
    trace_q: List[np.ndarray] = field(default_factory=list)


def quadratic_model(matvec: Callable[[np.ndarray], np.ndarray], b: np.ndarray, x: np.ndarray) -> float:
    """Q(x) = 1/2 x^T A x + b^T x, the quadratic whose minimizer solves A x = -b (Q(0) = 0)."""
    return float(0.5 * (x @ matvec(x)) + b @ x)


def pcg(matvec: Callable[[np.ndarray], np.ndarray], b: np.ndarray, blocks: Optional[np.ndarray],
        tol: float = 1e-6, max_iters: int = 500, trace: bool = False, eta: float = 0.0) -> PCGResult:
    """Solve A x = -b with block-Jacobi PCG from x_0 = 0 (blocks: (n, bs, bs) or None).

    Stops when |r_k| <= tol |r_0| (recurrence residual) or after max_iters.  With
    eta > 0 it also stops at the first iteration i >= 1 with
    i (Q_i - Q_{i-1}) / Q_i < eta, Q the quadratic model evaluated directly at the
    iterates: the truncated-Newton test of Nash and Sofer (1990), which the paper
    uses through its "same forcing sequence as Ceres" (Sec. 6.1)."""
    n = b.shape[0]
    if blocks is not None:
        bs = blocks.shape[1]
        chol = [sla.cho_factor(B, lower=True) for B in blocks]

        def prec(v):
            return np.concatenate([sla.cho_solve(c, v[bs * i: bs * i + bs]) for i, c in enumerate(chol)])
    else:
        def prec(v):
            return v.copy()

    x = np.zeros(n)
    r = -b.astype(np.float64).copy()
    r0 = float(np.linalg.norm(r))
    res = PCGResult(x, 0, 0.0, "zero_rhs")
    if r0 == 0.0:
        return res
    z = prec(r)
    p = z.copy()
    rz = float(r @ z)
    status = "max_iters"
    k = 0
    rn = r0
    q_prev = 0.0  # Q(x_0) = 0
    while k < max_iters:
        q = matvec(p)
        pq = float(p @ q)
        if not np.isfinite(pq) or pq <= 0.0:
            status = "breakdown"
            break
        if trace:
            res.trace_p.append(p.copy())
            res.trace_q.append(q.copy())
        alpha = rz / pq
        x = x + alpha * p
        r = r - alpha * q
        k += 1
        rn = float(np.linalg.norm(r))
        if rn <= tol * r0:
            status = "converged"
            break
        if eta > 0.0:
            q_cur = quadratic_model(matvec, b, x)
            if q_cur < 0.0 and k * (q_cur - q_prev) / q_cur < eta:
                status = "converged"
                break
            q_prev = q_cur
        z = prec(r)
        rz_new = float(r @ z)
        beta = rz_new / rz
        p = z + beta * p
        rz = rz_new
    res.x, res.iters, res.rel_res, res.status = x, k, rn / r0, status
    return res
