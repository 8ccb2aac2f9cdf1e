"""Damped normal equations and their explicit Schur complement (FP64).

The linearized, damped least-squares problem is Sec. 4.1, eq.
linearized_residual: minimize |r + J_p dx_p + J_l dx_l|^2 + lambda |D_p dx_p|^2
+ lambda |D_l dx_l|^2.  Its normal equations are eq. normal_eq with the blocks
H_pp = J_p^T J_p, H_pl = J_p^T J_l, H_ll = J_l^T J_l, b_p = J_p^T r,
b_l = J_l^T r (plus lambda D^2 on the diagonal).  The Schur complement
(Sec. 4.2, eq. red_normal_eq) is
    H~ = H_pp - H_pl H_ll^-1 H_lp,   b~ = b_p - H_pl H_ll^-1 b_l,
solved as H~ (-dx_p) = b~, followed by the back-substitution eq. backsub_sc,
    -dx_l = H_ll^-1 (b_l - H_lp (-dx_p)).
By Sec. 4.4 (eq. red_H, red_b, and the closing remark on the damped problem)
this is exactly the reduced camera system that nullspace marginalization
produces, so it is the reference for the GPU path.

With a Huber loss (Sec. 6.2, oracle.robust) the residual and Jacobian rows of
each observation are reweighted by sqrt(rho'(|r_o|^2)) at the linearization
point (IRLS) and the cost is sum_o rho(|r_o|^2); everything below then works on
the reweighted rows.

Column scaling (Sec. 5.4): every column of the full Jacobian is scaled to
unit norm, J~ = J S with s_c = 1 / |J_c| (a zero column keeps s_c = 1).  The
damping matrix is D^2 = diag(J~^T J~) (Sec. 4.1), which is the identity after
scaling, so D_p = D_l = I in scaled coordinates and dx = S dx~.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from typing import Optional

from .bookkeeping import Bookkeeping
from .camera import CameraState, linearize_observations
from .robust import huber_terms, huber_weights


@dataclass
class Linearization:
    r: np.ndarray  # (n, 2)
    Jp: np.ndarray  # (n, 2, 9) unscaled
    Jl: np.ndarray  # (n, 2, 3) unscaled
    ci: np.ndarray  # (n,)
    pi: np.ndarray  # (n,)
    n_cams: int
    n_points: int
    cost: float
    sp: np.ndarray  # (n_cams, 9) column scales
    sl: np.ndarray  # (n_points, 3)


def column_scales(Jp: np.ndarray, Jl: np.ndarray, ci: np.ndarray, pi: np.ndarray,
                  n_cams: int, n_points: int):
    """s_c = 1 / |J_c| over all rows of the full Jacobian; empty columns get 1."""
    cp = np.zeros((n_cams, 9))
    np.add.at(cp, ci, np.sum(Jp * Jp, axis=1))
    cl = np.zeros((n_points, 3))
    np.add.at(cl, pi, np.sum(Jl * Jl, axis=1))
    sp_ = np.where(cp > 0, 1.0 / np.sqrt(np.where(cp > 0, cp, 1.0)), 1.0)
    sl_ = np.where(cl > 0, 1.0 / np.sqrt(np.where(cl > 0, cl, 1.0)), 1.0)
    return sp_, sl_


def linearize(state: CameraState, bk: Bookkeeping, obs_uv: np.ndarray,
              huber_delta: Optional[float] = None) -> Linearization:
    uv = np.asarray(obs_uv, dtype=np.float64)[bk.obs_perm]
    r, Jp, Jl = linearize_observations(state, bk.ci, bk.pi, uv)
    if huber_delta is None:
        cost = float(np.sum(r * r))
    else:
        s = np.sum(r * r, axis=1)
        cost = float(np.sum(huber_terms(s, huber_delta)))
        sw = np.sqrt(huber_weights(s, huber_delta))
        r, Jp, Jl = r * sw[:, None], Jp * sw[:, None, None], Jl * sw[:, None, None]
    sp_, sl_ = column_scales(Jp, Jl, bk.ci, bk.pi, bk.n_cams, bk.n_points)
    return Linearization(r, Jp, Jl, bk.ci, bk.pi, bk.n_cams, bk.n_points, cost, sp_, sl_)


def scaled_jacobian_sparse(lin: Linearization):
    """J~_p (2n x 9 n_cams) and J~_l (2n x 3 n_points) as CSR matrices, and r (2n)."""
    n = lin.r.shape[0]
    rows = np.arange(2 * n).reshape(n, 2)
    Jps = lin.Jp * lin.sp[lin.ci][:, None, :]
    Jls = lin.Jl * lin.sl[lin.pi][:, None, :]
    rp = np.repeat(rows[:, :, None], 9, axis=2)
    cp = np.broadcast_to((9 * lin.ci)[:, None, None] + np.arange(9)[None, None, :], (n, 2, 9))
    Jp_m = sp.csr_matrix((Jps.ravel(), (rp.ravel(), cp.ravel())), shape=(2 * n, 9 * lin.n_cams))
    rl = np.repeat(rows[:, :, None], 3, axis=2)
    cl = np.broadcast_to((3 * lin.pi)[:, None, None] + np.arange(3)[None, None, :], (n, 2, 3))
    Jl_m = sp.csr_matrix((Jls.ravel(), (rl.ravel(), cl.ravel())), shape=(2 * n, 3 * lin.n_points))
    return Jp_m, Jl_m, lin.r.ravel().copy()


@dataclass
class ReducedSystem:
    H: np.ndarray  # (9 n_cams, 9 n_cams) dense, damped
    b: np.ndarray  # (9 n_cams,)
    lam: float
    # pieces kept for the back-substitution
    Hll_inv: sp.csr_matrix
    Hpl: sp.csr_matrix
    bl: np.ndarray


def reduced_camera_system(lin: Linearization, lam: float) -> ReducedSystem:
    """Explicit Schur complement of the damped, scaled normal equations (D = I)."""
    Jp_m, Jl_m, r = scaled_jacobian_sparse(lin)
    Hpp = (Jp_m.T @ Jp_m).toarray() + lam * np.eye(9 * lin.n_cams)
    Hpl = (Jp_m.T @ Jl_m).tocsr()
    bp = Jp_m.T @ r
    bl = Jl_m.T @ r
    # H_ll is block diagonal with 3x3 blocks; invert block by block
    Jls = lin.Jl * lin.sl[lin.pi][:, None, :]
    Hll = np.zeros((lin.n_points, 3, 3))
    np.add.at(Hll, lin.pi, np.einsum("nki,nkj->nij", Jls, Jls))
    Hll += lam * np.eye(3)[None]
    used = np.zeros(lin.n_points, dtype=bool)
    used[lin.pi] = True
    Hll[~used] = np.eye(3)  # landmarks without rows: their columns are empty
    inv = np.linalg.inv(Hll)
    inv[~used] = 0.0
    ii = (3 * np.arange(lin.n_points))[:, None, None] + np.arange(3)[None, :, None]
    jj = (3 * np.arange(lin.n_points))[:, None, None] + np.arange(3)[None, None, :]
    Hll_inv = sp.csr_matrix((inv.ravel(), (np.broadcast_to(ii, inv.shape).ravel(),
                                          np.broadcast_to(jj, inv.shape).ravel())),
                            shape=(3 * lin.n_points, 3 * lin.n_points))
    W = (Hpl @ Hll_inv).tocsr()
    H = Hpp - (W @ Hpl.T).toarray()
    b = bp - W @ bl
    return ReducedSystem(H, b, lam, Hll_inv, Hpl, bl)


def _sum_by(index: np.ndarray, values: np.ndarray, n: int) -> np.ndarray:
    """out[i] = sum of values[o] over all rows o with index[o] == i (values: (m, d))."""
    return np.stack([np.bincount(index, weights=values[:, j], minlength=n) for j in range(values.shape[1])],
                    axis=1)


def _chunks(n: int, size: int = 1 << 18):
    """Observation ranges of at most `size` rows (keeps temporaries small)."""
    return [(s, min(s + size, n)) for s in range(0, n, size)]


@dataclass
class ReducedOperator:
    """The damped reduced camera system of `reduced_camera_system`, applied to
    vectors instead of assembled (Sec. 4.2, eq. red_normal_eq):

        H~ v = (H_pp + lam I) v - H_pl (H_ll + lam I)^-1 H_lp v,

    with every product formed from the per-observation rows of the scaled
    Jacobian, so it needs O(#observations) memory.  b, the diagonal 9x9 blocks
    of H~ (the block-Jacobi preconditioner) and the back-substitution follow the
    same definitions.  For the large workloads, where the dense matrix of
    `reduced_camera_system` does not fit the CPU's memory or time."""
    lam: float
    n_cams: int
    n_points: int
    ci: np.ndarray
    pi: np.ndarray
    Jps: np.ndarray  # (n, 2, 9) scaled pose rows
    Jls: np.ndarray  # (n, 2, 3) scaled landmark rows
    Hll_inv: np.ndarray  # (n_points, 3, 3) (H_ll,l + lam I)^-1, zero for landmarks without rows
    bl: np.ndarray  # (n_points, 3)
    b: np.ndarray  # (9 n_cams,)
    blocks: np.ndarray  # (n_cams, 9, 9) diagonal blocks of H~

    def lp(self, v: np.ndarray) -> np.ndarray:
        """H_lp v as (n_points, 3)."""
        u = np.einsum("nij,nj->ni", self.Jps, v.reshape(self.n_cams, 9)[self.ci])  # J_p v per observation
        return _sum_by(self.pi, np.einsum("nki,nk->ni", self.Jls, u), self.n_points)

    def matvec(self, v: np.ndarray) -> np.ndarray:
        V = v.reshape(self.n_cams, 9)
        u = np.einsum("nij,nj->ni", self.Jps, V[self.ci])  # J_p v per observation
        hl = _sum_by(self.pi, np.einsum("nki,nk->ni", self.Jls, u), self.n_points)  # H_lp v
        w = np.einsum("lij,lj->li", self.Hll_inv, hl)  # (H_ll + lam I)^-1 H_lp v
        t = u - np.einsum("nij,nj->ni", self.Jls, w[self.pi])  # J_p v - J_l w per observation
        out = _sum_by(self.ci, np.einsum("nki,nk->ni", self.Jps, t), self.n_cams)  # J_p^T (...)
        return (out + self.lam * V).reshape(-1)


def reduced_system_operator(lin: Linearization, lam: float) -> ReducedOperator:
    """`reduced_camera_system` as an operator (see ReducedOperator)."""
    Jps = lin.Jp * lin.sp[lin.ci][:, None, :]
    Jls = lin.Jl * lin.sl[lin.pi][:, None, :]
    n = lin.ci.shape[0]
    Hll = np.zeros((lin.n_points, 9))
    bl = np.zeros((lin.n_points, 3))
    bp = np.zeros((lin.n_cams, 9))
    for s, e in _chunks(n):
        Hll += _sum_by(lin.pi[s:e], np.einsum("nki,nkj->nij", Jls[s:e], Jls[s:e]).reshape(-1, 9), lin.n_points)
        bl += _sum_by(lin.pi[s:e], np.einsum("nki,nk->ni", Jls[s:e], lin.r[s:e]), lin.n_points)
        bp += _sum_by(lin.ci[s:e], np.einsum("nki,nk->ni", Jps[s:e], lin.r[s:e]), lin.n_cams)
    Hll = Hll.reshape(-1, 3, 3) + lam * np.eye(3)[None]
    used = np.zeros(lin.n_points, dtype=bool)
    used[lin.pi] = True
    Hll[~used] = np.eye(3)
    inv = np.linalg.inv(Hll)
    inv[~used] = 0.0
    w = np.einsum("lij,lj->li", inv, bl)
    # b~ = b_p - H_pl w; diagonal blocks: per observation J_p^T J_p - G (H_ll + lam I)^-1 G^T, G = J_p^T J_l
    b = bp
    blocks = np.zeros((lin.n_cams, 81))
    for s, e in _chunks(n, 1 << 15):  # (m, 9, 9) temporaries of a few MB
        A, L = Jps[s:e], Jls[s:e]
        b -= _sum_by(lin.ci[s:e], np.einsum("nki,nk->ni", A, np.einsum("nij,nj->ni", L, w[lin.pi[s:e]])), lin.n_cams)
        # per observation (two rows): J_p^T J_p, G = J_p^T J_l and G Hinv G^T, written
        # out over the two rows and the three landmark columns
        G = A[:, 0, :, None] * L[:, 0, None, :] + A[:, 1, :, None] * L[:, 1, None, :]  # (m, 9, 3)
        Hi = inv[lin.pi[s:e]]
        GH = G[:, :, 0, None] * Hi[:, None, 0, :] + G[:, :, 1, None] * Hi[:, None, 1, :] + \
            G[:, :, 2, None] * Hi[:, None, 2, :]  # G Hinv, (m, 9, 3)
        term = (A[:, 0, :, None] * A[:, 0, None, :] + A[:, 1, :, None] * A[:, 1, None, :]
                - (GH[:, :, 0, None] * G[:, None, :, 0] + GH[:, :, 1, None] * G[:, None, :, 1]
                   + GH[:, :, 2, None] * G[:, None, :, 2]))
        blocks += _sum_by(lin.ci[s:e], term.reshape(-1, 81), lin.n_cams)
    blocks = blocks.reshape(-1, 9, 9) + lam * np.eye(9)[None]
    return ReducedOperator(lam, lin.n_cams, lin.n_points, lin.ci, lin.pi, Jps, Jls, inv, bl, b.reshape(-1), blocks)


def back_substitute(rs, dxp_scaled: np.ndarray) -> np.ndarray:
    """Scaled landmark increment dx~_l = -H_ll^-1 (b_l + H_lp dx~_p) (eq. backsub_sc).

    `rs` is the assembled ReducedSystem or the ReducedOperator of the same system."""
    if isinstance(rs, ReducedOperator):
        return -np.einsum("lij,lj->li", rs.Hll_inv, rs.bl + rs.lp(dxp_scaled)).reshape(-1)
    return -(rs.Hll_inv @ (rs.bl + rs.Hpl.T @ dxp_scaled))


def model_decrease(lin: Linearization, dxp_scaled: np.ndarray, dxl_scaled: np.ndarray) -> float:
    """E - |r + J~ dx~|^2 evaluated row by row as -sum u (2 r + u), u = J~ dx~.

    The undamped linear model is used, so the damping rows do not enter.
    """
    dp = dxp_scaled.reshape(lin.n_cams, 9) * lin.sp
    dl = dxl_scaled.reshape(lin.n_points, 3) * lin.sl
    u = np.einsum("nij,nj->ni", lin.Jp, dp[lin.ci]) + np.einsum("nij,nj->ni", lin.Jl, dl[lin.pi])
    return float(-np.sum(u * (2.0 * lin.r + u)))
