"""What a learned 9x9 block-diagonal preconditioner can gain over block-Jacobi (CPU).

The learned preconditioner (not in the paper; project-defined) emits one SPD
9x9 inverse block per camera.  Two facts bound what any such network can gain
over plain block-Jacobi, whatever it is trained on:

* Kaporin's condition number K(M^-1 A) = (tr(M^-1 A) / n)^n / det(M^-1 A), which
  bounds the number of CG iterations, is minimized over block-diagonal SPD M
  exactly by M = c blockdiag(A_ii): setting the derivative of
  n log tr(X A) - log det X over X = blockdiag(X_i) to zero gives
  X_i^-1 = (tr(X A) / n) A_ii for every block.  Checked on random SPD matrices
  against random block-diagonal alternatives.
* The most convergence-aligned training a network could receive: every
  camera's block a free parameter (an upper bound for any network of
  per-camera features), fitted on a real reduced camera system by gradient
  descent through unrolled PCG iterations (the A-norm error after K steps) on
  training right-hand sides.  On held-out right-hand sides, the system's own
  b~ among them, the fitted blocks need no fewer PCG iterations than
  block-Jacobi: the fit only specializes to the training vectors.

Parity with the paper is unpinned here by nature (the paper has no learned
part); these are properties of block-diagonal preconditioning.
"""

import numpy as np
import pytest

import oracle
from bal_synth import make_forward_problem


def _log_kaporin(A, Minv):
    w = np.linalg.eigvals(Minv @ A).real
    n = len(w)
    return n * np.log(np.sum(w) / n) - np.sum(np.log(w))


def _blockdiag(blocks):
    n = len(blocks)
    out = np.zeros((9 * n, 9 * n))
    for i, b in enumerate(blocks):
        out[9 * i:9 * i + 9, 9 * i:9 * i + 9] = b
    return out


def test_block_jacobi_minimizes_kaporin_condition_number():
    rng = np.random.default_rng(0)
    for trial in range(3):
        G = rng.normal(size=(54, 80))
        A = G @ G.T + 0.1 * np.eye(54)
        D = [A[9 * i:9 * i + 9, 9 * i:9 * i + 9] for i in range(6)]
        bj = _blockdiag([np.linalg.inv(d) for d in D])
        k_bj = _log_kaporin(A, bj)
        assert _log_kaporin(A, 3.7 * bj) == pytest.approx(k_bj, abs=1e-9)  # scale-free
        for _ in range(50):
            blocks = []
            for d in D:
                S = rng.normal(size=(9, 9))
                S = 0.25 * (S + S.T) / np.linalg.norm(S + S.T, 2)
                R = np.linalg.cholesky(d)
                blocks.append(np.linalg.inv(R @ (np.eye(9) + S) @ R.T) * np.exp(rng.normal()))
            assert _log_kaporin(A, _blockdiag(blocks)) >= k_bj - 1e-9


def _pcg_iters(A, b, apply_minv, tol=1e-6, max_iters=2000):
    x = np.zeros_like(b)
    r = -b.copy()
    r0 = np.linalg.norm(r)
    z = apply_minv(r)
    p = z.copy()
    rz = r @ z
    for k in range(1, max_iters + 1):
        q = A @ p
        a = rz / (p @ q)
        x += a * p
        r -= a * q
        if np.linalg.norm(r) <= tol * r0:
            return k
        z = apply_minv(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return max_iters


@pytest.mark.slow
def test_blocks_fitted_through_unrolled_pcg_do_not_beat_block_jacobi():
    import torch

    torch.manual_seed(0)
    p = make_forward_problem(np.random.default_rng(42), 16, 600, 16)
    bk = oracle.build_bookkeeping(p.n_cams, p.n_points, p.obs_cam, p.obs_pt, p.obs_uv)
    lin = oracle.linearize(oracle.state_from_bal(p.cameras, p.points), bk, p.obs_uv)
    rs = oracle.reduced_camera_system(lin, 1e-4)
    A, b = rs.H, rs.b
    n = A.shape[0] // 9
    D = np.stack([A[9 * i:9 * i + 9, 9 * i:9 * i + 9] for i in range(n)])
    rng = np.random.default_rng(1)
    train = rng.normal(size=(8, 9 * n))
    held_out = [b] + list(rng.normal(size=(3, 9 * n)))

    def apply_blocks(Minv):
        return lambda v: np.einsum("nab,nb->na", Minv, v.reshape(-1, 9)).ravel()

    bj_iters = [_pcg_iters(A, r, apply_blocks(np.linalg.inv(D))) for r in held_out]

    # free per-camera factors: M_i^-1 = C_i C_i^T, C_i = L_i^-T (I + tril(T_i)), T = 0 is block-Jacobi
    dt = torch.float64
    Linv_T = torch.tensor(np.linalg.inv(np.linalg.cholesky(D)).transpose(0, 2, 1), dtype=dt)
    At = torch.tensor(A, dtype=dt)
    tril = torch.tril(torch.ones(9, 9, dtype=dt))
    T = torch.zeros(n, 9, 9, dtype=dt, requires_grad=True)

    def minv(Tm):
        C = Linv_T @ (torch.eye(9, dtype=dt) + Tm * tril)
        return C @ C.transpose(1, 2)

    def loss(Tm, B, K=20):
        Mi = minv(Tm)
        pre = lambda V: torch.einsum("nab,mnb->mna", Mi, V.reshape(V.shape[0], -1, 9)).reshape(V.shape[0], -1)
        X, R = torch.zeros_like(B), -B.clone()
        Z = pre(R)
        P, RZ = Z.clone(), (R * Z).sum(1)
        Xs = torch.linalg.solve(At, -B.T).T
        for _ in range(K):
            Q = P @ At
            a = RZ / (P * Q).sum(1)
            X, R = X + a[:, None] * P, R - a[:, None] * Q
            Z = pre(R)
            RZn = (R * Z).sum(1)
            P, RZ = Z + (RZn / RZ)[:, None] * P, RZn
        E = X - Xs
        return torch.log((E * (E @ At)).sum(1) / (Xs * (Xs @ At)).sum(1)).mean()

    Bt = torch.tensor(train, dtype=dt)
    opt = torch.optim.Adam([T], lr=2e-3)
    first = None
    for _ in range(80):
        opt.zero_grad()
        l = loss(T, Bt)
        first = l.item() if first is None else first
        l.backward()
        opt.step()
    assert loss(T, Bt).item() < first - 0.05  # the fit does lower the training objective
    with torch.no_grad():
        fitted = minv(T).numpy()
    fit_iters = [_pcg_iters(A, r, apply_blocks(fitted)) for r in held_out]
    print(f"PCG iterations on held-out right-hand sides (b~ first): block-Jacobi {bj_iters}, fitted {fit_iters}")
    assert sum(fit_iters) >= 0.98 * sum(bj_iters), (bj_iters, fit_iters)
