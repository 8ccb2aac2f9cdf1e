"""FP64 reference of the learned block preconditioner (test infrastructure).

The paper has no learned component; this is the project's own definition,
written out plainly so the GPU kernels can be checked against it:

  network:   h1 = tanh(x W1 + b1), h2 = tanh(h1 W2 + b2), e = h2 W3 + b3,
             x in R^64, h1, h2 in R^128, e in R^81 read as a 9x9 matrix E
             (row-major); weights are rounded to bfloat16 before use.
  block:     T = I + alpha tanh(tril(E)) (lower triangle incl. diagonal,
             alpha = 0.1, so diag(T) >= 0.9), C = L^-T T with L the lower
             Cholesky factor of the damped block-Jacobi block P = L L^T, and
             the inverse-preconditioner block M^-1 = C C^T (SPD).  E = 0
             gives M^-1 = P^-1, i.e. plain block-Jacobi.
  loss:      for a PCG trace pair (p, q = A p) restricted to one camera,
             l = |M^-1 q - p|^2 / |p|^2; a batch loss is the mean.

Parity of this module with the paper is unpinned (the paper has no learned
part); it is pinned by central finite differences of its own loss and by the
SPD property, which are tested in tests/test_oracle_mlp.py.
"""

from __future__ import annotations

import numpy as np

N_IN, N_H, N_OUT = 64, 128, 81
ALPHA = 0.1
SHAPES = [("W1", (N_IN, N_H)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
          ("W3", (N_H, N_OUT)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)
TRIL = np.tril(np.ones((9, 9), dtype=bool))


def unpack(theta: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (round to nearest even on the top 16 bits of float32)."""
    f = np.asarray(a, dtype=np.float32).copy()
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(theta: np.ndarray, x: np.ndarray):
    P = unpack(theta)
    h1 = np.tanh(x @ P["W1"] + P["b1"])
    h2 = np.tanh(h1 @ P["W2"] + P["b2"])
    e = h2 @ P["W3"] + P["b3"]
    return e, (x, h1, h2)


def block_factor(E: np.ndarray, L: np.ndarray):
    """C = L^-T (I + alpha tanh(tril(E))) for E (n,9,9), L (n,9,9) lower."""
    th = np.tanh(np.where(TRIL, E, 0.0))
    T = np.eye(9)[None] + ALPHA * np.where(TRIL, th, 0.0)
    Linv_T = np.linalg.inv(L).transpose(0, 2, 1)
    return Linv_T @ T, T, th


def loss_and_grad(theta: np.ndarray, x: np.ndarray, L: np.ndarray, p: np.ndarray, q: np.ndarray):
    """Mean loss over n samples and its gradient w.r.t. theta (FP64, exact weights)."""
    n = x.shape[0]
    e, (x0, h1, h2) = forward(theta, x)
    E = e.reshape(n, 9, 9)
    C, T, th = block_factor(E, L)
    u = np.einsum("nba,nb->na", C, q)            # C^T q
    m = np.einsum("nab,nb->na", C, u)            # C C^T q
    r = m - p
    pp = np.sum(p * p, axis=1)
    loss = np.mean(np.sum(r * r, axis=1) / pp)
    g_m = (2.0 / n) * r / pp[:, None]            # dl/dm
    g_C = np.einsum("na,nb->nab", g_m, u)        # from m = C u
    g_u = np.einsum("nab,na->nb", C, g_m)        # C^T g_m
    g_C += np.einsum("na,nb->nab", q, g_u)       # from u = C^T q
    Linv = np.linalg.inv(L)
    g_T = Linv @ g_C                             # C = L^-T T
    g_E = np.where(TRIL, g_T * ALPHA * (1.0 - th * th), 0.0).reshape(n, 81)
    P = unpack(theta)
    g = {}
    g["W3"] = h2.T @ g_E
    g["b3"] = g_E.sum(0)
    d2 = (g_E @ P["W3"].T) * (1.0 - h2 * h2)
    g["W2"] = h1.T @ d2
    g["b2"] = d2.sum(0)
    d1 = (d2 @ P["W2"].T) * (1.0 - h1 * h1)
    g["W1"] = x0.T @ d1
    g["b1"] = d1.sum(0)
    return loss, np.concatenate([g[name].ravel() for name, _ in SHAPES])


def inverse_block(theta: np.ndarray, x: np.ndarray, L: np.ndarray) -> np.ndarray:
    e, _ = forward(theta, x)
    C, _, _ = block_factor(e.reshape(-1, 9, 9), L)
    return C @ C.transpose(0, 2, 1)


def init_params(seed: int = 0) -> np.ndarray:
    """Scaled-uniform first two layers; the last layer is zero, so the initial
    preconditioner is exactly block-Jacobi."""
    rng = np.random.default_rng(seed)
    th = []
    for name, shape in SHAPES:
        if name in ("W1", "W2"):
            lim = np.sqrt(6.0 / (shape[0] + shape[1]))
            th.append(rng.uniform(-lim, lim, size=shape).ravel())
        else:
            th.append(np.zeros(int(np.prod(shape))))
    return np.concatenate(th)
