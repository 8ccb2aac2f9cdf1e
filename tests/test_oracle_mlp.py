"""Pins of the FP64 learned-preconditioner reference (CPU).

The paper has no learned component, so parity with the paper is unpinned; the
reference is pinned by central finite differences of its own loss, by torch's
independent bfloat16 conversion, and by the SPD and block-Jacobi properties of
its block map.
"""

import numpy as np
import torch

from oracle import mlp


def _samples(rng, n):
    x = rng.normal(size=(n, mlp.N_IN))
    A = rng.normal(size=(n, 9, 9))
    P = A @ A.transpose(0, 2, 1) + 9 * np.eye(9)
    L = np.linalg.cholesky(P)
    p = rng.normal(size=(n, 9))
    q = np.einsum("nab,nb->na", P, p) + 0.3 * rng.normal(size=(n, 9))
    return x, L, p, q, P


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    theta = mlp.init_params(1) + 0.05 * rng.normal(size=mlp.N_PARAMS)
    x, L, p, q, _ = _samples(rng, 6)
    loss, g = mlp.loss_and_grad(theta, x, L, p, q)
    idx = rng.choice(mlp.N_PARAMS, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros(mlp.N_PARAMS)
        e[i] = h
        fd = (mlp.loss_and_grad(theta + e, x, L, p, q)[0] - mlp.loss_and_grad(theta - e, x, L, p, q)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_zero_output_is_block_jacobi_and_blocks_are_spd():
    rng = np.random.default_rng(1)
    x, L, p, q, P = _samples(rng, 5)
    theta0 = mlp.init_params(2)
    np.testing.assert_allclose(mlp.inverse_block(theta0, x, L), np.linalg.inv(P), rtol=1e-10, atol=1e-12)
    theta = rng.normal(size=mlp.N_PARAMS) * 3.0  # arbitrary, large outputs
    M = mlp.inverse_block(theta, x, L)
    for m in M:
        np.linalg.cholesky(0.5 * (m + m.T))  # positive definite
        assert np.allclose(m, m.T, atol=1e-12 * np.abs(m).max())


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(3)
    a = np.concatenate([rng.normal(size=1000).astype(np.float32), np.float32([1 + 2 ** -8, 1 + 3 * 2 ** -8, -2.5e-3])])
    ref = torch.from_numpy(a).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(mlp.bf16_round(a).astype(np.float32), ref)
