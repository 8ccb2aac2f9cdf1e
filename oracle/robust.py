"""Huber loss applied by iteratively reweighted least squares (FP64).

Test infrastructure: only tests/, the smoke check and bench.py's CPU baseline
use this package.

Sec. 6.2 (experimental setup) robustifies the residuals with the Huber norm,
parameter 1 pixel, implemented by IRLS as Ceres does.  Reading used here: per
observation s = |r_o|^2 (its 2-vector of pixel residuals), and the energy is
E = sum_o rho(s_o) with

    rho(s) = s                         for s <= delta^2,
    rho(s) = 2 delta sqrt(s) - delta^2  otherwise,

which is continuous with a continuous first derivative at s = delta^2.  At a
linearization point both residual rows and both Jacobian rows of observation o
are multiplied by sqrt(w_o), w_o = rho'(s_o) = min(1, delta / |r_o|): the
gradient of the reweighted least-squares problem, 2 sum_o w_o J_o^T r_o, is
then the gradient of E (Ceres applies exactly this scaling to a loss whose
second derivative is not positive, which the Huber loss's is not).  The
linearized model, and hence the LM's expected decrease, is that of the
reweighted problem; the actual decrease is measured on E.
"""

from __future__ import annotations

import numpy as np


def huber_terms(s: np.ndarray, delta: float) -> np.ndarray:
    """rho(s) per observation, s = |r_o|^2."""
    s = np.asarray(s, dtype=np.float64)
    d2 = delta * delta
    return np.where(s <= d2, s, 2.0 * delta * np.sqrt(np.maximum(s, d2)) - d2)


def huber_weights(s: np.ndarray, delta: float) -> np.ndarray:
    """rho'(s) = min(1, delta / sqrt(s)) per observation (1 at s = 0)."""
    s = np.asarray(s, dtype=np.float64)
    d2 = delta * delta
    return np.where(s <= d2, 1.0, delta / np.sqrt(np.maximum(s, d2)))
