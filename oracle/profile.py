"""Time-to-tolerance from the performance-profile definition (appendix A.2).

f_tau = f* + tau (f_0 - f*), with f* the smallest cost any compared run
reached and f_0 the initial cost; t_tau is the earliest time at which a run's
best cost so far is <= f_tau (infinity if never).
"""

from __future__ import annotations

import math
from typing import Sequence


def cost_threshold(f0: float, fstar: float, tau: float = 0.01) -> float:
    return fstar + tau * (f0 - fstar)


def time_to_tolerance(times: Sequence[float], costs: Sequence[float], f_tau: float) -> float:
    best = math.inf
    for t, c in zip(times, costs):
        best = min(best, c)
        if best <= f_tau:
            return float(t)
    return math.inf
