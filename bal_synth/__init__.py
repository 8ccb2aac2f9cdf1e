"""Seeded synthetic bundle-adjustment problems shaped like the BAL suite.

This package only *creates* inputs (scenes, observations, noise draws).  It
contains none of the solver's arithmetic: no Jacobians, no marginalization, no
linear solves, no Levenberg-Marquardt logic.  Both the FP64 oracle and the GPU
path consume exactly the arrays it returns.
"""

from .generate import (  # noqa: F401
    BASE_SEED,
    Problem,
    make_config,
    make_ring_problem,
    make_forward_problem,
    make_batch,
    concat_problems,
    split_batch,
    problem_stats,
)
