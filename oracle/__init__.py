"""FP64 CPU oracle for square-root bundle adjustment -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU product path never calls it.

The oracle computes what the method computes, by the plain definitions: the
paper proves (Sec. 4.4, eq. red_H / red_b and the damped remark closing that
section) that nullspace marginalization reaches exactly the Schur-complement
reduced system, so the oracle forms the damped normal equations (Sec. 4.1,
eq. normal_eq), reduces them with an explicit Schur complement (Sec. 4.2,
eq. red_normal_eq, back-substitution eq. backsub_sc), solves the reduced
camera system with a dense Cholesky factorization or block-Jacobi PCG
(Sec. 5.4), and drives it with Levenberg-Marquardt (Sec. 6.1), optionally with
the Huber loss of the experiments applied by IRLS (Sec. 6.2, ``robust``).  It shares no
code with the HIP path; only the input generator ``bal_synth`` serves both.

Readings of points the paper leaves open are stated in the docstrings of the
modules that implement them.
"""

from .camera import (  # noqa: F401
    so3_exp,
    so3_log,
    CameraState,
    state_from_bal,
    bal_from_state,
    project_residuals,
    linearize_observations,
    apply_update,
)
from .bookkeeping import Bookkeeping, build_bookkeeping, BookkeepingError  # noqa: F401
from .normal_equations import (  # noqa: F401
    Linearization,
    linearize,
    column_scales,
    scaled_jacobian_sparse,
    reduced_camera_system,
    reduced_system_operator,
    ReducedOperator,
    back_substitute,
    model_decrease,
)
from .solvers import dense_spd_solve, block_jacobi_blocks, pcg, quadratic_model  # noqa: F401
from .lm import LMOptions, LMResult, lm_solve, lm_attempt  # noqa: F401
from .profile import cost_threshold, time_to_tolerance  # noqa: F401
from .robust import huber_terms, huber_weights  # noqa: F401
