"""Launch shapes of the PCG product and their autotuner (GPU, through the C ABI).

Every shape must give the oracle's reduced camera system to the same bar as
the default shape (1e-4 relative in Frobenius norm).  Shapes that do not
regroup rows give bitwise the default shape's product; the bucket edge
rows_min_k and huge_rows regroup the rows of the largest blocks before their
partial products are added, so they are held to the oracle bar only.  The
autotuner must return the fastest of the shapes it timed (non-temporal loads
only when they gain more than 1%) and leave the solver's result unchanged
within rounding.
"""

import numpy as np
import pytest

import oracle
from paper_2103_01843_amd import SqrtBAError

from gpu_util import gpu_context, mixed_problem, oracle_lin

pytestmark = pytest.mark.gpu

DEFAULT = dict(rows_min_k=114, huge_rows=64, huge_side=0, large_separate=0, small_rows=4, persist_wgs=0,
               stream_loads=0)
SHAPES = [
    dict(DEFAULT, huge_side=1),
    dict(DEFAULT, large_separate=1),
    dict(DEFAULT, small_rows=8),
    dict(DEFAULT, persist_wgs=1024),
    dict(DEFAULT, persist_wgs=4096, small_rows=8, large_separate=1),
    dict(DEFAULT, huge_rows=128),
    dict(DEFAULT, huge_rows=512),
    dict(DEFAULT, huge_rows=1024),
    dict(DEFAULT, rows_min_k=61),
    dict(DEFAULT, rows_min_k=29, huge_rows=256, huge_side=1),
    dict(rows_min_k=29, huge_rows=1024, huge_side=1, large_separate=1, small_rows=8, persist_wgs=2048,
         stream_loads=0),
    dict(DEFAULT, stream_loads=1),
    dict(DEFAULT, stream_loads=1, large_separate=1, huge_side=1),
    dict(DEFAULT, rows_min_k=29, huge_rows=256, huge_side=1, large_separate=1, stream_loads=1),
    dict(DEFAULT, stream_loads=2),
    dict(DEFAULT, stream_loads=3, small_rows=8, large_separate=1, huge_side=1),
    dict(DEFAULT, stream_loads=2, persist_wgs=2048),
]


@pytest.fixture(scope="module")
def mixed():
    p = mixed_problem()
    bk, st, lin = oracle_lin(p)
    return p, lin


def test_every_shape_gives_the_reduced_system(mixed):
    p, lin = mixed
    lam = 1e-4
    ctx = gpu_context(p)
    ctx.linearize()
    ctx.marginalize()
    ctx.damp(lam)
    rs = oracle.reduced_camera_system(lin, lam)
    V = np.eye(rs.H.shape[0], dtype=np.float32)
    ctx.set_tuning(**DEFAULT)
    assert ctx.get_tuning() == DEFAULT
    ref = ctx.debug_rcs_matvec(V)
    for sh in SHAPES:
        ctx.set_tuning(**sh)
        assert ctx.get_tuning() == sh
        H = ctx.debug_rcs_matvec(V)
        e = np.linalg.norm(H.astype(np.float64) - rs.H) / np.linalg.norm(rs.H)
        assert e <= 1e-4, (sh, e)
        if sh["huge_rows"] == DEFAULT["huge_rows"] and sh["rows_min_k"] == DEFAULT["rows_min_k"]:
            np.testing.assert_array_equal(H, ref, err_msg=str(sh))
    ctx.close()


@pytest.mark.parametrize("bad", [dict(huge_rows=100), dict(huge_rows=32), dict(small_rows=5),
                                 dict(huge_side=2), dict(large_separate=-1), dict(rows_min_k=30),
                                 dict(rows_min_k=200), dict(persist_wgs=1000), dict(persist_wgs=-1),
                                 dict(stream_loads=4), dict(stream_loads=-1)])
def test_invalid_shapes_are_rejected(mixed, bad):
    p, _ = mixed
    ctx = gpu_context(p)
    before = ctx.get_tuning()
    with pytest.raises(SqrtBAError) as ei:
        ctx.set_tuning(**bad)
    assert ei.value.status == -1
    assert ctx.get_tuning() == before
    ctx.close()


def test_autotune_keeps_the_fastest_shape_and_the_result(mixed):
    p, _ = mixed
    plain = gpu_context(p, max_lm_iters=6)
    plain.set_tuning(**DEFAULT)
    ref = plain.lm_solve()[0]
    plain.close()
    ctx = gpu_context(p, max_lm_iters=6)
    best, trials = ctx.autotune(reps=3)
    assert best == ctx.get_tuning()
    assert len(trials) >= 10  # the mixed problem has landmarks in every size class
    ms = [t for _, t in trials]
    assert all(t > 0 for t in ms)
    fastest, t_fast = trials[int(np.argmin(ms))]
    if fastest != best:  # non-temporal loads are taken only when they gain more than 1%
        assert {k for k in best if best[k] != fastest[k]} == {"stream_loads"}, (best, fastest)
        assert t_fast >= 0.99 * min(t for sh, t in trials if sh == best)
    rep = ctx.lm_solve()[0]
    assert abs(rep.final_cost - ref.final_cost) <= 1e-5 * ref.final_cost
    ctx.close()
