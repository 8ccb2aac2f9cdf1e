"""Where the PCG convergence test runs (option pcg_test_kernel): in the per-camera
kernel after the next product (0) or in a kernel of its own after each update
(1).  Both take the same test on the same sums, so every result is the same bit
for bit; the second only skips the product after convergence (GPU)."""

import numpy as np
import pytest

from bal_synth import concat_problems, make_batch
from gpu_util import gpu_context, mixed_problem

pytestmark = pytest.mark.gpu

CASES = {
    "default": dict(),
    "forcing": dict(pcg_forcing_eta=0.1),
    "check_every_3": dict(pcg_check_every=3),
    "iteration_cap": dict(pcg_max_iters=7),
    "cap_at_chunk_end": dict(pcg_max_iters=8),
    "cap_two_chunks_of_4": dict(pcg_max_iters=8, pcg_check_every=4),
    "no_graph": dict(use_graph=0),
    "implicit": dict(landmark_blocks=1),
    "explicit_sc": dict(landmark_blocks=2),
}


@pytest.fixture(scope="module")
def problems():
    rng = np.random.default_rng(21)
    return {"mixed": mixed_problem(),
            "batch": concat_problems(make_batch(rng, 6, cams=(5, 20), points=(50, 200), k_hi=10))}


def _attempt(p, lam, **opts):
    ctx = gpu_context(p, **opts)
    ctx.linearize()
    ctx.marginalize()
    ctx.damp(lam)
    it, rel, st = ctx.solve()
    pred = ctx.back_substitute()
    new = ctx.update()
    cams = ctx.get_cameras()
    ctx.close()
    return it, rel, st, pred, new, cams


@pytest.mark.parametrize("name", ["mixed", "batch"])
@pytest.mark.parametrize("case", list(CASES))
def test_one_attempt_same_bits(problems, name, case):
    p = problems[name]
    for lam in (1e-4, 1e-1):
        a = _attempt(p, lam, pcg_test_kernel=0, **CASES[case])
        b = _attempt(p, lam, pcg_test_kernel=1, **CASES[case])
        assert a[0].sum() > 0
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y, err_msg=f"{name} {case} lambda {lam}")


def test_lm_solve_same_bits(problems):
    out = []
    for t in (0, 1, -1):  # -1: these problems are far below the automatic threshold, so 0
        ctx = gpu_context(problems["batch"], pcg_test_kernel=t, max_lm_iters=8)
        reps = ctx.lm_solve()
        hist = [[{k: v for k, v in h.items() if k != "t"} for h in ctx.history(i)] for i in range(len(reps))]
        out.append(([(r.final_cost, r.iterations, r.accepted, r.total_pcg_iters, r.status) for r in reps], hist))
        ctx.close()
    assert out[0] == out[1] == out[2]
    assert sum(r[3] for r in out[0][0]) > 0


@pytest.mark.parametrize("bad", [2, -2])
def test_invalid_option_is_rejected(problems, bad):
    from paper_2103_01843_amd import SqrtBAError
    with pytest.raises(SqrtBAError) as ei:
        gpu_context(problems["mixed"], pcg_test_kernel=bad)
    assert ei.value.status == -1


@pytest.mark.parametrize("graph", [0, 1])
def test_zero_right_hand_side(graph):
    """Two cameras on one axis and landmarks on it, observed at the image centre:
    every residual is exactly zero, so the reduced right-hand side is zero and
    both forms stop before the first iteration (status zero_rhs), with a zero
    step and a zero model decrease."""
    import torch
    from paper_2103_01843_amd import Context
    cams = np.array([[0, 0, 0, 0, 0, -10, 500, 0, 0], [0, 0, 0, 0, 0, -20, 500, 0, 0]], np.float32)
    pts = np.array([[0, 0, 1], [0, 0, 2], [0, 0, 3]], np.float32)
    oc = np.array([0, 1, 0, 1, 0, 1], np.int32)
    op = np.array([0, 0, 1, 1, 2, 2], np.int32)
    uv = np.zeros((6, 2), np.float32)
    out = []
    for t in (0, 1):
        with Context(stream=torch.cuda.current_stream(), pcg_test_kernel=t, use_graph=graph) as ctx:
            ctx.load(cams, pts, oc, op, uv)
            ctx.bind_torch_workspace()
            assert ctx.linearize()[0] == 0.0
            ctx.marginalize()
            ctx.damp(1e-4)
            it, rel, st = ctx.solve()
            pred = ctx.back_substitute()
            new = ctx.update()
            out.append((it.tolist(), st.tolist(), pred.tolist(), new.tolist()))
    assert out[0] == out[1]
    assert out[0][0] == [0] and out[0][1] == [3] and out[0][2] == [0.0] and out[0][3] == [0.0]
