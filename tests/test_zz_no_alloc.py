"""The reduced-camera-system product without allocation (sqrtba_rcs_matvec_noalloc).

Through the C ABI: its output equals that of sqrtba_debug_rcs_matvec (the same
kernels with the context's workspace as scratch) bit for bit, on two calls in a
row, the second on a smaller problem (so the shared static scratch holds the
larger problem's values when it starts), in FP32 and FP64; a problem whose
product needs more scratch than the static array holds, and landmark-block
forms other than explicit blocks, are rejected with SQRTBA_E_UNSUPPORTED.
"""

import numpy as np
import pytest

from bal_synth import make_config, make_ring_problem

from gpu_util import gpu_context, mixed_problem

pytestmark = pytest.mark.gpu

E_UNSUPPORTED = -6


def _product_both_ways(p, precision, seed):
    import torch

    dt = torch.float64 if precision == 64 else torch.float32
    ctx = gpu_context(p, precision=precision)
    ctx.linearize()
    ctx.marginalize()
    ctx.damp(1e-4)
    n = 9 * p.n_cams
    v = np.random.default_rng(seed).normal(size=n).astype(np.float64 if precision == 64 else np.float32)
    ref = ctx.debug_rcs_matvec(v)
    vd = torch.as_tensor(v).to("cuda")
    out = torch.full((n,), float("nan"), dtype=dt, device="cuda")
    torch.cuda.synchronize()
    ctx.rcs_matvec_noalloc(vd, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    ctx.close()
    return ref, got


@pytest.mark.parametrize("precision", [32, 64])
def test_noalloc_product_equals_the_workspace_product(precision):
    # first a problem with every size class, including row-block landmarks (k >= 114)
    big = mixed_problem(seed=5, n_cams=160, n_points=400)
    ref, got = _product_both_ways(big, precision, 1)
    assert np.all(np.isfinite(got))
    np.testing.assert_array_equal(got, ref)
    # then a smaller one: the static scratch still holds the first call's values
    small = make_config(0)
    ref, got = _product_both_ways(small, precision, 2)
    np.testing.assert_array_equal(got, ref)


def test_noalloc_product_rejects_what_does_not_fit():
    import torch
    from paper_2103_01843_amd import SqrtBAError

    # about 400k landmarks of 3..8 observations: ~84 MB of product outputs
    p = make_ring_problem(np.random.default_rng(3), 60, 400_000, lambda r, n: r.integers(3, 9, size=n))
    for blocks, label in ((0, "too large"), (1, "implicit blocks")):
        q = p if blocks == 0 else make_config(0)
        ctx = gpu_context(q, landmark_blocks=blocks)
        ctx.linearize()
        ctx.marginalize()
        ctx.damp(1e-4)
        v = torch.zeros(9 * q.n_cams, device="cuda")
        out = torch.zeros_like(v)
        with pytest.raises(SqrtBAError) as ei:
            ctx.rcs_matvec_noalloc(v, out)
        assert ei.value.status == E_UNSUPPORTED, label
        ctx.close()
