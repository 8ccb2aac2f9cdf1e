"""Device-resident inputs and outputs through the C ABI (the *_device calls).

A problem loaded from CUDA tensors must behave bit for bit like the same problem
loaded from host arrays: the same LM decisions, costs and final state, in FP32
and FP64, for a single problem and a batch.  Host memory handed to a *_device
call is rejected with SQRTBA_E_INVALID before anything is read.
"""

import ctypes

import numpy as np
import pytest

from bal_synth import concat_problems, make_batch, make_config

from gpu_util import gpu_context

pytestmark = pytest.mark.gpu


def _device_context(p, precision=32, **opts):
    import torch
    from paper_2103_01843_amd import Context

    dt = torch.float64 if precision == 64 else torch.float32
    ctx = Context(stream=torch.cuda.current_stream(), precision=precision, **opts)
    t = {
        "cameras": torch.as_tensor(p.cameras.astype(np.float64 if precision == 64 else np.float32)).to("cuda", dt),
        "points": torch.as_tensor(p.points).to("cuda", dt),
        "obs_cam": torch.as_tensor(p.obs_cam).to("cuda"),
        "obs_pt": torch.as_tensor(p.obs_pt).to("cuda"),
        "obs_uv": torch.as_tensor(p.obs_uv).to("cuda", dt),
    }
    ctx.load_device(t["cameras"], t["points"], t["obs_cam"], t["obs_pt"], t["obs_uv"], p.cam_off, p.pt_off)
    del t  # the library copied them
    torch.cuda.synchronize()
    ctx.bind_torch_workspace()
    return ctx


@pytest.mark.parametrize("precision", [32, 64])
@pytest.mark.parametrize("kind", ["single", "batch"])
def test_device_inputs_match_host_inputs_bitwise(precision, kind):
    import torch

    if kind == "single":
        p = make_config(0)
    else:
        p = concat_problems(make_batch(np.random.default_rng(31), 3, cams=(5, 12), points=(40, 90), k_hi=8))
    a = gpu_context(p, max_lm_iters=6, precision=precision)
    ra = a.lm_solve()
    ha = [a.history(i) for i in range(p.n_problems)]
    cams_a, pts_a = a.get_cameras(), a.get_landmarks()
    a.close()
    b = _device_context(p, precision, max_lm_iters=6)
    rb = b.lm_solve()
    hb = [b.history(i) for i in range(p.n_problems)]
    dt = torch.float64 if precision == 64 else torch.float32
    cams_b = b.get_cameras_device(torch.empty(p.n_cams * 9, dtype=dt, device="cuda")).cpu().numpy()
    pts_b = b.get_landmarks_device(torch.empty(p.n_points * 3, dtype=dt, device="cuda")).cpu().numpy()
    np.testing.assert_array_equal(b.get_cameras().ravel(), cams_b)
    b.close()
    for x, y in zip(ra, rb):
        assert x.final_cost == y.final_cost and x.iterations == y.iterations
    for x, y in zip(ha, hb):
        assert [(h["accepted"], h["pcg_iters"], h["new_cost"]) for h in x] == \
               [(h["accepted"], h["pcg_iters"], h["new_cost"]) for h in y]
    np.testing.assert_array_equal(cams_a.ravel(), cams_b)
    np.testing.assert_array_equal(pts_a.ravel(), pts_b)


def test_device_calls_reject_host_memory():
    import torch
    from paper_2103_01843_amd import Context, SqrtBAError
    from paper_2103_01843_amd.sqrtba import lib

    p = make_config(0)
    host = np.ascontiguousarray(p.cameras, dtype=np.float32)
    with Context(stream=torch.cuda.current_stream()) as ctx:
        st = lib().sqrtba_set_cameras_device(ctx._h, p.n_cams, ctypes.c_void_p(host.ctypes.data))
        assert st == -1
        with pytest.raises(ValueError):  # the binding checks the tensor first
            ctx.set_cameras_device(torch.as_tensor(host))
        ctx.set_cameras_device(torch.as_tensor(host).cuda())
        ctx.set_landmarks(p.points)
        with pytest.raises(SqrtBAError) as ei:  # invalid data: the host call's error
            bad = torch.as_tensor(p.obs_cam).cuda()
            bad[0] = p.n_cams
            ctx.set_observations_device(bad, torch.as_tensor(p.obs_pt).cuda(), torch.as_tensor(p.obs_uv).cuda())
        assert ei.value.status == -1
