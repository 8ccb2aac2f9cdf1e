"""The seeded input generator is deterministic and produces the intended shapes (CPU)."""

import numpy as np

from bal_synth import make_config, problem_stats, concat_problems, make_batch


def test_seeded_and_deterministic():
    a, b = make_config(0), make_config(0)
    for f in ["cameras", "points", "obs_cam", "obs_pt", "obs_uv"]:
        assert np.array_equal(getattr(a, f), getattr(b, f))
    assert a.cameras.dtype == np.float32 and a.obs_cam.dtype == np.int32


def test_tiny_ring_shape():
    s = problem_stats(make_config(0))
    assert s["n_cams"] == 16 and s["n_points"] == 500
    assert 3 <= s["k_mean"] <= 8 and s["k_max"] <= 8
    p = make_config(0)
    # the ring includes an identity rotation (angle 0) and a half turn (angle pi)
    th = np.linalg.norm(p.gt_cameras[:, :3], axis=1)
    assert th[0] == 0.0 and np.isclose(th[8], np.pi)


def test_every_landmark_has_two_distinct_observations():
    p = make_config(0)
    k = np.bincount(p.obs_pt, minlength=p.n_points)
    assert k.min() >= 2
    pairs = set(zip(p.obs_cam.tolist(), p.obs_pt.tolist()))
    assert len(pairs) == p.n_obs


def test_batch_offsets():
    rng = np.random.default_rng(7)
    probs = make_batch(rng, 3, cams=(5, 8), points=(20, 30))
    b = concat_problems(probs)
    assert b.n_problems == 3
    assert b.cam_off[-1] == b.n_cams and b.pt_off[-1] == b.n_points
    prob_c = np.searchsorted(b.cam_off, b.obs_cam, side="right") - 1
    prob_p = np.searchsorted(b.pt_off, b.obs_pt, side="right") - 1
    assert np.array_equal(prob_c, prob_p)


def test_split_batch_inverts_concat():
    from bal_synth import split_batch
    rng = np.random.default_rng(8)
    probs = make_batch(rng, 4, cams=(5, 9), points=(20, 40), k_hi=6)
    for p, q in zip(probs, split_batch(concat_problems(probs))):
        for f in ["cameras", "points", "obs_cam", "obs_pt", "obs_uv"]:
            assert np.array_equal(getattr(p, f), getattr(q, f)), f
