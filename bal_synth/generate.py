"""Seeded synthetic BAL-shaped bundle-adjustment problems.

The BAL problems the paper evaluates on (Sec. 6.2) are not available, so these
scenes stand in for them with the shapes of the paper's problem-size table
(appendix, Table 3): a small ring scene, a ladybug-like forward trajectory, a
batch of uneven ring scenes, a venice-like heavy-tailed scene and a dense
stress scene.

Data model (the BAL "Snavely" camera, Sec. 6.2): a camera is the 9-vector
(w, t, f, k1, k2) with w an angle-axis rotation.  A world point X maps to
P = R(w) X + t, p = -P_xy / P_z, and the observed pixel is
f * (1 + k1 |p|^2 + k2 |p|^4) * p (relative to the image centre), plus noise.
This module renders observations from ground truth with that model; it holds
no solver arithmetic.  Rotations are built with scipy's Rotation class.

Preprocessing follows Sec. 6.2: observations whose camera-frame depth -P_z is
small or negative at the perturbed initial state (threshold 0.1 scene units)
are dropped in double precision, then landmarks left with fewer than two
observations are removed.  All returned float arrays are float32, so the FP64
oracle and the FP32 GPU path start from bit-identical inputs.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np
from scipy.spatial.transform import Rotation

BASE_SEED = 20210301
DEPTH_MIN = 0.1


@dataclass
class Problem:
    name: str
    cameras: np.ndarray  # (n_p, 9) float32, BAL order (w, t, f, k1, k2)
    points: np.ndarray  # (n_l, 3) float32
    obs_cam: np.ndarray  # (n_o,) int32
    obs_pt: np.ndarray  # (n_o,) int32
    obs_uv: np.ndarray  # (n_o, 2) float32
    gt_cameras: np.ndarray  # (n_p, 9) float64
    gt_points: np.ndarray  # (n_l, 3) float64
    # CSR offsets over sub-problems for a batch (None for a single problem)
    cam_off: Optional[np.ndarray] = None
    pt_off: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)

    @property
    def n_cams(self) -> int:
        return int(self.cameras.shape[0])

    @property
    def n_points(self) -> int:
        return int(self.points.shape[0])

    @property
    def n_obs(self) -> int:
        return int(self.obs_cam.shape[0])

    @property
    def n_problems(self) -> int:
        return 1 if self.cam_off is None else int(len(self.cam_off) - 1)


# --------------------------------------------------------------------------
# data model: rendering of pixels from a scene (not solver arithmetic)
# --------------------------------------------------------------------------

def _cam_frame_points(cams: np.ndarray, pts: np.ndarray, ci: np.ndarray, pi: np.ndarray) -> np.ndarray:
    rot = Rotation.from_rotvec(cams[ci, 0:3]).as_matrix()
    return np.einsum("nij,nj->ni", rot, pts[pi]) + cams[ci, 3:6]


def _render(cams: np.ndarray, pts: np.ndarray, ci: np.ndarray, pi: np.ndarray) -> np.ndarray:
    P = _cam_frame_points(cams, pts, ci, pi)
    p = -P[:, 0:2] / P[:, 2:3]
    n2 = np.sum(p * p, axis=1, keepdims=True)
    f = cams[ci, 6:7]
    k1 = cams[ci, 7:8]
    k2 = cams[ci, 8:9]
    return f * (1.0 + k1 * n2 + k2 * n2 * n2) * p


# --------------------------------------------------------------------------
# sampling helpers
# --------------------------------------------------------------------------

def _distinct_rows(rng: np.random.Generator, n_rows: int, k: int, n: int) -> np.ndarray:
    """n_rows independent uniform k-subsets of range(n) (Floyd's algorithm, vectorized)."""
    out = np.empty((n_rows, k), dtype=np.int64)
    for col, j in enumerate(range(n - k, n)):
        t = rng.integers(0, j + 1, size=n_rows)
        if col:
            taken = np.any(out[:, :col] == t[:, None], axis=1)
            t = np.where(taken, j, t)
        out[:, col] = t
    return out


def _subsets_by_k(rng: np.random.Generator, ks: np.ndarray, n: int) -> List[np.ndarray]:
    """For each landmark j, ks[j] distinct camera indices from range(n), sorted."""
    res: List[Optional[np.ndarray]] = [None] * len(ks)
    for k in np.unique(ks):
        rows = np.nonzero(ks == k)[0]
        sub = np.sort(_distinct_rows(rng, len(rows), int(k), n), axis=1)
        for r, s in zip(rows, sub):
            res[r] = s
    return res  # type: ignore[return-value]


def _flatten(subsets: List[np.ndarray]):
    counts = np.fromiter((len(s) for s in subsets), dtype=np.int64, count=len(subsets))
    ci = np.concatenate(subsets).astype(np.int64)
    pi = np.repeat(np.arange(len(subsets), dtype=np.int64), counts)
    return ci, pi


def _perturb_cameras(rng: np.random.Generator, cams: np.ndarray, sigma: float) -> np.ndarray:
    """Perturb rotation and camera centre (not t), then rebuild t = -R c.

    Sec. 6.2 says the perturbation follows Ceres' BAL examples, which add
    Gaussian noise to the angle-axis vector and to the camera centre
    separately.  Intrinsics (f, k1, k2) get additive noise of the same sigma.
    """
    rot = Rotation.from_rotvec(cams[:, 0:3]).as_matrix()
    centre = -np.einsum("nji,nj->ni", rot, cams[:, 3:6])  # c = -R^T t
    w1 = cams[:, 0:3] + rng.normal(0.0, sigma, size=(cams.shape[0], 3))
    c1 = centre + rng.normal(0.0, sigma, size=(cams.shape[0], 3))
    intr1 = cams[:, 6:9] + rng.normal(0.0, sigma, size=(cams.shape[0], 3))
    t1 = -np.einsum("nij,nj->ni", Rotation.from_rotvec(w1).as_matrix(), c1)
    return np.concatenate([w1, t1, intr1], axis=1)


def _finish(name: str, rng: np.random.Generator, gt_cams: np.ndarray, gt_pts: np.ndarray,
            ci: np.ndarray, pi: np.ndarray, noise_px: float, cam_sigma: float,
            pt_sigma: float, meta: dict) -> Problem:
    uv = _render(gt_cams, gt_pts, ci, pi)
    if noise_px > 0:
        uv = uv + rng.normal(0.0, noise_px, size=uv.shape)
    cams0 = _perturb_cameras(rng, gt_cams, cam_sigma)
    pts0 = gt_pts + rng.normal(0.0, pt_sigma, size=gt_pts.shape)

    # visibility filter at the perturbed initial state, FP64 (Sec. 6.2)
    depth = -_cam_frame_points(cams0, pts0, ci, pi)[:, 2]
    keep = depth > DEPTH_MIN
    ci, pi, uv = ci[keep], pi[keep], uv[keep]
    cnt = np.bincount(pi, minlength=gt_pts.shape[0])
    good_pt = cnt >= 2
    keep = good_pt[pi]
    ci, pi, uv = ci[keep], pi[keep], uv[keep]
    remap = -np.ones(gt_pts.shape[0], dtype=np.int64)
    remap[good_pt] = np.arange(int(good_pt.sum()))
    pi = remap[pi]

    return Problem(
        name=name,
        cameras=cams0.astype(np.float32),
        points=pts0[good_pt].astype(np.float32),
        obs_cam=ci.astype(np.int32),
        obs_pt=pi.astype(np.int32),
        obs_uv=uv.astype(np.float32),
        gt_cameras=gt_cams,
        gt_points=gt_pts[good_pt],
        meta=meta,
    )


def _intrinsics(rng: np.random.Generator, n: int) -> np.ndarray:
    f = rng.uniform(400.0, 600.0, size=n)
    k1 = rng.normal(0.0, 1e-3, size=n)
    k2 = rng.normal(0.0, 1e-3, size=n)
    return np.stack([f, k1, k2], axis=1)


def _ring_cameras(rng: np.random.Generator, n: int, radius: float) -> np.ndarray:
    """n cameras evenly on a ring of the world XZ plane, each looking at the origin.

    Camera i sits at radius * (sin phi, 0, cos phi) with phi = 2 pi i / n; its
    world-to-camera rotation is a rotation by -phi about +y, so the camera's -z
    axis points at the origin and world +y is up.  phi = 0 gives the identity
    rotation and phi = pi a rotation by pi.
    """
    phi = 2.0 * np.pi * np.arange(n) / n
    w = np.zeros((n, 3))
    w[:, 1] = -phi
    t = np.zeros((n, 3))
    t[:, 2] = -radius
    return np.concatenate([w, t, _intrinsics(rng, n)], axis=1)


# --------------------------------------------------------------------------
# scene families
# --------------------------------------------------------------------------

def make_ring_problem(rng: np.random.Generator, n_cams: int, n_points: int,
                      k_sampler: Callable[[np.random.Generator, int], np.ndarray],
                      name: str = "ring", radius: float = 10.0, box: float = 2.0,
                      noise_px: float = 1.0, cam_sigma: float = 1e-2,
                      pt_sigma: float = 5e-2) -> Problem:
    gt_cams = _ring_cameras(rng, n_cams, radius)
    gt_pts = rng.uniform(-box, box, size=(n_points, 3))
    ks = np.clip(k_sampler(rng, n_points), 2, n_cams).astype(np.int64)
    # every ring camera sees the whole box (depth >= radius - sqrt(3) box > 0.1)
    ci, pi = _flatten(_subsets_by_k(rng, ks, n_cams))
    return _finish(name, rng, gt_cams, gt_pts, ci, pi, noise_px, cam_sigma, pt_sigma,
                   {"family": "ring"})


def make_forward_problem(rng: np.random.Generator, n_cams: int = 500, n_points: int = 100_000,
                         k_max: int = 50, name: str = "forward", noise_px: float = 1.0,
                         cam_sigma: float = 1e-2, pt_sigma: float = 5e-2) -> Problem:
    """Ladybug-like: cameras every unit along world -z looking along -z with yaw jitter.

    The trajectory is centred on the origin.  Landmark j has k = 2 + Geom(1/3)
    observations (support {0,1,...}), clamped to
    k_max, with one landmark forced to k_max.  It is seen by k consecutive
    cameras starting at a uniform index and lies 5..20 units ahead of the last
    of them, off the motion axis by 0.1..0.5 of that depth sideways and within
    +-0.3 of it in height, so every image coordinate stays within |p| < 0.6 as
    in real BAL images while off-axis points keep parallax.
    """
    yaw = rng.uniform(-0.05, 0.05, size=n_cams)
    w = np.zeros((n_cams, 3))
    w[:, 1] = yaw
    centres = np.zeros((n_cams, 3))
    centres[:, 2] = -(np.arange(n_cams, dtype=np.float64) - 0.5 * (n_cams - 1))  # centred on 0
    rot = Rotation.from_rotvec(w).as_matrix()
    t = -np.einsum("nij,nj->ni", rot, centres)
    gt_cams = np.concatenate([w, t, _intrinsics(rng, n_cams)], axis=1)

    ks = 2 + (rng.geometric(1.0 / 3.0, size=n_points) - 1)
    ks = np.minimum(ks, min(k_max, n_cams))
    ks[rng.integers(0, n_points)] = min(k_max, n_cams)
    start = (rng.random(n_points) * (n_cams - ks + 1)).astype(np.int64)
    last = start + ks - 1
    depth = rng.uniform(5.0, 20.0, size=n_points)
    side = np.where(rng.random(n_points) < 0.5, -1.0, 1.0)
    lat_x = side * rng.uniform(0.1, 0.5, size=n_points) * depth
    lat_y = rng.uniform(-0.3, 0.3, size=n_points) * depth
    gt_pts = np.stack([lat_x, lat_y, centres[last, 2] - depth], axis=1)
    counts = ks
    pi = np.repeat(np.arange(n_points, dtype=np.int64), counts)
    offs = np.concatenate([[0], np.cumsum(counts)[:-1]])
    ci = start[pi] + (np.arange(pi.shape[0]) - offs[pi])
    return _finish(name, rng, gt_cams, gt_pts, ci, pi, noise_px, cam_sigma, pt_sigma,
                   {"family": "forward"})


def _k_uniform(lo: int, hi: int):
    return lambda rng, n: rng.integers(lo, hi + 1, size=n)


def _k_venice(rng: np.random.Generator, n: int) -> np.ndarray:
    y = rng.lognormal(mean=0.40, sigma=1.30, size=n)
    return np.minimum(400, 2 + np.floor(y).astype(np.int64))


def _k_dense(rng: np.random.Generator, n: int) -> np.ndarray:
    e = np.floor(rng.exponential(160.0, size=n)).astype(np.int64)
    return 50 + np.minimum(450, e)


def make_batch(rng: np.random.Generator, n_problems: int = 256, cams=(5, 60), points=(200, 5000),
               k_hi: int = 30, noise_px: float = 1.0) -> List[Problem]:
    out = []
    for b in range(n_problems):
        nc = int(rng.integers(cams[0], cams[1] + 1))
        npt = int(rng.integers(points[0], points[1] + 1))
        out.append(make_ring_problem(rng, nc, npt, _k_uniform(2, min(k_hi, nc)),
                                     name=f"batch{b}", noise_px=noise_px))
    return out


def concat_problems(probs: List[Problem], name: str = "batch") -> Problem:
    """Stack independent problems into one with per-problem CSR offsets."""
    cam_off = np.zeros(len(probs) + 1, dtype=np.int64)
    pt_off = np.zeros(len(probs) + 1, dtype=np.int64)
    for i, p in enumerate(probs):
        cam_off[i + 1] = cam_off[i] + p.n_cams
        pt_off[i + 1] = pt_off[i] + p.n_points
    return Problem(
        name=name,
        cameras=np.concatenate([p.cameras for p in probs]),
        points=np.concatenate([p.points for p in probs]),
        obs_cam=np.concatenate([p.obs_cam.astype(np.int64) + cam_off[i] for i, p in enumerate(probs)]).astype(np.int32),
        obs_pt=np.concatenate([p.obs_pt.astype(np.int64) + pt_off[i] for i, p in enumerate(probs)]).astype(np.int32),
        obs_uv=np.concatenate([p.obs_uv for p in probs]),
        gt_cameras=np.concatenate([p.gt_cameras for p in probs]),
        gt_points=np.concatenate([p.gt_points for p in probs]),
        cam_off=cam_off,
        pt_off=pt_off,
        meta={"family": "batch", "n_problems": len(probs)},
    )


def split_batch(p: Problem) -> List[Problem]:
    """The independent problems of a stacked batch (inverse of concat_problems)."""
    if p.cam_off is None:
        return [p]
    prob = np.searchsorted(p.cam_off, p.obs_cam.astype(np.int64), side="right") - 1
    out = []
    for i in range(p.n_problems):
        c0, c1, l0, l1 = p.cam_off[i], p.cam_off[i + 1], p.pt_off[i], p.pt_off[i + 1]
        m = prob == i
        out.append(Problem(f"{p.name}[{i}]", p.cameras[c0:c1], p.points[l0:l1],
                           (p.obs_cam[m] - c0).astype(np.int32), (p.obs_pt[m] - l0).astype(np.int32),
                           p.obs_uv[m], p.gt_cameras[c0:c1], p.gt_points[l0:l1]))
    return out


CONFIG_NAMES = ["tiny-ring", "ladybug-like", "batch-256", "venice-like", "dense-stress"]


def make_config(i: int, seed: Optional[int] = None, noise_px: float = 1.0) -> Problem:
    """The five workloads: 0 tiny ring, 1 ladybug-like, 2 batch of 256, 3 venice-like, 4 dense."""
    rng = np.random.default_rng(BASE_SEED + i if seed is None else seed)
    if i == 0:
        p = make_ring_problem(rng, 16, 500, _k_uniform(3, 8), name=CONFIG_NAMES[0], noise_px=noise_px)
    elif i == 1:
        p = make_forward_problem(rng, 500, 100_000, 50, name=CONFIG_NAMES[1], noise_px=noise_px)
    elif i == 2:
        p = concat_problems(make_batch(rng, 256, noise_px=noise_px), name=CONFIG_NAMES[2])
    elif i == 3:
        p = make_ring_problem(rng, 1778, 1_000_000, _k_venice, name=CONFIG_NAMES[3], noise_px=noise_px)
    elif i == 4:
        p = make_ring_problem(rng, 2000, 50_000, _k_dense, name=CONFIG_NAMES[4], noise_px=noise_px)
    else:
        raise ValueError(f"no config {i}")
    p.meta["config"] = i
    return p


def problem_stats(p: Problem) -> dict:
    k = np.bincount(p.obs_pt, minlength=p.n_points).astype(np.float64)
    return {
        "name": p.name,
        "n_problems": p.n_problems,
        "n_cams": p.n_cams,
        "n_points": p.n_points,
        "n_obs": p.n_obs,
        "k_mean": float(k.mean()),
        "k_std": float(k.std()),
        "k_max": int(k.max()),
        "lmb_bytes": float(np.sum((2 * k + 3) * (9 * k + 4) * 4)),
        "bhat_bytes": float(np.sum(72.0 * k * k)),
    }
