"""Index bookkeeping of observations, written from the definitions (FP64 oracle side).

Storage (Sec. 5.1): residuals are grouped by landmark, so J_l is block-sparse
with one 2k x 3 block per landmark, and each landmark's rows form one dense
landmark block that holds only the camera columns it observes.  Inside a block
the observations are ordered by ascending camera index.

Preprocessing (Sec. 6.2): a landmark left with fewer than two observations is
removed.  Here such a landmark stays in the arrays but is inactive: its
observations take no part in the cost or the solve, and it is held fixed.  A
camera with no active observation is inactive too; its columns are empty.

Invalid input raises BookkeepingError: an index out of range, a non-finite
pixel, a duplicate (camera, landmark) pair, or an observation whose camera and
landmark belong to different sub-problems of a batch.
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np


class BookkeepingError(ValueError):
    pass


@dataclass
class Bookkeeping:
    n_cams: int
    n_points: int
    obs_perm: np.ndarray  # (n_act,) int64: input index of each active observation, sorted by (lm, cam)
    lm_off: np.ndarray  # (n_points + 1,) int64 CSR over the sorted active observations
    lm_active: np.ndarray  # (n_points,) bool, >= 2 observations
    cam_active: np.ndarray  # (n_cams,) bool
    cam_off: np.ndarray  # (n_cams + 1,) int64 CSR of the camera lists
    cam_obs: np.ndarray  # (n_act,) int64: sorted-observation positions, per camera ascending
    ci: np.ndarray  # (n_act,) camera of each sorted active observation
    pi: np.ndarray  # (n_act,) landmark of each sorted active observation

    @property
    def n_active_obs(self) -> int:
        return int(self.obs_perm.shape[0])


def build_bookkeeping(n_cams: int, n_points: int, obs_cam: np.ndarray, obs_pt: np.ndarray,
                      obs_uv: Optional[np.ndarray] = None,
                      cam_off: Optional[np.ndarray] = None,
                      pt_off: Optional[np.ndarray] = None) -> Bookkeeping:
    obs_cam = np.asarray(obs_cam, dtype=np.int64)
    obs_pt = np.asarray(obs_pt, dtype=np.int64)
    if n_cams <= 0 or n_points <= 0:
        raise BookkeepingError("need at least one camera and one landmark")
    if obs_cam.shape != obs_pt.shape or obs_cam.ndim != 1 or obs_cam.shape[0] == 0:
        raise BookkeepingError("observation arrays must be 1-D, non-empty and equally long")
    if obs_cam.min() < 0 or obs_cam.max() >= n_cams:
        raise BookkeepingError("camera index out of range")
    if obs_pt.min() < 0 or obs_pt.max() >= n_points:
        raise BookkeepingError("landmark index out of range")
    if obs_uv is not None and not np.all(np.isfinite(obs_uv)):
        raise BookkeepingError("non-finite observation")
    if cam_off is not None:
        prob_of_cam = np.searchsorted(np.asarray(cam_off), np.arange(n_cams), side="right") - 1
        prob_of_pt = np.searchsorted(np.asarray(pt_off), np.arange(n_points), side="right") - 1
        if np.any(prob_of_cam[obs_cam] != prob_of_pt[obs_pt]):
            raise BookkeepingError("observation links two different sub-problems")

    order = np.lexsort((obs_cam, obs_pt))  # primary key landmark, secondary camera
    sc, sp = obs_cam[order], obs_pt[order]
    if sc.shape[0] > 1 and np.any((sc[1:] == sc[:-1]) & (sp[1:] == sp[:-1])):
        raise BookkeepingError("duplicate (camera, landmark) observation")

    count = np.bincount(sp, minlength=n_points)
    lm_active = count >= 2
    keep = lm_active[sp]
    obs_perm = order[keep]
    ci, pi = sc[keep], sp[keep]
    act_count = np.where(lm_active, count, 0)
    lm_off = np.concatenate([[0], np.cumsum(act_count)]).astype(np.int64)

    cam_count = np.bincount(ci, minlength=n_cams)
    cam_active = cam_count > 0
    cam_off_ = np.concatenate([[0], np.cumsum(cam_count)]).astype(np.int64)
    cam_obs = np.argsort(ci, kind="stable").astype(np.int64)
    return Bookkeeping(n_cams, n_points, obs_perm.astype(np.int64), lm_off, lm_active, cam_active,
                       cam_off_, cam_obs, ci, pi)
