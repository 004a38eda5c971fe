"""Trajectory segments of a feature (Section 3.4), the oracle.

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the product
library.  Plain Python over each trajectory.

When a particle's steps are spread over several features (or leave the
feature), its trajectory is split into pieces, and a piece is drawn only
where at least two consecutive timesteps lie in the same feature.  Read here
(R) as: walk each trajectory in time, cut it into maximal runs of equal
feature id, and keep every run of two or more steps; steps in shorter runs,
and steps in no feature (id -1), are dropped.
"""
from __future__ import annotations

import numpy as np


def feature_segments(ids: np.ndarray) -> np.ndarray:
    """ids int [T][P]: feature id of each particle-step (-1: none).  Returns
    int64 [T][P]: the id where the step lies in a run of >= 2 consecutive
    steps of that id, else -1."""
    ids = np.asarray(ids)
    T, P = ids.shape
    out = np.full((T, P), -1, np.int64)
    for p in range(P):
        t = 0
        while t < T:
            f = int(ids[t, p])
            end = t + 1
            while end < T and int(ids[end, p]) == f:
                end += 1
            if f >= 0 and end - t >= 2:
                out[t:end, p] = f
            t = end
    return out


def mask_segments(pm: np.ndarray) -> np.ndarray:
    """The same rule for one grown feature: pm uint8 [T][P] member flags ->
    uint8 [T][P], the members in runs of >= 2 consecutive member steps."""
    ids = np.where(np.asarray(pm) != 0, 0, -1)
    return (feature_segments(ids) >= 0).astype(np.uint8)


def point_features(pl: np.ndarray, feat: np.ndarray) -> np.ndarray:
    """Feature id of each point sample from its centre label (-1 stays -1)."""
    pl = np.asarray(pl)
    feat = np.asarray(feat)
    return np.where(pl >= 0, feat[np.maximum(pl, 0)], -1)
