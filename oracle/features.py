"""Inputs of the brick-activity predictor, computed plainly from the samples.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The predictor sees the field and point samples of the paper's data model
(Section 3.1) summarised per brick-step: a brick is 8 x 8 x 8 voxels of one
timestep (the last brick of an axis may be cut short by the grid).  Per
brick-step:
  min, max, mean of the field values that are not NaN ((-1, -1, -1) when the
  brick holds no such value);
  the number of particle-steps whose position lies in the brick, a
  particle-step tau being placed at field step tau // rate and in the voxel
  floor(position) when every coordinate lies in [0, dim) (the field-to-point
  index of Section 3.1; NaN lies nowhere).
The network input of brick-step (t, bz, by, bx) has 16 bfloat16 channels:
  0..2  min, max, mean minus c, where c is the field lower bound (0 when it is
        not finite), each difference taken in float32;
  3     log1p(count) / 4 in float32;
  4..7  the same four at t - 1 (at t = 0: 0, 0, 0, 0);
  8..15 zero.
Each value is rounded to bfloat16 to nearest, ties to even.

The statistics are computed with numpy reductions over each brick's slice
(the mean in float64) and the counts with one histogram; nothing is blocked
or reordered beyond that.
"""
from __future__ import annotations

import numpy as np


def bf16_bits(a) -> np.ndarray:
    """bfloat16 bit patterns of float32 values, round to nearest even
    (bfloat16 is float32 with the low 16 mantissa bits dropped)."""
    u = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


def brick_dims(X: int, Y: int, Z: int, T: int) -> tuple:
    """(T, D, H, W): bricks per axis, the last one cut short by the grid."""
    return T, (Z + 7) // 8, (Y + 7) // 8, (X + 7) // 8


def brick_stats(field: np.ndarray) -> np.ndarray:
    """float64 [T][D][H][W][3]: min, max, mean of each brick-step's non-NaN
    field values, or (-1, -1, -1) when it has none."""
    f = np.asarray(field, np.float32)
    T, Z, Y, X = f.shape
    _, D, H, W = brick_dims(X, Y, Z, T)
    out = np.empty((T, D, H, W, 3), np.float64)
    for t in range(T):
        for bz in range(D):
            for by in range(H):
                for bx in range(W):
                    v = f[t, bz * 8:bz * 8 + 8, by * 8:by * 8 + 8, bx * 8:bx * 8 + 8]
                    v = v[~np.isnan(v)].astype(np.float64)
                    out[t, bz, by, bx] = (v.min(), v.max(), v.mean()) if v.size else (-1.0, -1.0, -1.0)
    return out


def brick_counts(xyz: np.ndarray, dims: tuple, T: int, rate: int = 1) -> np.ndarray:
    """int64 [T][D][H][W]: particle-steps per brick-step.  xyz [Tp][P][3] in
    voxel units; step tau lies at field step tau // rate."""
    X, Y, Z = dims
    _, D, H, W = brick_dims(X, Y, Z, T)
    out = np.zeros((T, D, H, W), np.int64)
    q = np.asarray(xyz, np.float32)
    Tp = q.shape[0]
    c = np.floor(q)  # float32 floor of the stored coordinates
    with np.errstate(invalid="ignore"):
        ok = ((c[..., 0] >= 0) & (c[..., 0] < np.float32(X)) & (c[..., 1] >= 0) & (c[..., 1] < np.float32(Y))
              & (c[..., 2] >= 0) & (c[..., 2] < np.float32(Z)))
    tau, p = np.nonzero(ok)
    t = tau // rate
    keep = t < T
    tau, p, t = tau[keep], p[keep], t[keep]
    x = c[tau, p, 0].astype(np.int64) // 8
    y = c[tau, p, 1].astype(np.int64) // 8
    z = c[tau, p, 2].astype(np.int64) // 8
    np.add.at(out, (t, z, y, x), 1)
    assert Tp >= 0
    return out


def features(field: np.ndarray, xyz, f_lo: float, rate: int = 1) -> np.ndarray:
    """bfloat16 bit patterns [T][D][H][W][16] of the network input (module
    docstring).  xyz may be None (no particles: counts 0)."""
    f = np.asarray(field, np.float32)
    T, Z, Y, X = f.shape
    st = brick_stats(f)
    cnt = (brick_counts(xyz, (X, Y, Z), T, rate) if xyz is not None and np.asarray(xyz).size
           else np.zeros(st.shape[:4], np.int64))
    lo = np.float32(f_lo)
    c = lo if (np.isfinite(lo) and abs(float(lo)) < 1e30) else np.float32(0.0)
    # statistics as the float32 values they are, then the differences in float32
    s32 = st.astype(np.float32)
    cur = np.empty(st.shape[:4] + (4,), np.float32)
    cur[..., :3] = s32 - c
    cur[..., 3] = (np.log1p(cnt.astype(np.float64)).astype(np.float32) * np.float32(0.25))
    prev = np.zeros_like(cur)
    prev[1:] = cur[:-1]
    x = np.zeros(st.shape[:4] + (16,), np.uint16)
    x[..., 0:4] = bf16_bits(cur)
    x[..., 4:8] = bf16_bits(prev)
    return x
