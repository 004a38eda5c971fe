"""The grower's fixed point iterated literally (brute force).

TEST INFRASTRUCTURE ONLY (see the package docstring).

M is the least fixed point of F(X) = S_adm ∪ (Adm ∩ (X ∪ N(X))), where N(X)
holds every node that shares an edge with a node of X (edges: six spatial grid
neighbours and t±1 of a voxel, a particle-step and the voxel holding it, a
particle-step and the same particle at t±1 -- the data model of Section 3.1
and the trajectory coupling motivated in Section 1).  Starting from
X_0 = S_adm, synchronous full sweeps X_{k+1} = F(X_k) are repeated until a
sweep changes nothing; the number of sweeps, counting that last one, is
D + 1 where D is the largest breadth-first level.

With forward_only (causal coupling) a particle-step is a neighbour of the
same particle's previous step only: N(X) gains (i, t+1) from (i, t) in X, not
(i, t-1).  With rate r the particles hold their own steps, r per field step;
particle step tau couples with a voxel of field step tau // r.
"""
from __future__ import annotations

import numpy as np


def _band(v, lo, hi):
    return (np.float32(lo) <= v) & (v <= np.float32(hi))


def particle_voxels(xyz: np.ndarray, dims):
    """(valid [T][P] bool, cx, cy, cz int64 arrays over all steps): the voxel
    covering each stored position, voxel i covering [i, i+1)."""
    X, Y, Z = dims
    c = np.floor(xyz)  # stays fp32
    with np.errstate(invalid="ignore"):
        ok = ((c[..., 0] >= 0) & (c[..., 0] < np.float32(X)) &
              (c[..., 1] >= 0) & (c[..., 1] < np.float32(Y)) &
              (c[..., 2] >= 0) & (c[..., 2] < np.float32(Z)))
    ci = np.where(ok[..., None], c, 0).astype(np.int64)
    return ok, ci[..., 0], ci[..., 1], ci[..., 2]


def sweep_grow(field, xyz, attr, crit, seeds, max_sweeps: int | None = None,
               forward_only: bool = False, rate: int = 1):
    """Returns (Mf bool [T][Z][Y][X], Mp bool [Tp][P], sweeps, dropped)."""
    field = np.asarray(field, np.float32)
    T, Z, Y, X = field.shape
    f_lo, f_hi, a_lo, a_hi = (np.float32(v) for v in crit)
    with np.errstate(invalid="ignore"):
        Af = _band(field, f_lo, f_hi)
    P = 0 if xyz is None else xyz.shape[1]
    if P:
        with np.errstate(invalid="ignore"):
            Ap = _band(np.asarray(attr, np.float32), a_lo, a_hi)
        ok, cx, cy, cz = particle_voxels(np.asarray(xyz, np.float32), (X, Y, Z))
        tt, pp = np.nonzero(ok)
        bx, by, bz = cx[tt, pp], cy[tt, pp], cz[tt, pp]
        tf = tt // rate  # field step of each particle step
    else:
        Ap = np.zeros((T if xyz is None else xyz.shape[0], 0), bool)
    Mf = np.zeros_like(Af)
    Mp = np.zeros_like(Ap)
    dropped = 0
    for x, y, z, t in np.asarray(seeds, np.int64).reshape(-1, 4):
        if not (0 <= x < X and 0 <= y < Y and 0 <= z < Z and 0 <= t < T):
            raise IndexError("seed out of range")
        if Af[t, z, y, x]:
            Mf[t, z, y, x] = True
        else:
            dropped += 1
    sweeps = 0
    while True:
        sweeps += 1
        Nf = Mf.copy()
        for ax in range(4):
            n = Mf.shape[ax]
            lo = [slice(None)] * 4
            hi = [slice(None)] * 4
            lo[ax] = slice(0, n - 1)
            hi[ax] = slice(1, n)
            Nf[tuple(hi)] |= Mf[tuple(lo)]
            Nf[tuple(lo)] |= Mf[tuple(hi)]
        Np = Mp.copy()
        if P:
            Np[1:] |= Mp[:-1]
            if not forward_only:
                Np[:-1] |= Mp[1:]
            from_p = Mp[tt, pp]
            Nf[tf[from_p], bz[from_p], by[from_p], bx[from_p]] = True
            Np[tt, pp] |= Mf[tf, bz, by, bx]
        nMf = Af & Nf
        nMp = Ap & Np
        if np.array_equal(nMf, Mf) and np.array_equal(nMp, Mp):
            break
        Mf, Mp = nMf, nMp
        if max_sweeps is not None and sweeps >= max_sweeps:
            break
    return Mf, Mp, sweeps, dropped
