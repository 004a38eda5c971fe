"""Invariants that single out the grown set, and the coupled graph as an
explicit edge list for a library connected-components routine.

TEST INFRASTRUCTURE ONLY (see the package docstring).

A candidate (Mf, Mp) equals the grown set M iff
  I1  every member is admissible;
  I2  every admissible seed is a member;
  I3  no admissible node adjacent to a member lies outside the set (closure);
  I4  every member is connected to an admissible seed inside the set.
(I1-I3 make the set contain the least fixed point; I1 and I4 make it lie
inside the reachable set.)
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

from .sweep import particle_voxels


def _band(v, lo, hi):
    with np.errstate(invalid="ignore"):
        return (np.float32(lo) <= v) & (v <= np.float32(hi))


def admissible(field, attr, crit):
    f_lo, f_hi, a_lo, a_hi = crit
    Af = _band(np.asarray(field, np.float32), f_lo, f_hi)
    Ap = None if attr is None else _band(np.asarray(attr, np.float32), a_lo, a_hi)
    return Af, Ap


def edge_list(field, xyz, attr, crit, restrict_f=None, restrict_p=None, trajectories=True, rate=1):
    """Edges (a, b) between admissible nodes.  Voxel node id = canonical index
    ((t*Z+z)*Y+y)*X+x; particle node id = V + t*P + i.  Optional boolean
    restrict_* masks further limit the node set (used for I4).  Trajectory
    edges (i, t) - (i, t+1) come in the order (earlier, later); trajectories
    = False leaves them out.  rate: particle steps per field step (particle
    step tau lies in field step tau // rate); particle node id = V + tau*P + i."""
    field = np.asarray(field, np.float32)
    T, Z, Y, X = field.shape
    V = field.size
    Af, Ap = admissible(field, attr, crit)
    if restrict_f is not None:
        Af = Af & restrict_f
    idx = np.arange(V, dtype=np.int64).reshape(T, Z, Y, X)
    A, B = [], []
    for ax in range(4):
        n = field.shape[ax]
        lo = [slice(None)] * 4
        hi = [slice(None)] * 4
        lo[ax] = slice(0, n - 1)
        hi[ax] = slice(1, n)
        m = Af[tuple(lo)] & Af[tuple(hi)]
        A.append(idx[tuple(lo)][m])
        B.append(idx[tuple(hi)][m])
    P = 0 if xyz is None else xyz.shape[1]
    if P:
        if restrict_p is not None:
            Ap = Ap & restrict_p
        Tp = xyz.shape[0]
        pid = V + np.arange(Tp * P, dtype=np.int64).reshape(Tp, P)
        if trajectories:
            m = Ap[:-1] & Ap[1:]
            A.append(pid[:-1][m])
            B.append(pid[1:][m])
        ok, cx, cy, cz = particle_voxels(np.asarray(xyz, np.float32), (X, Y, Z))
        tt = np.broadcast_to((np.arange(Tp) // rate)[:, None], (Tp, P))
        vox = idx[tt, cz, cy, cx]
        m = ok & Ap & Af[tt, cz, cy, cx]
        A.append(pid[m])
        B.append(vox[m])
    return np.concatenate(A), np.concatenate(B), V, (xyz.shape[0] * P if P else 0)


def components_grow(field, xyz, attr, crit, seeds):
    """M from scipy's connected components of the explicit graph."""
    field = np.asarray(field, np.float32)
    T, Z, Y, X = field.shape
    a, b, V, Q = edge_list(field, xyz, attr, crit)
    N = V + Q
    g = sp.coo_matrix((np.ones(len(a), np.int8), (a, b)), shape=(N, N))
    _, lab = connected_components(g, directed=False)
    Af, _ = admissible(field, attr, crit)
    keep = set()
    for x, y, z, t in np.asarray(seeds, np.int64).reshape(-1, 4):
        if Af[t, z, y, x]:
            keep.add(lab[((t * Z + z) * Y + y) * X + x])
    member = np.isin(lab, np.fromiter(keep, np.int64, len(keep)))
    P = 0 if xyz is None else xyz.shape[1]
    return member[:V].reshape(T, Z, Y, X), member[V:].reshape(T, P)


def reach_grow(field, xyz, attr, crit, seeds, forward_only=True, rate=1):
    """M as the nodes reachable from the admissible seeds in the directed
    graph: every non-trajectory edge both ways, trajectory edges from t to
    t + 1 only (forward_only) or both ways; scipy's breadth-first order from
    a virtual source linked to the admissible seeds."""
    from scipy.sparse.csgraph import breadth_first_order
    field = np.asarray(field, np.float32)
    T, Z, Y, X = field.shape
    a, b, V, Q = edge_list(field, xyz, attr, crit, trajectories=False, rate=rate)
    src, dst = [a, b], [b, a]
    P = 0 if xyz is None else xyz.shape[1]
    if P:
        _, Ap = admissible(field, attr, crit)
        Tp = xyz.shape[0]
        pid = V + np.arange(Tp * P, dtype=np.int64).reshape(Tp, P)
        m = Ap[:-1] & Ap[1:]
        src.append(pid[:-1][m])
        dst.append(pid[1:][m])
        if not forward_only:
            src.append(pid[1:][m])
            dst.append(pid[:-1][m])
    Af, _ = admissible(field, attr, crit)
    N = V + Q
    sd = [((t * Z + z) * Y + y) * X + x for x, y, z, t in np.asarray(seeds, np.int64).reshape(-1, 4)
          if Af[t, z, y, x]]
    src.append(np.full(len(sd), N, np.int64))
    dst.append(np.asarray(sd, np.int64))
    s, d = np.concatenate(src), np.concatenate(dst)
    g = sp.coo_matrix((np.ones(len(s), np.int8), (s, d)), shape=(N + 1, N + 1)).tocsr()
    order = breadth_first_order(g, N, directed=True, return_predecessors=False)
    member = np.zeros(N + 1, bool)
    member[order] = True
    return member[:V].reshape(T, Z, Y, X), member[V:N].reshape(-1, P) if P else np.zeros(
        (T if xyz is None else xyz.shape[0], 0), bool)


def check_invariants(field, xyz, attr, crit, seeds, Mf, Mp):
    """Returns {'I1': bool, 'I2': bool, 'I3': bool, 'I4': bool}."""
    field = np.asarray(field, np.float32)
    T, Z, Y, X = field.shape
    P = 0 if xyz is None else xyz.shape[1]
    Mf = np.asarray(Mf, bool).reshape(T, Z, Y, X)
    Mp = np.asarray(Mp, bool).reshape(T, P)
    Af, Ap = admissible(field, attr, crit)
    if Ap is None:
        Ap = np.zeros((T, 0), bool)
    res = {}
    res["I1"] = bool(not (Mf & ~Af).any() and not (Mp & ~Ap).any())
    sd = np.asarray(seeds, np.int64).reshape(-1, 4)
    ok2 = True
    for x, y, z, t in sd:
        if Af[t, z, y, x] and not Mf[t, z, y, x]:
            ok2 = False
    res["I2"] = ok2
    # I3: an edge with exactly one endpoint inside the set violates closure.
    a, b, V, Q = edge_list(field, xyz, attr, crit)
    member = np.concatenate([Mf.ravel(), Mp.ravel()])
    res["I3"] = bool(not (member[a] ^ member[b]).any())
    # I4: components of the graph induced on the set itself.
    a, b, V, Q = edge_list(field, xyz, attr, crit, restrict_f=Mf, restrict_p=Mp)
    N = V + Q
    g = sp.coo_matrix((np.ones(len(a), np.int8), (a, b)), shape=(N, N))
    _, lab = connected_components(g, directed=False)
    seed_labels = {lab[((t * Z + z) * Y + y) * X + x] for x, y, z, t in sd if Mf[t, z, y, x]}
    mem_labels = lab[member]
    res["I4"] = bool(np.isin(mem_labels, np.fromiter(seed_labels, np.int64,
                                                      len(seed_labels))).all())
    return res
