"""Seeded inputs for the clustering tests in which centres drift: a field of
a few moving Gaussian blobs over low noise, and particles in two tight swarms
that cross the domain (so that dense groups of point samples pull their
centres).  With value weights far above the space-time weight, samples pick
centres by value and the centres wander about a whole grid cell from their
seeds within a few iterations, so that many samples end up with a centre
seeded two or more cells away.  Inputs only: no clustering arithmetic."""
import numpy as np

F32 = np.float32


def swarm_case(seed, T=8, Z=16, Y=16, X=16, P=3000):
    rng = np.random.default_rng(seed)
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    field = (0.05 * rng.random((T, Z, Y, X))).astype(F32)
    for _ in range(4):
        c = rng.random(4) * np.array([X, Y, Z, T])
        s = rng.uniform(2, 4)
        r2 = ((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2) / (2 * s * s) + (t - c[3]) ** 2 / 8
        field += np.exp(-r2).astype(F32)
    xyz = np.empty((T, P, 3))
    for h in range(2):
        c0 = rng.random(3) * np.array([X, Y, Z])
        v = rng.normal(size=3)
        v /= np.linalg.norm(v)
        sl = slice(h * P // 2, (h + 1) * P // 2)
        for tt in range(T):
            xyz[tt, sl] = c0 + 1.2 * tt * v + rng.normal(scale=0.7, size=(P // 2, 3))
    xyz = np.mod(xyz, [X, Y, Z]).astype(F32)
    attr = rng.random((T, P), dtype=F32)
    return field, xyz, attr


SWARM_K = (4, 4, 4, 2)
SWARM_W = (0.05, 4.0, 4.0)   # (w_d, w_f, w_p): value terms dominate
SWARM_CF = 1.0
