"""Seeded synthetic inputs for the coupled point + field region grower.

This module only produces inputs; it holds none of the grower's arithmetic
(no thresholds are applied, no binning, no propagation).  Both the CPU oracle
and the GPU library consume the arrays it returns.

The paper's datasets (Section 4: the S3D lifted ethylene jet flame and the
Beijing taxi trajectories with traffic fields) are not available, so these
inputs stand in for them while keeping their shape (Section 3.1 data model,
Section 4.1 data sizes): a dense regular grid of field samples F(t) per
timestep, and a sparser set of moving points P(t) that carry their own value
and are stored at every timestep, so they form trajectories.

Recipe
------
Field f[t, z, y, x] (fp32) = sum over blobs b of
    A_b * exp(-|x_v - c_b(t)|^2 / (2 sigma_b^2)) + eta,
  x_v = voxel centre (i + 0.5, j + 0.5, k + 0.5),
  sigma_b ~ U[3, 6], A_b ~ U[0.5, 1], d_b uniform on the unit sphere,
  c_b(t) = c_b0 + 0.5 * t * d_b  (0.5 voxel per timestep),
  c_b0 ~ U[0.2 dim, 0.8 dim] per axis, eta ~ U[0, 0.05) i.i.d.
  Each Gaussian is evaluated inside a box of half-width ceil(5 sigma_b) around
  its centre (beyond it the term is below 4e-6 * A_b) in float64; the sum is
  cast to fp32 once.
  Crossing mode: blobs come in pairs that meet at m ~ U[0.3 dim, 0.7 dim] at
  time t_m ~ U[0.3 T, 0.7 T]; each blob of a pair starts at
  c_b0 = m - 0.5 * t_m * d_b with its own direction, so paths split and merge.
Particles: positions uniform in [0, 2 pi)^3, advected by the steady ABC flow
  (A = B = C = 1): u = (sin z + cos y, sin x + cos z, sin y + cos x), one RK4
  step of dt = 0.05 per stored timestep (t = 0 stores the initial position).
  Stored position (fp32, voxel units) = (p * dim / 2 pi) mod dim, cast once;
  a cast that rounds up to dim is stored as 0.
Attribute: trilinear sample of the fp32 field at timestep t at the stored
  position minus 0.5 (voxel centres), clamp-to-edge, float64, cast to fp32.
  Mode "noise": an independent U[0, 1) value instead (decouples the particle
  criterion from the field criterion).
Particle rate r (the paper's particles are saved more often than the field):
  r * T stored particle steps, one RK4 step of dt = 0.05 / r each (the same
  motion per field step), the attribute of step tau sampled from field step
  tau // r.  r = 1 is the recipe above, unchanged.
Planar (2D + t) instances are Z = 1 grids: stored z lies in [0, 1), so every
  particle moves in the one layer, and the blobs are evaluated at z = 0.5.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

__all__ = [
    "CONFIGS",
    "BlobSet",
    "make_blobs",
    "make_field",
    "make_particles",
    "sample_attribute",
    "make_instance",
    "make_config",
    "make_city",
    "blob_seeds",
    "make_queries",
]

_PARTICLE_CHUNK = 1 << 16


def _ss(seed) -> np.random.SeedSequence:
    return seed if isinstance(seed, np.random.SeedSequence) else np.random.SeedSequence(seed)


def _workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


class BlobSet:
    """Moving Gaussian blobs: centre c0 (n,3) in (x,y,z) voxel units,
    direction d (n,3), sigma (n,), amplitude (n,)."""

    def __init__(self, c0, d, sigma, amp):
        self.c0 = np.asarray(c0, np.float64)
        self.d = np.asarray(d, np.float64)
        self.sigma = np.asarray(sigma, np.float64)
        self.amp = np.asarray(amp, np.float64)

    def __len__(self):
        return len(self.sigma)

    def centre(self, b: int, t: float) -> np.ndarray:
        return self.c0[b] + 0.5 * t * self.d[b]


def _unit_vectors(rng: np.random.Generator, n: int) -> np.ndarray:
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def make_blobs(rng: np.random.Generator, n: int, dims, T: int,
               crossing: bool = False) -> BlobSet:
    dims = np.asarray(dims, np.float64)  # (X, Y, Z)
    sigma = rng.uniform(3.0, 6.0, size=n)
    amp = rng.uniform(0.5, 1.0, size=n)
    d = _unit_vectors(rng, n)
    if not crossing:
        c0 = rng.uniform(0.2, 0.8, size=(n, 3)) * dims
    else:
        if n % 2:
            raise ValueError("crossing blobs come in pairs")
        m = rng.uniform(0.3, 0.7, size=(n // 2, 3)) * dims
        tm = rng.uniform(0.3 * T, 0.7 * T, size=n // 2)
        m = np.repeat(m, 2, axis=0)
        tm = np.repeat(tm, 2)
        c0 = m - 0.5 * tm[:, None] * d
    return BlobSet(c0, d, sigma, amp)


def _field_step(blobs: BlobSet, dims, t: int, noise_seed) -> np.ndarray:
    X, Y, Z = dims
    rng = np.random.Generator(np.random.PCG64(noise_seed))
    f = rng.random((Z, Y, X)) * 0.05
    for b in range(len(blobs)):
        c = blobs.centre(b, t)
        s = blobs.sigma[b]
        r = int(math.ceil(5.0 * s))
        lo = [max(0, int(math.floor(c[a])) - r) for a in range(3)]
        hi = [min(dims[a], int(math.floor(c[a])) + r + 1) for a in range(3)]
        if any(h <= l for l, h in zip(lo, hi)):
            continue
        g = []
        for a in range(3):
            xs = np.arange(lo[a], hi[a], dtype=np.float64) + 0.5 - c[a]
            g.append(np.exp(-(xs * xs) / (2.0 * s * s)))
        f[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] += (
            blobs.amp[b] * g[2][:, None, None] * g[1][None, :, None] * g[0][None, None, :])
    return f.astype(np.float32)


def make_field(blobs: BlobSet, dims, T: int, seed: int) -> np.ndarray:
    """fp32 [T][Z][Y][X]; each timestep's noise has its own child stream so the
    result does not depend on the thread count."""
    X, Y, Z = (int(v) for v in dims)
    children = _ss(seed).spawn(T)
    out = np.empty((T, Z, Y, X), np.float32)

    def one(t):
        out[t] = _field_step(blobs, (X, Y, Z), t, children[t])

    with ThreadPoolExecutor(_workers()) as ex:
        list(ex.map(one, range(T)))
    return out


def _abc(p: np.ndarray) -> np.ndarray:
    x, y, z = p[:, 0], p[:, 1], p[:, 2]
    return np.stack([np.sin(z) + np.cos(y), np.sin(x) + np.cos(z),
                     np.sin(y) + np.cos(x)], axis=1)


def _store(p: np.ndarray, dims) -> np.ndarray:
    scale = np.asarray(dims, np.float64) / (2.0 * math.pi)
    q = np.mod(p * scale, np.asarray(dims, np.float64)).astype(np.float32)
    for a in range(3):
        col = q[:, a]
        col[col >= np.float32(dims[a])] = np.float32(0.0)
    return q


def make_particles(P: int, dims, T: int, seed: int, dt: float = 0.05) -> np.ndarray:
    """fp32 [T][P][3] positions in voxel units (x, y, z)."""
    out = np.empty((T, P, 3), np.float32)
    if P == 0:
        return out
    nchunk = (P + _PARTICLE_CHUNK - 1) // _PARTICLE_CHUNK
    children = _ss(seed).spawn(nchunk)

    def one(c):
        a, b = c * _PARTICLE_CHUNK, min(P, (c + 1) * _PARTICLE_CHUNK)
        rng = np.random.Generator(np.random.PCG64(children[c]))
        p = rng.uniform(0.0, 2.0 * math.pi, size=(b - a, 3))
        out[0, a:b] = _store(p, dims)
        for t in range(1, T):
            k1 = _abc(p)
            k2 = _abc(p + 0.5 * dt * k1)
            k3 = _abc(p + 0.5 * dt * k2)
            k4 = _abc(p + dt * k3)
            p = p + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
            out[t, a:b] = _store(p, dims)

    with ThreadPoolExecutor(_workers()) as ex:
        list(ex.map(one, range(nchunk)))
    return out


def _trilinear(ft: np.ndarray, q: np.ndarray) -> np.ndarray:
    Z, Y, X = ft.shape
    s = q.astype(np.float64) - 0.5
    i0 = np.floor(s)
    w = s - i0
    i0 = i0.astype(np.int64)
    lims = (X, Y, Z)
    lo = [np.clip(i0[:, a], 0, lims[a] - 1) for a in range(3)]
    hi = [np.clip(i0[:, a] + 1, 0, lims[a] - 1) for a in range(3)]
    acc = np.zeros(len(q), np.float64)
    for cz in (0, 1):
        zz = hi[2] if cz else lo[2]
        wz = w[:, 2] if cz else 1.0 - w[:, 2]
        for cy in (0, 1):
            yy = hi[1] if cy else lo[1]
            wy = w[:, 1] if cy else 1.0 - w[:, 1]
            for cx in (0, 1):
                xx = hi[0] if cx else lo[0]
                wx = w[:, 0] if cx else 1.0 - w[:, 0]
                acc += wz * wy * wx * ft[zz, yy, xx].astype(np.float64)
    return acc


def sample_attribute(field: np.ndarray, xyz: np.ndarray, rate: int = 1) -> np.ndarray:
    """fp32 [Tp][P]: the field at each stored particle position (trilinear),
    step tau sampled from field step tau // rate."""
    T, P = xyz.shape[0], xyz.shape[1]
    out = np.empty((T, P), np.float32)
    if P == 0:
        return out

    def one(t):
        for a in range(0, P, 1 << 20):
            b = min(P, a + (1 << 20))
            out[t, a:b] = _trilinear(field[t // rate], xyz[t, a:b]).astype(np.float32)

    with ThreadPoolExecutor(_workers()) as ex:
        list(ex.map(one, range(T)))
    return out


def blob_seeds(rng: np.random.Generator, blobs: BlobSet, dims, T: int, S: int,
               distinct: bool = True) -> np.ndarray:
    """int32 [S][4] (x, y, z, t): the voxel holding c_b(t) of S blobs
    (distinct blobs when possible), t ~ U{0..T-1}, clamped into the grid."""
    n = len(blobs)
    if distinct and S <= n:
        bs = rng.choice(n, size=S, replace=False)
    else:
        bs = rng.integers(0, n, size=S)
    ts = rng.integers(0, T, size=S)
    out = np.empty((S, 4), np.int32)
    for k, (b, t) in enumerate(zip(bs, ts)):
        c = np.floor(blobs.centre(int(b), int(t))).astype(np.int64)
        for a in range(3):
            out[k, a] = min(max(c[a], 0), dims[a] - 1)
        out[k, 3] = t
    return out


def make_instance(X: int, Y: int, Z: int, T: int, P: int, *, n_blobs: int = 4,
                  seed: int = 0, n_seeds: int = 1, tau_f: float = 0.3,
                  tau_p: float = 0.3, attr_mode: str = "field",
                  crossing: bool = False, first_seed_blob0_t0: bool = False, rate: int = 1) -> dict:
    """A generic instance of the recipe above, for any grid shape; rate =
    particle steps per field step (the particles hold rate * T steps)."""
    ss = np.random.SeedSequence(seed)
    s_blob, s_noise, s_part, s_seed, s_attr = ss.spawn(5)
    dims = (X, Y, Z)
    blobs = make_blobs(np.random.Generator(np.random.PCG64(s_blob)), n_blobs, dims, T,
                       crossing=crossing)
    field = make_field(blobs, dims, T, s_noise)
    xyz = make_particles(P, dims, rate * T, s_part, dt=0.05 / rate)
    if attr_mode == "field":
        attr = sample_attribute(field, xyz, rate)
    elif attr_mode == "noise":
        attr = np.random.Generator(np.random.PCG64(s_attr)).random((rate * T, P)).astype(np.float32)
    else:
        raise ValueError(attr_mode)
    rng = np.random.Generator(np.random.PCG64(s_seed))
    if first_seed_blob0_t0:
        c = np.floor(blobs.centre(0, 0)).astype(np.int64)
        seeds = np.array([[min(max(c[a], 0), dims[a] - 1) for a in range(3)] + [0]],
                         np.int32)
    else:
        seeds = blob_seeds(rng, blobs, dims, T, n_seeds)
    crit = np.array([tau_f, np.inf, tau_p, np.inf], np.float32)
    return dict(dims=dims, T=T, P=P, field=field, xyz=xyz, attr=attr, seeds=seeds,
                crit=crit, blobs=blobs, seed=seed, rate=rate)


# name -> (X, Y, Z, T, P, blobs, seeds, tau, crossing, data seed)
CONFIGS = {
    1: dict(name="tiny-32^3x8", X=32, Y=32, Z=32, T=8, P=4096, n_blobs=4, n_seeds=1,
            tau=0.3, crossing=False, seed=1),
    2: dict(name="single-128^3x32", X=128, Y=128, Z=128, T=32, P=262144, n_blobs=16,
            n_seeds=8, tau=0.3, crossing=False, seed=2),
    3: dict(name="scale-256^3x64", X=256, Y=256, Z=256, T=64, P=4194304, n_blobs=64,
            n_seeds=32, tau=0.25, crossing=True, seed=3),
}


# A planar (2D + t) city-like workload in the shape of the paper's taxi case
# (about a million grid locations per timestep, tens of thousands of
# vehicles, positions saved more often than the traffic field): 1024 x 1024
# x 1 cells, 48 field steps, 28,672 particles at 4 steps per field step; 1,024
# crossing blobs stand in for congestion, threshold 0.2 (about 10% of the
# cells), 32 seeds.
CITY = dict(name="city-2d-1024^2x48-r4", X=1024, Y=1024, Z=1, T=48, rate=4, P=28672, n_blobs=1024,
            n_seeds=32, tau=0.2, crossing=True, seed=4)


def make_city(**kw) -> dict:
    """The planar city-like workload above (keyword arguments override).
    Particles lie on the layer's mid-plane (z = 0.5, like the field samples'
    voxel centres), so the clustering's z differences vanish, as in a 2D + t
    method without a z coordinate."""
    c = dict(CITY, **kw)
    inst = make_instance(c["X"], c["Y"], c["Z"], c["T"], c["P"], n_blobs=c["n_blobs"], seed=c["seed"],
                         n_seeds=c["n_seeds"], tau_f=c["tau"], tau_p=c["tau"], crossing=c["crossing"],
                         rate=c["rate"])
    if c["Z"] == 1:
        inst["xyz"][..., 2] = np.float32(0.5)
    return inst


def make_config(k: int, *, attr_mode: str = "field", tau_p_offset: float = 0.0,
                T: int | None = None, P: int | None = None) -> dict:
    """Configurations 1-3 of the workload table (config 4 is config 2's data
    plus make_queries; config 5 is config 3's data).  T and P may be cut for
    bounded samples of the same workload (fewer timesteps / particles)."""
    c = CONFIGS[k]
    return make_instance(c["X"], c["Y"], c["Z"], c["T"] if T is None else T,
                         c["P"] if P is None else P, n_blobs=c["n_blobs"],
                         seed=c["seed"], n_seeds=c["n_seeds"], tau_f=c["tau"],
                         tau_p=c["tau"] + tau_p_offset, attr_mode=attr_mode,
                         crossing=c["crossing"], first_seed_blob0_t0=(k == 1))


def make_queries(inst: dict, Q: int = 256, seed: int = 4, max_seeds: int = 16,
                 jitter: int = 2, lo: float = 0.15, hi: float = 0.6):
    """Batched queries: per query n ~ U{1..max_seeds} seeds at the voxel of a
    random blob centre c_b(t) plus a U{-jitter..jitter}^3 offset, clamped; the
    field and attribute thresholds ~ U[lo, hi] independently.
    Returns (crit fp32 [Q][4] = (f_lo, f_hi, a_lo, a_hi), seeds int32 [S][5] =
    (x, y, z, t, q))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    blobs, dims, T = inst["blobs"], inst["dims"], inst["T"]
    crit = np.empty((Q, 4), np.float32)
    crit[:, 0] = rng.uniform(lo, hi, size=Q).astype(np.float32)
    crit[:, 1] = np.inf
    crit[:, 2] = rng.uniform(lo, hi, size=Q).astype(np.float32)
    crit[:, 3] = np.inf
    rows = []
    for q in range(Q):
        n = int(rng.integers(1, max_seeds + 1))
        for _ in range(n):
            b = int(rng.integers(0, len(blobs)))
            t = int(rng.integers(0, T))
            c = np.floor(blobs.centre(b, t)).astype(np.int64)
            c = c + rng.integers(-jitter, jitter + 1, size=3)
            rows.append([min(max(int(c[a]), 0), dims[a] - 1) for a in range(3)] + [t, q])
    return crit, np.asarray(rows, np.int32).reshape(-1, 5)
