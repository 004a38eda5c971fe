"""4D SLIC clustering of point and field samples (Section 3.2), the oracle.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product library.  Plain numpy,
slow, written for a reader who checks it against the paper.

What it computes (Section 3.2.1-3.2.3; the readings that fix what the paper
leaves open are marked R and listed in the design notes):

  samples   one field sample per voxel-step: position (x+0.5, y+0.5, z+0.5)
            (R: the voxel centre), time t, value f; one point sample per
            particle-step: its position, time tau / r in field steps (fp32;
            r particle steps per field step, Section 3.4 on different
            temporal resolutions; r = 1: time t), value a.  A sample with a
            non-finite position or value is not clustered (label -1) (R).
  seeding   k = (kx, ky, kz, kt) centres on a 4D rectilinear grid, interval
            C_d = E_d / k_d with E = (X, Y, Z, T) (Section 3.2.1), in fp32.
            The seed cell of a sample is floor(pos_d / C_d) clamped to
            [0, k_d - 1]; centre id = ((ct*kz + cz)*ky + cy)*kx + cx.
            A seed centre sits at ((i + 0.5) C_d) with values 0 (R).
  initial   every sample goes to the nearest seed centre, which on a
            rectilinear grid under the (diagonal) space-time metric is its
            seed cell's centre (Section 3.2.1).
  update    a centre is the mean of its samples (Section 3.2.2): location over
            both types, f_c over field samples, p_c over point samples.  R:
            sums are exact integer sums of q(v) = rint(v * 2^20) (so the order
            of summation cannot matter), and mean = dbl(sum) / n * 2^-20 with
            dbl(s) = float64(s >> 32) * 2^32 + float64(s & 0xffffffff).  A
            centre without samples keeps its previous location and values; one
            without samples of a type keeps that type's previous value.
  assign    each centre searches the 2C_1 x 2C_2 x 2C_3 x 2C_4 window around
            itself (Section 3.2.2), the samples with |pos_d - c_d| <= C_d on
            every axis (fp32 difference, c_d the centre rounded to fp32), and
            rates them by D_f or D_p (Section 3.2.3) with S_st of Section
            3.2.1:
              S = sqrt(((dx*dx + dy*dy) + dz*dz) + (cf*dt)*(cf*dt))
              D = w_v*|v - v_c| + w_d*S
            in IEEE fp32, in that order (R), dx = x_s - x_c and so on.  A
            sample takes the centre with the smallest D among those whose
            window holds it, ties to the lowest id (R); a sample no window
            holds keeps its label (R).  Every centre is searched: a centre
            that drifted far from its seed cell still claims the samples of
            its window.
  converge  after the centres of an iteration are computed, the loop stops
            when every one of the six values of every centre changed by at
            most eps * |old| (R: the "percent change" of Section 3.2.2 read as
            a relative change, in fp64) -- or after max_iter assignments.
"""
from __future__ import annotations

import numpy as np

Q_BITS = 20
Q_SCALE = float(1 << Q_BITS)
F32 = np.float32


def grid_interval(dims_xyzt, k):
    """C_d = E_d / k_d in fp32 (Section 3.2.1)."""
    return np.array([F32(e) / F32(kk) for e, kk in zip(dims_xyzt, k)], dtype=F32)


def seed_cell(pos, C, kd):
    """floor(pos / C) clamped to [0, kd - 1], fp32 division."""
    c = np.floor((pos.astype(F32) / F32(C)).astype(F32))
    c = np.where(np.isnan(c), 0, c)  # non-finite samples are not clustered; any cell will do
    return np.clip(c, 0, kd - 1).astype(np.int64)


def centre_id(cx, cy, cz, ct, k):
    kx, ky, kz, _ = k
    return ((ct * kz + cz) * ky + cy) * kx + cx


def quantise(v):
    """q(v) = rint(v * 2^20) as an exact integer (v fp32 -> fp64 is exact)."""
    return np.rint(np.asarray(v, np.float64) * Q_SCALE).astype(np.int64)


def to_double(s):
    """dbl(s) = float64(s >> 32) * 2^32 + float64(s & 0xffffffff)."""
    s = np.asarray(s, np.int64)
    hi = (s >> 32).astype(np.float64)
    lo = (s & 0xFFFFFFFF).astype(np.float64)
    return hi * 4294967296.0 + lo


def samples(field, xyz, attr, rate=1):
    """Flatten both sample types: positions (fp32 [n][3]), times (fp32 [n],
    in field steps), values (fp32 [n]), type (0 field, 1 point), validity."""
    T, Z, Y, X = field.shape
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    fpos = np.stack([x.ravel() + 0.5, y.ravel() + 0.5, z.ravel() + 0.5], 1).astype(F32)
    ft = t.ravel().astype(F32)
    fv = field.ravel().astype(F32)
    P = attr.shape[1] if attr is not None else 0
    if P:
        Tp = attr.shape[0]
        ppos = xyz.reshape(Tp * P, 3).astype(F32)
        pt = np.repeat((np.arange(Tp, dtype=F32) / F32(rate)).astype(F32), P)
        pv = attr.reshape(Tp * P).astype(F32)
    else:
        ppos = np.zeros((0, 3), F32)
        pt = np.zeros(0, F32)
        pv = np.zeros(0, F32)
    pos = np.concatenate([fpos, ppos])
    tt = np.concatenate([ft, pt])
    val = np.concatenate([fv, pv])
    typ = np.concatenate([np.zeros(len(fv), np.int64), np.ones(len(pv), np.int64)])
    valid = np.isfinite(val) & np.all(np.isfinite(pos), axis=1)
    return pos, tt, val, typ, valid


def seed_centres(C, k):
    """Seed centres: location ((i + 0.5) C_d), values 0; [K][6] fp64 as
    (x, y, z, t, p, f)."""
    kx, ky, kz, kt = k
    K = kx * ky * kz * kt
    cen = np.zeros((K, 6), np.float64)
    for ct in range(kt):
        for cz in range(kz):
            for cy in range(ky):
                for cx in range(kx):
                    i = centre_id(cx, cy, cz, ct, k)
                    cen[i, 0] = float(F32(cx + 0.5) * C[0])
                    cen[i, 1] = float(F32(cy + 0.5) * C[1])
                    cen[i, 2] = float(F32(cz + 0.5) * C[2])
                    cen[i, 3] = float(F32(ct + 0.5) * C[3])
    return cen


def initial_labels(pos, tt, valid, C, k):
    """Nearest seed centre = the seed cell's centre."""
    cx = seed_cell(pos[:, 0], C[0], k[0])
    cy = seed_cell(pos[:, 1], C[1], k[1])
    cz = seed_cell(pos[:, 2], C[2], k[2])
    ct = seed_cell(tt.astype(F32), C[3], k[3])
    lab = centre_id(cx, cy, cz, ct, k)
    return np.where(valid, lab, -1)


def update_centres(pos, tt, val, typ, lab, prev, K):
    """Means of the assigned samples from exact integer sums (see header).
    Returns the new [K][6] centres and the counts [K][2] (field, point)."""
    m = lab >= 0
    ids = lab[m]
    qx, qy, qz = quantise(pos[m, 0]), quantise(pos[m, 1]), quantise(pos[m, 2])
    qt = quantise(tt[m])
    qv = quantise(val[m])
    isf = typ[m] == 0

    def isum(w, sel=None):
        # exact in int64 while |sum| < 2^63, which the bounds on dimensions and
        # values guarantee (fewer than 2^31 samples of |q| < 2^31)
        idx = ids if sel is None else ids[sel]
        ww = w if sel is None else w[sel]
        acc = np.zeros(K, np.int64)
        np.add.at(acc, idx, ww)
        return acc

    n_all = np.bincount(ids, minlength=K).astype(np.int64)
    n_f = np.bincount(ids[isf], minlength=K).astype(np.int64)
    n_p = n_all - n_f
    sx, sy, sz, st = isum(qx), isum(qy), isum(qz), isum(qt)
    sf = isum(qv, isf)
    sp = isum(qv, ~isf)
    cen = prev.copy()
    for j, s in enumerate((sx, sy, sz, st)):
        has = n_all > 0
        cen[has, j] = to_double(s[has]) / n_all[has].astype(np.float64) / Q_SCALE
    hp = n_p > 0
    cen[hp, 4] = to_double(sp[hp]) / n_p[hp].astype(np.float64) / Q_SCALE
    hf = n_f > 0
    cen[hf, 5] = to_double(sf[hf]) / n_f[hf].astype(np.float64) / Q_SCALE
    return cen, np.stack([n_f, n_p], 1)


def _distance(pos, ts, val, typ, cc, wv, wd, cf):
    """D of samples against one centre cc (fp32 [6] as x, y, z, t, p, f), in
    the fixed fp32 order of the header; also the window test."""
    dx = (pos[:, 0] - cc[0]).astype(F32)
    dy = (pos[:, 1] - cc[1]).astype(F32)
    dz = (pos[:, 2] - cc[2]).astype(F32)
    dt = (ts - cc[3]).astype(F32)
    vc = np.where(typ == 0, cc[5], cc[4]).astype(F32)
    ctd = (cf * dt).astype(F32)
    sq = (((dx * dx + dy * dy).astype(F32) + dz * dz).astype(F32) + ctd * ctd).astype(F32)
    S = np.sqrt(sq).astype(F32)
    D = (wv * np.abs((val - vc).astype(F32)) + wd * S).astype(F32)
    return dx, dy, dz, dt, D


def assign(pos, tt, val, typ, lab, cen, C, k, w, cf):
    """One assignment pass (Section 3.2.2-3.2.3, fp32 as in the header),
    centre by centre as the paper describes it: centre i, in id order, rates
    every sample inside its window and takes those it rates strictly better
    than any earlier centre did (so ties stay with the lowest id).  Samples
    are indexed by x so that a centre only looks at the slab of samples its
    window can reach; the window test itself is the exact fp32 one.
    w = (w_d, w_f, w_p); k is unused (the search does not depend on the seed
    grid)."""
    wd, wf, wp = F32(w[0]), F32(w[1]), F32(w[2])
    cf = F32(cf)
    c32 = cen.astype(F32)
    C = np.asarray(C, F32)
    n = len(val)
    best_d = np.full(n, np.inf, F32)
    best_i = np.full(n, -1, np.int64)
    ts = tt.astype(F32)
    wv = np.where(typ == 0, wf, wp).astype(F32)
    live = lab >= 0
    order = np.argsort(np.where(live, pos[:, 0], np.inf).astype(np.float64), kind="stable")
    xs = np.where(live, pos[:, 0], np.inf).astype(np.float64)[order]
    for i in range(len(cen)):
        cc = c32[i]
        # every sample with |fl(x - c_x)| <= C_x lies within C_x (1 + 2^-23)
        # of c_x, so this slab holds them all; the exact test follows
        r = float(C[0]) * (1.0 + 2.0 ** -20) + 2.0 ** -20 * abs(float(cc[0]))
        a = np.searchsorted(xs, float(cc[0]) - r, side="left")
        b = np.searchsorted(xs, float(cc[0]) + r, side="right")
        if a >= b:
            continue
        idx = order[a:b]
        # the window test on y, z, t first (the same fp32 differences), then
        # the distances of the samples inside
        idx = idx[(np.abs((pos[idx, 1] - cc[1]).astype(F32)) <= C[1]) &
                  (np.abs((pos[idx, 2] - cc[2]).astype(F32)) <= C[2]) &
                  (np.abs((ts[idx] - cc[3]).astype(F32)) <= C[3])]
        dx, dy, dz, dt, D = _distance(pos[idx], ts[idx], val[idx], typ[idx], cc, wv[idx], wd, cf)
        inwin = ((np.abs(dx) <= C[0]) & (np.abs(dy) <= C[1]) & (np.abs(dz) <= C[2]) &
                 (np.abs(dt) <= C[3]))
        better = inwin & (D < best_d[idx])
        sel = idx[better]
        best_d[sel] = D[better]
        best_i[sel] = i
    out = np.where(best_i >= 0, best_i, lab)
    return np.where(live, out, -1)


def assign_brute(pos, tt, val, typ, lab, cen, C, w, cf, chunk=256):
    """The same pass sample by sample: every sample against every centre
    (brute force over K, numpy argmin takes the lowest id among equal D).
    An independent formulation of `assign`, used to pin it and to check
    sampled labels at sizes where `assign` would take long."""
    wd, wf, wp = F32(w[0]), F32(w[1]), F32(w[2])
    cf = F32(cf)
    c32 = cen.astype(F32)
    C = np.asarray(C, F32)
    out = np.array(lab, np.int64, copy=True)
    ts = tt.astype(F32)
    for s0 in range(0, len(val), chunk):
        sl = slice(s0, min(len(val), s0 + chunk))
        p = pos[sl].astype(F32)[:, None, :]
        d = (p - c32[None, :, :3]).astype(F32)
        dt = (ts[sl][:, None] - c32[None, :, 3]).astype(F32)
        inwin = (np.all(np.abs(d) <= C[None, None, :3], axis=2) & (np.abs(dt) <= C[3]))
        vc = np.where((typ[sl] == 0)[:, None], c32[None, :, 5], c32[None, :, 4]).astype(F32)
        wv = np.where(typ[sl] == 0, wf, wp).astype(F32)[:, None]
        ctd = (cf * dt).astype(F32)
        sq = (((d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]).astype(F32) + d[..., 2] * d[..., 2]).astype(F32)
              + ctd * ctd).astype(F32)
        D = (wv * np.abs((val[sl][:, None] - vc).astype(F32)) + wd * np.sqrt(sq).astype(F32)).astype(F32)
        D = np.where(inwin, D, np.inf).astype(F32)
        j = np.argmin(D, axis=1)
        has = inwin.any(axis=1)
        out[sl] = np.where(has & (out[sl] >= 0), j, out[sl])
    return out


def converged(new, old, eps):
    """Every value changed by at most eps * |old| (fp64)."""
    return bool(np.all(np.abs(new - old) <= eps * np.abs(old)))


def slic(field, xyz, attr, k, w, cf, eps, max_iter, rate=1):
    """The whole clustering.  field fp32 [T][Z][Y][X]; xyz fp32 [Tp][P][3] and
    attr fp32 [Tp][P] (or None), rate particle steps per field step; k = (kx,
    ky, kz, kt); w = (w_d, w_f, w_p).  Returns (field labels int64
    [T][Z][Y][X], point labels int64 [Tp][P], centres fp64 [K][6] as (x, y,
    z, t, p, f), counts [K][2], iterations)."""
    T, Z, Y, X = field.shape
    k = tuple(int(v) for v in k)
    K = k[0] * k[1] * k[2] * k[3]
    C = grid_interval((X, Y, Z, T), k)
    pos, tt, val, typ, valid = samples(field, xyz, attr, rate)
    lab = initial_labels(pos, tt, valid, C, k)
    prev = seed_centres(C, k)
    it = 0
    while True:
        cen, counts = update_centres(pos, tt, val, typ, lab, prev, K)
        if (it > 0 and converged(cen, prev, eps)) or it == max_iter:
            break
        lab = assign(pos, tt, val, typ, lab, cen, C, k, w, cf)
        prev = cen
        it += 1
    V = X * Y * Z * T
    fl = lab[:V].reshape(T, Z, Y, X)
    P = attr.shape[1] if attr is not None else 0
    pl = lab[V:].reshape(attr.shape[0] if attr is not None else T, P)
    return fl, pl, cen, counts, it


# ---- cluster merging and feature statistics (Section 3.3) -------------------
#
#   match     two centres match when, for each sample type, either neither has
#             samples of it or both do and their means differ by at most
#             eps_m * max(|a|, |b|) (R: the "percent difference" of Section
#             3.3, relative to the larger magnitude); a centre without samples
#             matches nothing (R).  Location is ignored (Section 3.3).
#   merge     features are the connected components of "match" (R: merging is
#             transitive), each named by its lowest centre id.
#   stats     per feature: field and point sample counts; mean field and point
#             values from the exact integer sums of the update (same formula);
#             population standard deviations of the field and point values
#             (fp64); extent: least and greatest x, y, z, t of its samples.


def _matches(a, b, eps):
    return np.abs(a - b) <= eps * np.maximum(np.abs(a), np.abs(b))


def merge_centres(cen, counts, eps_m):
    """Feature id (lowest centre id of its component) of every centre; -1 for
    a centre without samples.  The match relation is evaluated row block by
    row block; its transitive closure is scipy's connected components."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    K = len(cen)
    nf, npt = counts[:, 0], counts[:, 1]
    has = (nf + npt) > 0
    rows, cols = [], []
    for i0 in range(0, K, 1024):
        i = np.arange(i0, min(K, i0 + 1024))[:, None]
        j = np.arange(K)[None, :]
        ok = has[i] & has[j] & (j > i)
        for col, n in ((5, nf), (4, npt)):
            both = (n[i] > 0) & (n[j] > 0)
            none = (n[i] == 0) & (n[j] == 0)
            ok &= none | (both & _matches(cen[i, col], cen[j, col], eps_m))
        r, c = np.nonzero(ok)
        rows.append(r + i0)
        cols.append(c)
    r = np.concatenate(rows) if rows else np.zeros(0, np.int64)
    c = np.concatenate(cols) if cols else np.zeros(0, np.int64)
    g = coo_matrix((np.ones(len(r), np.int8), (r, c)), shape=(K, K))
    _, comp = connected_components(g, directed=False)
    low = np.full(comp.max() + 1 if K else 0, K, np.int64)
    np.minimum.at(low, comp, np.arange(K))
    return np.where(has, low[comp], -1).astype(np.int64)


def feature_stats(field, xyz, attr, fl, pl, feat, rate=1):
    """Per feature id (indexed by its lowest centre id, [K] rows; rows of
    non-features are zero): n_f, n_p, mean f, mean p, std f, std p, then
    x min, x max, y min, y max, z min, z max, t min, t max.  fp64 [K][14]."""
    K = len(feat)
    pos, tt, val, typ, valid = samples(field, xyz, attr, rate)
    lab = np.concatenate([fl.ravel(), pl.ravel()]) if pl is not None else fl.ravel()
    m = lab >= 0
    F = feat[lab[m]]
    pos, tt, val, typ = pos[m], tt[m], val[m], typ[m]
    out = np.zeros((K, 14), np.float64)
    qv = quantise(val)
    for ty, (cn, cm, cs) in ((0, (0, 2, 4)), (1, (1, 3, 5))):
        sel = typ == ty
        n = np.bincount(F[sel], minlength=K).astype(np.int64)
        s = np.zeros(K, np.int64)
        np.add.at(s, F[sel], qv[sel])
        mean = np.where(n > 0, to_double(s) / np.maximum(n, 1).astype(np.float64) / Q_SCALE, 0.0)
        dev = val[sel].astype(np.float64) - mean[F[sel]]
        ss = np.zeros(K, np.float64)
        np.add.at(ss, F[sel], dev * dev)
        out[:, cn] = n
        out[:, cm] = mean
        out[:, cs] = np.where(n > 0, np.sqrt(ss / np.maximum(n, 1)), 0.0)
    coords = [pos[:, 0], pos[:, 1], pos[:, 2], tt.astype(np.float32)]
    for d, c in enumerate(coords):
        lo = np.full(K, np.inf)
        hi = np.full(K, -np.inf)
        np.minimum.at(lo, F, c.astype(np.float64))
        np.maximum.at(hi, F, c.astype(np.float64))
        has = (out[:, 0] + out[:, 1]) > 0
        out[:, 6 + 2 * d] = np.where(has, lo, 0.0)
        out[:, 7 + 2 * d] = np.where(has, hi, 0.0)
    return out
