"""Pins of the 4D SLIC oracle (Section 3.2) against closed forms, hand-placed
configurations and independent re-computations (fp64 means by bincount, the
distance metric in fp64), so that a dropped term, a wrong window, a wrong
weight or a wrong mean fails here."""
import numpy as np
import pytest

from oracle import slic as S

F32 = np.float32


def rand_case(seed, T=4, Z=4, Y=8, X=8, P=30):
    rng = np.random.default_rng(seed)
    field = rng.random((T, Z, Y, X), dtype=F32)
    xyz = (rng.random((T, P, 3)) * np.array([X, Y, Z])).astype(F32)
    attr = rng.random((T, P), dtype=F32)
    return field, xyz, attr


def test_one_centre_is_the_global_mean():
    """k = (1,1,1,1): every sample in centre 0, whose location and values are
    the plain means (Section 3.2.2), up to the 2^-20 quantisation."""
    field, xyz, attr = rand_case(1)
    T, Z, Y, X = field.shape
    fl, pl, cen, cnt, it = S.slic(field, xyz, attr, (1, 1, 1, 1), (1.0, 1.0, 1.0), 1.0, 1e-9, 5)
    assert (fl == 0).all() and (pl == 0).all()
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    mx = np.concatenate([(x + 0.5).ravel(), xyz[..., 0].ravel().astype(np.float64)]).mean()
    mz = np.concatenate([(z + 0.5).ravel(), xyz[..., 2].ravel().astype(np.float64)]).mean()
    mt = np.concatenate([t.ravel(), np.repeat(np.arange(T), xyz.shape[1])]).mean()
    assert abs(cen[0, 0] - mx) < 1e-6 and abs(cen[0, 2] - mz) < 1e-6 and abs(cen[0, 3] - mt) < 1e-9
    assert abs(cen[0, 4] - attr.astype(np.float64).mean()) < 1e-6
    assert abs(cen[0, 5] - field.astype(np.float64).mean()) < 1e-6
    assert cnt[0].tolist() == [field.size, attr.size]


def test_uniform_grid_stays_on_its_cells():
    """Value weights 0, field only, C_d dividing E_d: every centre is its
    cell's centroid and every voxel's nearest centre is its own cell's, so
    the first assignment changes nothing and the loop stops after it."""
    T, Z, Y, X = 4, 4, 8, 8
    field = np.random.default_rng(2).random((T, Z, Y, X), dtype=F32)
    k = (2, 2, 2, 2)
    fl, pl, cen, cnt, it = S.slic(field, None, None, k, (1.0, 0.0, 0.0), 1.0, 0.0, 10)
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    want = ((t // 2 * 2 + z // 2) * 2 + y // 4) * 2 + x // 4
    assert (fl == want).all()
    assert it == 1
    # centroid of cell (0,0,0,0): x in 0.5..3.5, t in {0, 1}
    assert cen[0, 0] == 2.0 and cen[0, 1] == 2.0 and cen[0, 2] == 1.0 and cen[0, 3] == 0.5


def _assign_by_hand(points, values, centres, C, k, w, cf):
    """One point-sample assignment computed with plain float64 loops over
    every centre (no seed-cell search), the window |d| <= C_d per axis."""
    out = []
    for (x, y, z, t), v in zip(points, values):
        best = None
        for i, c in enumerate(centres):
            d = np.array([x - c[0], y - c[1], z - c[2], t - c[3]])
            if np.any(np.abs(d) > np.asarray(C, np.float64)):
                continue
            S_st = np.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2 + (cf * d[3]) ** 2)
            D = w[2] * abs(v - c[4]) + w[0] * S_st
            if best is None or D < best[0]:
                best = (D, i)
        out.append(best[1] if best else -2)
    return out


def _assign_oracle(points, values, centres, C, k, w, cf, prev=None):
    pos = np.asarray([p[:3] for p in points], F32)
    tt = np.asarray([p[3] for p in points], np.int64)
    val = np.asarray(values, F32)
    typ = np.ones(len(values), np.int64)
    lab = np.zeros(len(values), np.int64) if prev is None else np.asarray(prev)
    return S.assign(pos, tt, val, typ, lab, np.asarray(centres, np.float64), np.asarray(C, F32), k, w, cf).tolist()


def test_window_half_width_is_C_and_value_term_counts():
    """Two centres along x (C_x = 4): a point 4.1 from centre 1 is outside its
    window even with a perfect value match; at 3.5 it is inside and the value
    term (w_p large) decides for centre 1 although centre 0 is nearer."""
    C = (4.0, 8.0, 8.0, 8.0)
    k = (2, 1, 1, 1)
    cen = [[2.0, 4.0, 4.0, 4.0, 0.0, 0.0], [6.0, 4.0, 4.0, 4.0, 1.0, 0.0]]
    w = (1.0, 0.0, 100.0)
    pts = [(1.9, 4.0, 4.0, 4), (2.5, 4.0, 4.0, 4), (2.5, 4.0, 4.0, 4)]
    vals = [1.0, 1.0, 0.0]
    assert _assign_oracle(pts, vals, cen, C, k, w, 1.0) == [0, 1, 0]
    assert _assign_by_hand(pts, vals, cen, C, k, w, 1.0) == [0, 1, 0]


def test_time_factor_scales_the_time_distance():
    """Centres at the same place, one and three timesteps away: with c_f = 0
    they tie (lowest id wins); with c_f > 0 the nearer in time wins."""
    C = (8.0, 8.0, 8.0, 4.0)
    k = (1, 1, 1, 2)
    cen = [[4.0, 4.0, 4.0, 1.0, 0.0, 0.0], [4.0, 4.0, 4.0, 5.0, 0.0, 0.0]]
    pts = [(4.0, 4.0, 4.0, 4)]
    assert _assign_oracle(pts, [0.0], cen, C, k, (1.0, 0.0, 0.0), 0.0) == [0]
    assert _assign_oracle(pts, [0.0], cen, C, k, (1.0, 0.0, 0.0), 1.0) == [1]
    assert _assign_by_hand(pts, [0.0], cen, C, k, (1.0, 0.0, 0.0), 1.0) == [1]


def test_no_candidate_keeps_the_label():
    C = (1.0, 1.0, 1.0, 1.0)
    cen = [[0.5, 0.5, 0.5, 0.5, 0.0, 0.0]]
    assert _assign_oracle([(3.0, 3.0, 3.0, 3)], [0.0], cen, C, (1, 1, 1, 1), (1.0, 0.0, 0.0), 1.0,
                          prev=[7]) == [7]


@pytest.mark.parametrize("seed", [3, 4, 5])
def test_assignment_is_the_metric_minimum(seed):
    """Every assigned sample's own centre has the smallest D (fp64 re-computed
    over the same candidate centres) up to fp32 rounding."""
    field, xyz, attr = rand_case(seed, P=60)
    T, Z, Y, X = field.shape
    k = (2, 2, 2, 2)
    w = (1.0, 3.0, 2.0)
    cf = 0.7
    C = S.grid_interval((X, Y, Z, T), k)
    pos, tt, val, typ, valid = S.samples(field, xyz, attr)
    lab = S.initial_labels(pos, tt, valid, C, k)
    cen, _ = S.update_centres(pos, tt, val, typ, lab, S.seed_centres(C, k), 16)
    new = S.assign(pos, tt, val, typ, lab, cen, C, k, w, cf)
    c32 = cen.astype(F32).astype(np.float64)
    p64 = pos.astype(np.float64)
    for i in range(0, len(val), 7):
        d = p64[i] - c32[:, :3]
        dt = tt[i] - c32[:, 3]
        inwin = np.all(np.abs(d) <= C[:3].astype(np.float64), 1) & (np.abs(dt) <= float(C[3]))
        S_st = np.sqrt((d ** 2).sum(1) + (cf * dt) ** 2)
        vc = c32[:, 5] if typ[i] == 0 else c32[:, 4]
        D = (w[1] if typ[i] == 0 else w[2]) * np.abs(float(val[i]) - vc) + w[0] * S_st
        assert inwin[new[i]]
        assert D[new[i]] <= D[inwin].min() + 1e-4 * (1 + D[inwin].min())


@pytest.mark.parametrize("seed", [6, 7])
def test_centres_are_member_means(seed):
    """After a run, each non-empty centre is the mean of its members (fp64,
    by bincount), to within the 2^-20 quantisation."""
    field, xyz, attr = rand_case(seed, P=40)
    fl, pl, cen, cnt, it = S.slic(field, xyz, attr, (2, 2, 1, 2), (1.0, 2.0, 2.0), 0.5, 1e-6, 6)
    T, Z, Y, X = field.shape
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    lab = np.concatenate([fl.ravel(), pl.ravel()])
    xs = np.concatenate([(x + 0.5).ravel(), xyz[..., 0].ravel().astype(np.float64)])
    ts = np.concatenate([t.ravel(), np.repeat(np.arange(T), xyz.shape[1])]).astype(np.float64)
    K = 8
    n = np.bincount(lab, minlength=K)
    mx = np.bincount(lab, xs, minlength=K) / np.maximum(n, 1)
    mt = np.bincount(lab, ts, minlength=K) / np.maximum(n, 1)
    nf = np.bincount(fl.ravel(), minlength=K)
    mf = np.bincount(fl.ravel(), field.ravel().astype(np.float64), minlength=K) / np.maximum(nf, 1)
    np_ = np.bincount(pl.ravel(), minlength=K)
    mp = np.bincount(pl.ravel(), attr.ravel().astype(np.float64), minlength=K) / np.maximum(np_, 1)
    for c in range(K):
        if n[c]:
            assert abs(cen[c, 0] - mx[c]) < 1e-6 and abs(cen[c, 3] - mt[c]) < 1e-6
        if nf[c]:
            assert abs(cen[c, 5] - mf[c]) < 1e-6
        if np_[c]:
            assert abs(cen[c, 4] - mp[c]) < 1e-6
    assert (cnt[:, 0] == nf).all() and (cnt[:, 1] == np_).all()


def test_non_finite_samples_are_not_clustered():
    field, xyz, attr = rand_case(8, P=10)
    field[0, 0, 0, 0] = np.nan
    xyz[1, 2, 0] = np.inf
    attr[2, 3] = np.nan
    fl, pl, cen, cnt, it = S.slic(field, xyz, attr, (2, 1, 1, 1), (1.0, 1.0, 1.0), 1.0, 1e-6, 3)
    assert fl[0, 0, 0, 0] == -1 and pl[1, 2] == -1 and pl[2, 3] == -1
    assert cnt[:, 0].sum() == field.size - 1 and cnt[:, 1].sum() == attr.size - 2


def test_fixed_point_means_are_order_free():
    """Exact integer sums: permuting the samples leaves the centres bit-equal."""
    rng = np.random.default_rng(9)
    pos = rng.random((500, 3)).astype(F32) * 8
    tt = rng.integers(0, 4, 500)
    val = rng.random(500).astype(F32)
    typ = rng.integers(0, 2, 500)
    lab = rng.integers(0, 4, 500)
    prev = np.zeros((4, 6))
    a, _ = S.update_centres(pos, tt, val, typ, lab, prev, 4)
    p = rng.permutation(500)
    b, _ = S.update_centres(pos[p], tt[p], val[p], typ[p], lab[p], prev, 4)
    assert a.tobytes() == b.tobytes()


def test_empty_centre_keeps_its_values():
    pos = np.array([[1.0, 1.0, 1.0]], F32)
    prev = np.array([[9.0, 9.0, 9.0, 9.0, 5.0, 6.0], [1.0, 1.0, 1.0, 1.0, 2.0, 3.0]])
    cen, cnt = S.update_centres(pos, np.array([2]), np.array([0.5], F32), np.array([0]), np.array([1]), prev, 2)
    assert (cen[0] == prev[0]).all()  # no samples
    assert cen[1, 4] == 2.0           # no point samples: p_c kept
    assert cen[1, 5] == 0.5 and cen[1, 0] == 1.0 and cen[1, 3] == 2.0


# ---- cluster merging and feature statistics (Section 3.3) ----

def _cen(rows):
    """centres from (f, p, n_f, n_p) rows"""
    cen = np.zeros((len(rows), 6))
    cnt = np.zeros((len(rows), 2), np.int64)
    for i, (f, p, nf, np_) in enumerate(rows):
        cen[i, 5], cen[i, 4], cnt[i] = f, p, (nf, np_)
    return cen, cnt


def test_merge_is_transitive_and_named_by_lowest_id():
    """1.00 ~ 1.09 ~ 1.18 at eps 0.1 (relative to the larger value), 1.00 and
    1.18 do not match directly but share a feature; 5.0 stays alone."""
    cen, cnt = _cen([(1.18, 0.0, 4, 0), (5.0, 0.0, 4, 0), (1.00, 0.0, 4, 0), (1.09, 0.0, 4, 0)])
    assert S.merge_centres(cen, cnt, 0.1).tolist() == [0, 1, 0, 0]
    assert S.merge_centres(cen, cnt, 0.0).tolist() == [0, 1, 2, 3]


def test_merge_needs_both_types_to_match():
    """Same field mean, point means apart: no merge; a centre with no point
    samples never merges with one that has them; empty centres never merge."""
    cen, cnt = _cen([(1.0, 0.2, 3, 3), (1.0, 0.9, 3, 3), (1.0, 0.2, 3, 0), (1.0, 0.2, 0, 0), (1.0, 0.21, 2, 2)])
    assert S.merge_centres(cen, cnt, 0.1).tolist() == [0, 1, 2, -1, 0]


def test_feature_stats_match_numpy_per_feature():
    field, xyz, attr = rand_case(12, P=25)
    fl, pl, cen, cnt, it = S.slic(field, xyz, attr, (2, 2, 2, 2), (1.0, 2.0, 2.0), 0.5, 1e-6, 4)
    feat = S.merge_centres(cen, cnt, 0.15)
    st = S.feature_stats(field, xyz, attr, fl, pl, feat)
    T, Z, Y, X = field.shape
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    ff = feat[fl.ravel()]
    fp = feat[pl.ravel()]
    for F in np.unique(feat[feat >= 0]):
        mf = ff == F
        mp = fp == F
        assert st[F, 0] == mf.sum() and st[F, 1] == mp.sum()
        if mf.any():
            fv = field.ravel()[mf].astype(np.float64)
            assert abs(st[F, 2] - fv.mean()) < 1e-6 and abs(st[F, 4] - fv.std()) < 1e-6
        if mp.any():
            pv = attr.ravel()[mp].astype(np.float64)
            assert abs(st[F, 3] - pv.mean()) < 1e-6 and abs(st[F, 5] - pv.std()) < 1e-6
        xs = np.concatenate([(x + 0.5).ravel()[mf], xyz[..., 0].ravel()[mp]])
        ts = np.concatenate([t.ravel()[mf], np.repeat(np.arange(T), xyz.shape[1])[mp]])
        assert st[F, 6] == xs.min() and st[F, 7] == xs.max()
        assert st[F, 12] == ts.min() and st[F, 13] == ts.max()
    assert st[:, 0].sum() == field.size and st[:, 1].sum() == attr.size


def test_every_centre_is_searched_hand_placed():
    """Section 3.2.2: a centre searches the 2C window around itself wherever
    it has moved.  Four centres along x (C_x = 2); centre 3, seeded in the
    last cell, has drifted into the first cells, where a sample of cell 0
    lies within C_x of it.  Its value matches the sample's, so with a large
    value weight it wins over the near centres 0 and 1 -- although its seed
    cell is three cells from the sample's."""
    C = (2.0, 8.0, 8.0, 8.0)
    k = (4, 1, 1, 1)
    cen = [[1.0, 4.0, 4.0, 4.0, 0.0, 0.0], [3.0, 4.0, 4.0, 4.0, 0.2, 0.0],
           [5.0, 4.0, 4.0, 4.0, 0.3, 0.0], [2.5, 4.0, 4.0, 4.0, 0.9, 0.0]]
    w = (0.1, 0.0, 10.0)
    pts = [(1.5, 4.0, 4.0, 4), (1.5, 4.0, 4.0, 4), (6.9, 4.0, 4.0, 4)]
    vals = [0.9, 0.0, 0.9]
    # sample 3 lies 4.4 from centre 3: outside its window; centre 2 wins
    assert _assign_oracle(pts, vals, cen, C, k, w, 1.0) == [3, 0, 2]
    assert _assign_by_hand(pts, vals, cen, C, k, w, 1.0) == [3, 0, 2]
    pos = np.asarray([p[:3] for p in pts], F32)
    brute = S.assign_brute(pos, np.asarray([p[3] for p in pts], np.int64), np.asarray(vals, F32),
                           np.ones(3, np.int64), np.zeros(3, np.int64), np.asarray(cen, np.float64),
                           np.asarray(C, F32), w, 1.0)
    assert brute.tolist() == [3, 0, 2]


def test_drifting_centres_centre_search_equals_brute_force():
    """k = (4, 4, 4, 2), six iterations on the swarm inputs: the centres
    drift by more than half a cell (so that centres seeded two cells away
    from a sample can hold it in their window), many samples take such a
    centre, and at every iteration the centre-by-centre search equals the
    sample-by-sample brute force over all centres."""
    from tests.slic_cases import SWARM_CF, SWARM_K, SWARM_W, swarm_case
    field, xyz, attr = swarm_case(0)
    T, Z, Y, X = field.shape
    k, w, cf = SWARM_K, SWARM_W, SWARM_CF
    K = int(np.prod(k))
    C = S.grid_interval((X, Y, Z, T), k)
    pos, tt, val, typ, valid = S.samples(field, xyz, attr)
    lab = S.initial_labels(pos, tt, valid, C, k)
    seeds = S.seed_centres(C, k)
    prev = seeds
    cells = [S.seed_cell(pos[:, d], C[d], k[d]) for d in range(3)] + [S.seed_cell(tt.astype(F32), C[3], k[3])]
    far_total = 0
    max_drift = 0.0
    for _ in range(6):
        cen, _ = S.update_centres(pos, tt, val, typ, lab, prev, K)
        max_drift = max(max_drift, float(np.max(np.abs(cen[:, :4] - seeds[:, :4]) / C.astype(np.float64))))
        new = S.assign(pos, tt, val, typ, lab, cen, C, k, w, cf)
        assert np.array_equal(new, S.assign_brute(pos, tt, val, typ, lab, cen, C, w, cf))
        r = new.copy()
        own = []
        for d in range(3):
            own.append(r % k[d])
            r //= k[d]
        own.append(r)
        far = np.zeros(len(new), bool)
        for d in range(4):
            far |= np.abs(own[d] - cells[d]) > 1
        far_total += int((far & (new >= 0)).sum())
        lab, prev = new, cen
    assert max_drift > 0.5
    assert far_total > 100
