"""Pins of the CPU oracle against things other than itself.

* hand-derived fixtures (tests/golden/*.json, each citing its passage);
* brute force: the fixed-point definition iterated with synchronous sweeps,
  and scipy connected components of the explicit coupled graph;
* special cases that reduce to textbook labelling (field only: 4D / 3D
  face-connected components via scipy.ndimage.label);
* closed forms (everything admissible, nothing admissible);
* the invariants I1-I4 that single out the result;
* metamorphic properties (monotone in thresholds and seeds, union over
  seeds, invariance under reordering particles and seeds).
"""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st
from scipy import ndimage

from oracle import bfs, check_invariants, components_grow, oracle_grow, sweep_grow
from paper_1903_12294_amd import synth
from tests import golden_io


def _grow(inst, crit=None, seeds=None, **kw):
    return oracle_grow(inst["field"], inst["xyz"], inst["attr"],
                       inst["crit"] if crit is None else crit,
                       inst["seeds"] if seeds is None else seeds, **kw)


def _bool_field(words, field):
    return golden_io.unpack_field(words, field.shape)


@pytest.mark.parametrize("case", golden_io.all_cases(), ids=lambda c: c["name"])
def test_golden_fixture(case, oracle_lib):
    fm, pm, st_ = _grow(case)
    assert np.array_equal(_bool_field(fm, case["field"]), case["Mf"])
    assert np.array_equal(pm.astype(bool), case["Mp"])
    assert st_["seeds_dropped"] == case["dropped"]
    assert st_["depth"] == case["depth"]
    assert st_["members_field"] == case["Mf"].sum()
    assert st_["members_particle"] == case["Mp"].sum()


_SPECIAL = [np.float32(v) for v in (0.0, 0.25, 0.5, 0.75, 1.0, np.nan, np.inf, -np.inf)]


def _random_instance(rng, X, Y, Z, T, P, S):
    vals = np.array(_SPECIAL, np.float32)
    field = vals[rng.integers(0, len(vals), size=(T, Z, Y, X))]
    # mostly admissible-ish values so that components are non-trivial
    field = np.where(rng.random(field.shape) < 0.55, np.float32(1.0), field).astype(np.float32)
    attr = vals[rng.integers(0, len(vals), size=(T, P))]
    attr = np.where(rng.random(attr.shape) < 0.6, np.float32(1.0), attr).astype(np.float32)
    dims = np.array([X, Y, Z], np.float32)
    xyz = (rng.random((T, P, 3)) * (dims + 0.6) - 0.3).astype(np.float32)
    # sprinkle exact edges: -0.0, dim, largest float below dim, NaN, inf
    edge = rng.random((T, P, 3)) < 0.1
    choice = rng.integers(0, 5, size=(T, P, 3))
    below = np.nextafter(np.broadcast_to(dims, (T, P, 3)), np.float32(0))
    cands = np.stack([np.full((T, P, 3), -0.0, np.float32),
                      np.broadcast_to(dims, (T, P, 3)).astype(np.float32), below,
                      np.full((T, P, 3), np.nan, np.float32),
                      np.full((T, P, 3), np.inf, np.float32)])
    picked = np.take_along_axis(cands, choice[None], 0)[0]
    xyz = np.where(edge, picked, xyz).astype(np.float32)
    seeds = np.stack([rng.integers(0, X, S), rng.integers(0, Y, S), rng.integers(0, Z, S),
                      rng.integers(0, T, S)], axis=1).astype(np.int32)
    lo = rng.choice(np.array([0.25, 0.5, 0.75], np.float32))
    hi = rng.choice(np.array([np.inf, 0.75, 1.0], np.float32))
    alo = rng.choice(np.array([0.25, 0.5, 1.0], np.float32))
    ahi = rng.choice(np.array([np.inf, 1.0], np.float32))
    return dict(field=field, xyz=xyz, attr=attr, seeds=seeds,
                crit=np.array([lo, hi, alo, ahi], np.float32))


@settings(max_examples=250, deadline=None, derandomize=True)
@given(X=st.integers(1, 6), Y=st.integers(1, 5), Z=st.integers(1, 5), T=st.integers(1, 4),
       P=st.integers(0, 40), S=st.integers(0, 4), seed=st.integers(0, 2**31 - 1))
def test_random_tiny_three_ways(X, Y, Z, T, P, S, seed):
    oracle_lib = bfs.load()
    inst = _random_instance(np.random.default_rng(seed), X, Y, Z, T, P, S)
    fm, pm, st_ = _grow(inst, lib=oracle_lib)
    Mf = _bool_field(fm, inst["field"])
    Mp = pm.astype(bool)
    sf, sp_, sweeps, dropped = sweep_grow(inst["field"], inst["xyz"], inst["attr"],
                                          inst["crit"], inst["seeds"])
    cf, cp = components_grow(inst["field"], inst["xyz"], inst["attr"], inst["crit"],
                             inst["seeds"])
    assert np.array_equal(Mf, sf) and np.array_equal(Mp, sp_)
    assert np.array_equal(Mf, cf) and np.array_equal(Mp, cp)
    assert sweeps == st_["depth"] + 1
    assert dropped == st_["seeds_dropped"]
    inv = check_invariants(inst["field"], inst["xyz"], inst["attr"], inst["crit"],
                           inst["seeds"], Mf, Mp)
    assert all(inv.values()), inv


def test_invariants_reject_wrong_sets(oracle_lib):
    """The checker itself: the empty set fails I2, the admissible set fails I4
    (when it has an unseeded component), a one-node-short set fails I3, an
    inadmissible extra node fails I1."""
    inst = synth.make_instance(16, 12, 10, 4, 200, n_blobs=3, seed=7, n_seeds=1)
    fm, pm, _ = _grow(inst)
    Mf, Mp = _bool_field(fm, inst["field"]), pm.astype(bool)
    args = (inst["field"], inst["xyz"], inst["attr"], inst["crit"], inst["seeds"])
    assert Mf.sum() > 10
    r = check_invariants(*args, np.zeros_like(Mf), np.zeros_like(Mp))
    assert not r["I2"]
    Af = inst["field"] >= inst["crit"][0]
    Ap = inst["attr"] >= inst["crit"][2]
    if (Af & ~Mf).any():
        assert not check_invariants(*args, Af, Ap)["I4"]
    short = Mf.copy()
    idx = np.argwhere(Mf)
    # drop a member that is not a seed
    seeds = {tuple(s) for s in inst["seeds"][:, [3, 2, 1, 0]].tolist()}
    for k in idx:
        if tuple(k) not in seeds:
            short[tuple(k)] = False
            break
    assert not check_invariants(*args, short, Mp)["I3"]
    extra = Mf.copy()
    extra[tuple(np.argwhere(~Af)[0])] = True
    assert not check_invariants(*args, extra, Mp)["I1"]


def _ndimage_grow(field, crit, seeds):
    Af = (crit[0] <= field) & (field <= crit[1])
    lab, _ = ndimage.label(Af, structure=ndimage.generate_binary_structure(Af.ndim, 1))
    keep = {lab[t, z, y, x] for x, y, z, t in seeds if lab[t, z, y, x] > 0}
    return np.isin(lab, list(keep)) & (lab > 0)


@pytest.mark.parametrize("k", [1])
def test_field_only_is_4d_face_connected_labelling(k, oracle_lib):
    """P = 0: the grower reduces to 4D connected-component labelling with the
    8-neighbour cross (6 spatial + t±1), keeping the components of the
    admissible seeds."""
    inst = synth.make_config(k)
    fm, _, _ = oracle_grow(inst["field"], None, None, inst["crit"], inst["seeds"])
    assert np.array_equal(_bool_field(fm, inst["field"]),
                          _ndimage_grow(inst["field"], inst["crit"], inst["seeds"]))


@pytest.mark.parametrize("seed", range(6))
def test_field_only_random_4d_and_3d(seed, oracle_lib):
    rng = np.random.default_rng(100 + seed)
    T = 1 if seed % 2 else 3
    field = rng.random((T, 9, 11, 13)).astype(np.float32)
    crit = np.array([0.45, np.inf, 0, np.inf], np.float32)
    seeds = np.stack([rng.integers(0, 13, 5), rng.integers(0, 11, 5), rng.integers(0, 9, 5),
                      rng.integers(0, T, 5)], axis=1).astype(np.int32)
    fm, _, st_ = oracle_grow(field, None, None, crit, seeds)
    got = _bool_field(fm, field)
    if T == 1:  # plain 3D six-connected flood fill
        Af = field[0] >= crit[0]
        lab, _ = ndimage.label(Af, structure=ndimage.generate_binary_structure(3, 1))
        keep = {lab[z, y, x] for x, y, z, t in seeds if lab[z, y, x] > 0}
        exp = (np.isin(lab, list(keep)) & (lab > 0))[None]
    else:
        exp = _ndimage_grow(field, crit, seeds)
    assert np.array_equal(got, exp)


def test_all_admissible_closed_form(oracle_lib):
    """With every node admissible the 4D grid is one component, and a particle
    joins (all of its steps) iff at least one of its steps lies in a voxel."""
    inst = synth.make_config(1)
    crit = np.array([-np.inf, np.inf, -np.inf, np.inf], np.float32)
    fm, pm, st_ = _grow(inst, crit=crit)
    assert _bool_field(fm, inst["field"]).all()
    c = np.floor(inst["xyz"])
    X, Y, Z = inst["dims"]
    binned = ((c[..., 0] >= 0) & (c[..., 0] < X) & (c[..., 1] >= 0) & (c[..., 1] < Y) &
              (c[..., 2] >= 0) & (c[..., 2] < Z))
    exp = np.broadcast_to(binned.any(axis=0), pm.shape)
    assert np.array_equal(pm.astype(bool), exp)
    assert st_["members_field"] == inst["field"].size


def test_nothing_admissible(oracle_lib):
    inst = synth.make_config(1)
    crit = np.array([np.inf, np.inf, np.inf, np.inf], np.float32)
    fm, pm, st_ = _grow(inst, crit=crit)
    assert not fm.any() and not pm.any()
    assert st_["seeds_dropped"] == len(inst["seeds"]) and st_["depth"] == 0


def test_seed_out_of_range_is_an_error(oracle_lib):
    inst = synth.make_instance(8, 8, 8, 2, 10, seed=3)
    for bad in ([8, 0, 0, 0], [0, -1, 0, 0], [0, 0, 8, 0], [0, 0, 0, 2]):
        with pytest.raises(bfs.OracleError) as e:
            _grow(inst, seeds=np.array([bad], np.int32))
        assert e.value.code == -2


@pytest.mark.parametrize("variant", ["field", "noise", "stress_tau"])
def test_config1_three_ways_and_invariants(variant, oracle_lib):
    if variant == "field":
        inst = synth.make_config(1)
    elif variant == "noise":
        inst = synth.make_config(1, attr_mode="noise")
    else:
        inst = synth.make_config(1, tau_p_offset=-0.15)
    fm, pm, st_ = _grow(inst)
    Mf, Mp = _bool_field(fm, inst["field"]), pm.astype(bool)
    sf, sp_, sweeps, _ = sweep_grow(inst["field"], inst["xyz"], inst["attr"], inst["crit"],
                                    inst["seeds"])
    cf, cp = components_grow(inst["field"], inst["xyz"], inst["attr"], inst["crit"],
                             inst["seeds"])
    assert np.array_equal(Mf, sf) and np.array_equal(Mp, sp_) and sweeps == st_["depth"] + 1
    assert np.array_equal(Mf, cf) and np.array_equal(Mp, cp)
    assert all(check_invariants(inst["field"], inst["xyz"], inst["attr"], inst["crit"],
                                inst["seeds"], Mf, Mp).values())
    if variant != "field":
        # the coupling edges change the answer in the stress variants
        fo, _, _ = oracle_grow(inst["field"], None, None, inst["crit"], inst["seeds"])
        assert not np.array_equal(_bool_field(fo, inst["field"]), Mf)


@pytest.fixture(scope="module")
def small_inst():
    return synth.make_instance(24, 20, 18, 6, 800, n_blobs=4, seed=11, n_seeds=3,
                               tau_f=0.3, tau_p=0.2)


def test_monotone_in_thresholds(small_inst, oracle_lib):
    fm_hi, pm_hi, _ = _grow(small_inst)
    crit = small_inst["crit"].copy()
    crit[0] -= np.float32(0.05)
    crit[2] -= np.float32(0.05)
    fm_lo, pm_lo, _ = _grow(small_inst, crit=crit)
    assert not (fm_hi & ~fm_lo).any() and not (pm_hi & ~pm_lo).any()
    assert (fm_lo != fm_hi).any()


def test_union_over_seeds(small_inst, oracle_lib):
    s = small_inst["seeds"]
    f_all, p_all, _ = _grow(small_inst)
    f_u = np.zeros_like(f_all)
    p_u = np.zeros_like(p_all)
    for k in range(len(s)):
        f, p, _ = _grow(small_inst, seeds=s[k:k + 1])
        f_u |= f
        p_u |= p
    assert np.array_equal(f_all, f_u) and np.array_equal(p_all, p_u)


def test_reordering_particles_and_seeds(small_inst, oracle_lib):
    rng = np.random.default_rng(5)
    f0, p0, st0 = _grow(small_inst)
    perm = rng.permutation(small_inst["xyz"].shape[1])
    inst = dict(small_inst, xyz=small_inst["xyz"][:, perm], attr=small_inst["attr"][:, perm])
    f1, p1, st1 = oracle_grow(inst["field"], inst["xyz"], inst["attr"], inst["crit"],
                              small_inst["seeds"][::-1].copy())
    assert np.array_equal(f0, f1)
    assert np.array_equal(p0[:, perm], p1)
    assert st0["depth"] == st1["depth"]
