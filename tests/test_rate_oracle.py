"""Pins of particles stored at their own temporal rate (r particle steps per
field step; the paper's datasets save particles more often than the field):
particle step tau lies at time tau / r and couples with field step
floor(tau / r).

Hand-placed cases fix the mapping; repeating every particle step r times must
reproduce the rate-1 result step for step (the upsampled trajectories visit
the same voxels); the breadth-first oracle, the fixed-point sweeps and
scipy's reachability over the explicit graph must agree at any rate; the
clustering's point samples carry fractional times."""
import numpy as np
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st

from oracle import oracle_grow, reach_grow, sweep_grow
from oracle import slic as oslic
from oracle.bfs import OracleError
from tests.test_oracle_pins import _random_instance

BAND = np.array([0.5, 1.5, 0.5, 1.5], np.float32)


def _bits(fmask, shape):
    n = int(np.prod(shape))
    return np.unpackbits(fmask.view(np.uint8), bitorder="little")[:n].astype(bool).reshape(shape)


def _row_case():
    """X = 3 voxels in a row, T = 2 field steps, one particle at r = 2 (Tp = 4).
    The field is admissible at (x=0, t=0) (the seed) and (x=2, t=1)."""
    field = np.zeros((2, 1, 1, 3), np.float32)
    field[0, 0, 0, 0] = 1.0
    field[1, 0, 0, 2] = 1.0
    xyz = np.full((4, 1, 3), 0.5, np.float32)
    xyz[:, 0, 0] = [0.5, 0.5, 2.5, 2.5]
    attr = np.ones((4, 1), np.float32)
    seeds = np.array([[0, 0, 0, 0]], np.int32)
    return field, xyz, attr, seeds


def test_steps_map_to_the_field_step_holding_their_time():
    field, xyz, attr, seeds = _row_case()
    fm, pm, _ = oracle_grow(field, xyz, attr, BAND, seeds, rate=2)
    # steps 0, 1 lie in field step 0 (voxel 0 joins them), steps 2, 3 in field
    # step 1, where the particle reaches the admissible voxel x = 2
    assert pm[:, 0].tolist() == [1, 1, 1, 1]
    assert _bits(fm, field.shape)[1, 0, 0, 2]
    # moving step 1 to x = 2.5 puts it in voxel (2, t=0), not (2, t=1)
    xyz[1, 0, 0] = 2.5
    fm, pm, _ = oracle_grow(field, xyz, attr, BAND, seeds, rate=2)
    assert pm[:, 0].tolist() == [1, 1, 1, 1]
    assert _bits(fm, field.shape).sum() == 2
    # forward-only: the particle joins at step 0 and keeps every later step
    fm, pm, _ = oracle_grow(field, xyz, attr, BAND, seeds, rate=2, forward_only=True)
    assert pm[:, 0].tolist() == [1, 1, 1, 1]


def test_a_particle_entering_later_joins_later_in_forward_mode():
    field, xyz, attr, seeds = _row_case()
    xyz[:, 0, 0] = [1.5, 1.5, 2.5, 2.5]          # meets the feature only at step 2
    field[1, 0, 0, 1] = 1.0                        # a bridge (1, t=1) - (2, t=1)
    field[1, 0, 0, 0] = 1.0                        # and (0, t=0) - (0, t=1) - (1, t=1)
    fm, pm, _ = oracle_grow(field, xyz, attr, BAND, seeds, rate=2)
    assert pm[:, 0].tolist() == [1, 1, 1, 1]
    fm, pm, _ = oracle_grow(field, xyz, attr, BAND, seeds, rate=2, forward_only=True)
    assert pm[:, 0].tolist() == [0, 0, 1, 1]


def test_too_many_steps_is_an_error():
    field, xyz, attr, seeds = _row_case()
    with pytest.raises(OracleError):
        oracle_grow(field, xyz[:3], attr[:3], BAND, seeds, rate=1)  # Tp = 3 > 1 * T


@pytest.mark.parametrize("r", [2, 3])
@pytest.mark.parametrize("forward_only", [False, True])
@pytest.mark.parametrize("seed", range(6))
def test_repeating_steps_changes_nothing(seed, forward_only, r):
    rng = np.random.default_rng(100 + seed)
    inst = _random_instance(rng, 6, 5, 4, 4, 30, 4)
    args = (inst["field"], inst["xyz"], inst["attr"], inst["crit"], inst["seeds"])
    fm1, pm1, _ = oracle_grow(*args, forward_only=forward_only)
    xyz_r = np.repeat(inst["xyz"], r, axis=0)
    attr_r = np.repeat(inst["attr"], r, axis=0)
    fmr, pmr, _ = oracle_grow(inst["field"], xyz_r, attr_r, inst["crit"], inst["seeds"],
                              forward_only=forward_only, rate=r)
    assert np.array_equal(fm1, fmr)
    assert np.array_equal(np.repeat(pm1, r, axis=0), pmr)


@settings(max_examples=150, deadline=None, derandomize=True)
@given(X=st.integers(1, 6), Y=st.integers(1, 4), Z=st.integers(1, 4), T=st.integers(1, 4),
       P=st.integers(0, 20), S=st.integers(0, 4), r=st.integers(1, 4), fwd=st.booleans(),
       seed=st.integers(0, 2**31 - 1))
def test_three_formulations_agree_at_any_rate(X, Y, Z, T, P, S, r, fwd, seed):
    rng = np.random.default_rng(seed)
    Tp = int(rng.integers(1, r * T + 1)) if r > 1 else T
    base = _random_instance(rng, X, Y, Z, Tp, P, 0)
    inst = _random_instance(rng, X, Y, Z, T, 0, S)
    args = (inst["field"], base["xyz"], base["attr"], inst["crit"], inst["seeds"])
    fm, pm, st_ = oracle_grow(*args, forward_only=fwd, rate=r)
    Mf, Mp, sweeps, _ = sweep_grow(*args, forward_only=fwd, rate=r)
    Rf, Rp = reach_grow(*args, forward_only=fwd, rate=r)
    shape = inst["field"].shape
    assert np.array_equal(_bits(fm, shape), Mf) and np.array_equal(Mf, Rf)
    assert np.array_equal(pm.astype(bool), Mp) and np.array_equal(Mp, Rp)
    assert sweeps == st_["depth"] + 1


def test_clustering_point_times_are_fractional():
    T, r = 4, 2
    field = np.zeros((T, 2, 2, 2), np.float32)
    xyz = np.full((T * r, 1, 3), 0.75, np.float32)
    attr = np.zeros((T * r, 1), np.float32)
    pos, tt, val, typ, valid = oslic.samples(field, xyz, attr, rate=r)
    assert tt[typ == 1].tolist() == [0.0, 0.5, 1.0, 1.5, 2.0, 2.5, 3.0, 3.5]
    # k_t = 2 on T = 4: interval C_t = 2, so points before time 2 seed in cell 0
    C = oslic.grid_interval((2, 2, 2, T), (1, 1, 1, 2))
    lab = oslic.initial_labels(pos, tt, valid, C, (1, 1, 1, 2))
    assert lab[typ == 1].tolist() == [0, 0, 0, 0, 1, 1, 1, 1]


def test_clustering_one_centre_mean_time_with_rate():
    rng = np.random.default_rng(5)
    T, r, P = 3, 4, 7
    field = rng.random((T, 2, 3, 4), dtype=np.float32)
    xyz = (rng.random((T * r - 1, P, 3)) * np.array([4, 3, 2])).astype(np.float32)
    attr = rng.random((T * r - 1, P), dtype=np.float32)
    fl, pl, cen, cnt, it = oslic.slic(field, xyz, attr, (1, 1, 1, 1), (1, 1, 1), 1, 1e-6, 3, rate=r)
    times = np.concatenate([np.repeat(np.arange(T), field[0].size), np.repeat(np.arange(T * r - 1) / r, P)])
    assert abs(cen[0, 3] - times.mean()) < 1e-6
    assert pl.shape == (T * r - 1, P) and (pl == 0).all()
