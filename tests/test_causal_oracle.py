"""Pins of forward-only (causal) trajectory coupling in the oracles: a
trajectory edge leads from (i, t) to (i, t + 1) only, every other edge stays
undirected, and the grown set is what the seeds reach along directed edges.

Hand-worked cases fix the expected sets; on random tiny instances the C
breadth-first oracle, the numpy fixed-point sweeps and scipy's directed
breadth-first order over an explicit graph must agree, and the causal set must
lie inside the undirected one."""
import numpy as np
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st

from oracle import oracle_grow, reach_grow, sweep_grow
from tests.test_oracle_pins import _random_instance

BAND = np.array([0.5, 1.5, 0.5, 1.5], np.float32)


def _bits(fmask, shape):
    n = int(np.prod(shape))
    return np.unpackbits(fmask.view(np.uint8), bitorder="little")[:n].astype(bool).reshape(shape)


def _line_case():
    """X = 4 voxels in a row (Y = Z = 1), T = 5.  The field is admissible at
    (x=0, t=2) (the seed) and at (x=3, t=3) only.  Particle 0 sits in voxel 0
    at every step; particle 1 sits in voxel 3 at every step; particle 2 sits in
    voxel 3 at t <= 3 and in voxel 1 after.  Every particle-step is admissible."""
    T, X = 5, 4
    field = np.zeros((T, 1, 1, X), np.float32)
    field[2, 0, 0, 0] = 1.0
    field[3, 0, 0, 3] = 1.0
    xyz = np.full((T, 3, 3), 0.5, np.float32)
    xyz[:, 0, 0] = 0.5
    xyz[:, 1, 0] = 3.5
    xyz[:, 2, 0] = np.where(np.arange(T) <= 3, 3.5, 1.5)
    attr = np.ones((T, 3), np.float32)
    seeds = np.array([[0, 0, 0, 2]], np.int32)
    return field, xyz, attr, seeds


def test_line_case_undirected():
    # undirected: particle 0 joins whole (steps 0..4 through the seed voxel);
    # the voxel (3, t=3) is never reached (no member particle is in it)
    field, xyz, attr, seeds = _line_case()
    fm, pm, st_ = oracle_grow(field, xyz, attr, BAND, seeds)
    assert pm[:, 0].tolist() == [1, 1, 1, 1, 1]
    assert pm[:, 1:].sum() == 0
    assert _bits(fm, field.shape).sum() == 1


def test_line_case_forward_only():
    # causal: particle 0 joins at t = 2 and keeps its later steps only
    field, xyz, attr, seeds = _line_case()
    fm, pm, _ = oracle_grow(field, xyz, attr, BAND, seeds, forward_only=True)
    assert pm[:, 0].tolist() == [0, 0, 1, 1, 1]
    assert pm[:, 1:].sum() == 0
    Mf, Mp, _, _ = sweep_grow(field, xyz, attr, BAND, seeds, forward_only=True)
    assert np.array_equal(Mp, pm.astype(bool))
    assert np.array_equal(Mf, _bits(fm, field.shape))


def test_forward_then_back_into_the_field():
    """Particle 0 (causal member from t = 2) passes voxel (3, t=3): put it
    there at t = 3, so the voxel joins, and through it particles 1 and 2
    join at t = 3 -- with their later steps only."""
    field, xyz, attr, seeds = _line_case()
    xyz[3, 0, 0] = 3.5
    fm, pm, _ = oracle_grow(field, xyz, attr, BAND, seeds, forward_only=True)
    assert pm[:, 0].tolist() == [0, 0, 1, 1, 1]
    assert pm[:, 1].tolist() == [0, 0, 0, 1, 1]
    assert pm[:, 2].tolist() == [0, 0, 0, 1, 1]
    assert _bits(fm, field.shape).sum() == 2
    # undirected, the same particles join whole
    _, pu, _ = oracle_grow(field, xyz, attr, BAND, seeds)
    assert pu.sum() == 15


def test_gap_stops_the_forward_run():
    field, xyz, attr, seeds = _line_case()
    attr[4, 0] = 9.0  # outside the band: particle 0's run ends at t = 3
    _, pm, _ = oracle_grow(field, xyz, attr, BAND, seeds, forward_only=True)
    assert pm[:, 0].tolist() == [0, 0, 1, 1, 0]


@settings(max_examples=200, deadline=None, derandomize=True)
@given(X=st.integers(1, 6), Y=st.integers(1, 5), Z=st.integers(1, 4), T=st.integers(1, 5),
       P=st.integers(0, 25), S=st.integers(0, 5), seed=st.integers(0, 2**31 - 1))
def test_three_formulations_agree(X, Y, Z, T, P, S, seed):
    rng = np.random.default_rng(seed)
    inst = _random_instance(rng, X, Y, Z, T, P, S)
    args = (inst["field"], inst["xyz"], inst["attr"], inst["crit"], inst["seeds"])
    fm, pm, st_ = oracle_grow(*args, forward_only=True)
    Mf, Mp, sweeps, dropped = sweep_grow(*args, forward_only=True)
    Rf, Rp = reach_grow(*args, forward_only=True)
    shape = inst["field"].shape
    assert np.array_equal(_bits(fm, shape), Mf) and np.array_equal(Mf, Rf)
    assert np.array_equal(pm.astype(bool), Mp) and np.array_equal(Mp, Rp)
    assert sweeps == st_["depth"] + 1 and dropped == st_["seeds_dropped"]
    # inside the undirected set; the directed graph with both ways is the same
    fu, pu, _ = oracle_grow(*args)
    Uf, Up = reach_grow(*args, forward_only=False)
    assert np.array_equal(_bits(fu, shape), Uf) and np.array_equal(pu.astype(bool), Up)
    assert not (Mf & ~Uf).any() and not (Mp & ~Up).any()


@pytest.mark.parametrize("seed", range(5))
def test_one_step_or_no_particles_changes_nothing(seed):
    rng = np.random.default_rng(seed)
    for T, P in ((1, 30), (4, 0)):
        inst = _random_instance(rng, 5, 4, 3, T, P, 4)
        args = (inst["field"], inst["xyz"], inst["attr"], inst["crit"], inst["seeds"])
        a = oracle_grow(*args, forward_only=True)
        b = oracle_grow(*args)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
