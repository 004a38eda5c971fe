"""Pins of the per-seed component ids in the oracle: each node carries the
index of the lowest seed whose own region holds it.

Checked against what fixes them independently: with undirected coupling the
regions are connected components, so every component of scipy's labelling
of the explicit graph carries one id, the lowest index of the admissible
seeds inside it; the labelled nodes are exactly the union grow; hand-placed
cases fix ties, dropped seeds and the forward-only direction."""
import numpy as np
import pytest
import scipy.sparse as sp
from hypothesis import given, settings
from hypothesis import strategies as st
from scipy.sparse.csgraph import connected_components

from oracle import edge_list, oracle_grow, oracle_seed_ids
from tests.test_causal_oracle import BAND, _line_case
from tests.test_oracle_pins import _random_instance


def _bits(fmask, n):
    return np.unpackbits(fmask.view(np.uint8), bitorder="little")[:n].astype(bool)


@settings(max_examples=120, deadline=None, derandomize=True)
@given(X=st.integers(1, 6), Y=st.integers(1, 5), Z=st.integers(1, 4), T=st.integers(1, 5),
       P=st.integers(0, 25), S=st.integers(0, 6), seed=st.integers(0, 2**31 - 1))
def test_components_carry_their_lowest_seed(X, Y, Z, T, P, S, seed):
    rng = np.random.default_rng(seed)
    inst = _random_instance(rng, X, Y, Z, T, P, S)
    args = (inst["field"], inst["xyz"], inst["attr"], inst["crit"])
    fid, pid = oracle_seed_ids(*args, inst["seeds"])
    ids = np.concatenate([fid.ravel(), pid.ravel()])
    # labelled = the union grow
    fm, pm, _ = oracle_grow(*args, inst["seeds"])
    V = inst["field"].size
    assert np.array_equal(ids[:V] >= 0, _bits(fm, V))
    assert np.array_equal(ids[V:] >= 0, pm.ravel() != 0)
    # each component: one id, its lowest admissible seed
    a, b, V, Q = edge_list(*args)
    g = sp.coo_matrix((np.ones(len(a), np.int8), (a, b)), shape=(V + Q, V + Q))
    _, lab = connected_components(g, directed=False)
    Af = (np.float32(inst["crit"][0]) <= inst["field"]) & (inst["field"] <= np.float32(inst["crit"][1]))
    low = {}
    for i, (x, y, z, t) in enumerate(inst["seeds"]):
        if Af[t, z, y, x]:
            c = lab[((t * Z + z) * Y + y) * X + x]
            low.setdefault(c, i)
    want = np.array([low.get(c, -1) for c in lab], np.int64)
    assert np.array_equal(ids, want)


def _two_blobs():
    """A 6 x 1 x 1 x 1 field admissible at x = 0, 1 and x = 4, 5 (two blobs)."""
    field = np.array([1, 1, 0, 0, 1, 1], np.float32).reshape(1, 1, 1, 6)
    return field


def test_lowest_index_wins_and_dropped_seeds_name_nothing():
    field = _two_blobs()
    seeds = np.array([[2, 0, 0, 0],    # 0: not admissible, dropped
                      [5, 0, 0, 0],    # 1: right blob
                      [0, 0, 0, 0],    # 2: left blob
                      [4, 0, 0, 0],    # 3: right blob again
                      [1, 0, 0, 0]],   # 4: left blob again
                     np.int32)
    fid, _ = oracle_seed_ids(field, None, None, BAND, seeds)
    assert fid.ravel().tolist() == [2, 2, -1, -1, 1, 1]


def test_duplicate_seeds():
    field = _two_blobs()
    seeds = np.array([[4, 0, 0, 0], [4, 0, 0, 0], [0, 0, 0, 0]], np.int32)
    fid, _ = oracle_seed_ids(field, None, None, BAND, seeds)
    assert fid.ravel().tolist() == [2, 2, -1, -1, 0, 0]


def test_forward_only_regions_overlap():
    """Line case with particle 0 passing voxel (3, t=3): seed 0 at that voxel
    reaches every particle at t >= 3; seed 1 at (0, t=2) also reaches
    particle 0 at t = 2.  The overlap keeps id 0; particle 0 at t = 2 and the
    seed voxel of seed 1 get id 1."""
    field, xyz, attr, _ = _line_case()
    xyz[3, 0, 0] = 3.5
    seeds = np.array([[3, 0, 0, 3], [0, 0, 0, 2]], np.int32)
    fid, pid = oracle_seed_ids(field, xyz, attr, BAND, seeds, forward_only=True)
    assert pid[:, 0].tolist() == [-1, -1, 1, 0, 0]
    assert pid[:, 1].tolist() == [-1, -1, -1, 0, 0]
    assert pid[:, 2].tolist() == [-1, -1, -1, 0, 0]
    assert fid[2, 0, 0, 0] == 1 and fid[3, 0, 0, 3] == 0
    # undirected, both seeds share one component: id 0 everywhere it reaches
    fid_u, pid_u = oracle_seed_ids(field, xyz, attr, BAND, seeds)
    assert set(np.unique(pid_u)) == {0} and set(np.unique(fid_u)) == {-1, 0}


@pytest.mark.parametrize("forward_only", [False, True])
def test_no_seeds(forward_only):
    field = _two_blobs()
    fid, pid = oracle_seed_ids(field, None, None, BAND, np.zeros((0, 4), np.int32), forward_only)
    assert (fid == -1).all() and pid.shape == (1, 0)
