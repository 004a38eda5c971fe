"""Pins of the trajectory segment rule's oracle (Section 3.4): hand-worked
trajectories, and on random inputs the local characterisation (a step stays
iff a time neighbour of the same particle carries the same feature), which
the oracle does not use (it walks runs)."""
import numpy as np
import pytest

from oracle import segments as oseg

A, B, N = 3, 7, -1


@pytest.mark.parametrize("ids,want", [
    ([A, A, A], [A, A, A]),                      # one feature throughout: kept whole
    ([A], [N]),                                  # a single step is no segment
    ([A, B, A, B], [N, N, N, N]),                # alternating: nothing consecutive
    ([A, A, B, B, A], [A, A, B, B, N]),          # split into two segments, a stray end
    ([N, N, A, A], [N, N, A, A]),                # steps in no feature are never kept
    ([A, N, A], [N, N, N]),                      # a gap splits a run into singletons
    ([B, B, N, A, A, A, N, B], [B, B, N, A, A, A, N, N]),
])
def test_worked_trajectories(ids, want):
    got = oseg.feature_segments(np.array(ids)[:, None])
    assert got[:, 0].tolist() == want


def test_particles_are_independent_columns():
    ids = np.array([[A, B], [A, A], [B, A]])
    assert oseg.feature_segments(ids).tolist() == [[A, N], [A, A], [N, A]]


def test_no_steps_and_no_particles():
    assert oseg.feature_segments(np.zeros((0, 4), np.int64)).shape == (0, 4)
    assert oseg.feature_segments(np.zeros((5, 0), np.int64)).shape == (5, 0)


def _local(ids):
    T, P = ids.shape
    out = np.full((T, P), -1, np.int64)
    for t in range(T):
        for p in range(P):
            f = ids[t, p]
            if f < 0:
                continue
            if (t > 0 and ids[t - 1, p] == f) or (t + 1 < T and ids[t + 1, p] == f):
                out[t, p] = f
    return out


@pytest.mark.parametrize("T,nf,seed", [(2, 2, 0), (9, 3, 1), (70, 2, 2), (130, 4, 3)])
def test_runs_equal_local_rule(T, nf, seed):
    rng = np.random.default_rng(seed)
    ids = rng.integers(-1, nf, size=(T, 40))
    got = oseg.feature_segments(ids)
    assert np.array_equal(got, _local(ids))
    kept = got >= 0
    assert np.all(got[kept] == ids[kept])        # a kept step keeps its own id


def test_mask_runs_of_lengths():
    # runs of 1, 2, 3 and 1 member steps, separated by gaps
    col = [1, 0, 1, 1, 0, 1, 1, 1, 0, 0, 1]
    pm = np.array(col, np.uint8)[:, None]
    assert oseg.mask_segments(pm)[:, 0].tolist() == [0, 0, 1, 1, 0, 1, 1, 1, 0, 0, 0]
    full = np.ones((64, 3), np.uint8)
    assert np.array_equal(oseg.mask_segments(full), full)
    assert oseg.mask_segments(np.ones((1, 3), np.uint8)).sum() == 0


def test_point_features():
    pl = np.array([[0, 2, -1], [1, 1, 3]])
    feat = np.array([0, 0, 2, 2])
    assert oseg.point_features(pl, feat).tolist() == [[0, 2, -1], [0, 0, 2]]
