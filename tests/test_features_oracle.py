"""Pins of the predictor-input reference (oracle/features.py): closed forms,
hand-placed particles, the t - 1 channels, bfloat16 rounding, and a per-voxel
brute force on tiny random grids."""
import math

import numpy as np

from oracle import features as of


def _bf16_value(bits):
    return (np.asarray(bits, np.uint32) << 16).view(np.float32)


def test_bf16_rounding_ties_to_even():
    one = np.float32(1.0)
    half_ulp = np.float32(2.0 ** -8)  # halfway between 1 and the next bfloat16 (1 + 2^-7)
    vals = np.array([one, one + half_ulp, one + 3 * half_ulp, one + half_ulp + np.float32(2.0 ** -20),
                     -2.5, 0.0, -0.0], np.float32)
    got = _bf16_value(of.bf16_bits(vals))
    want = np.array([1.0, 1.0, 1.0 + 2.0 ** -6, 1.0 + 2.0 ** -7, -2.5, 0.0, -0.0], np.float32)
    assert np.array_equal(got, want)
    assert np.signbit(got[-1])


def test_constant_brick_closed_form():
    field = np.full((2, 8, 8, 8), 0.75, np.float32)
    x = of.features(field, None, 0.25)
    assert x.shape == (2, 1, 1, 1, 16)
    v = _bf16_value(x[..., :8])
    assert np.array_equal(v[0, 0, 0, 0], np.array([0.5, 0.5, 0.5, 0, 0, 0, 0, 0], np.float32))
    assert np.array_equal(v[1, 0, 0, 0], np.array([0.5, 0.5, 0.5, 0, 0.5, 0.5, 0.5, 0], np.float32))
    assert not x[..., 8:].any()


def test_nan_brick_and_infinite_bound():
    field = np.zeros((1, 8, 8, 16), np.float32)
    field[:, :, :, :8] = np.nan          # first brick: no value
    field[0, 3, 4, 9] = 2.0              # second brick: zeros and one 2
    st = of.brick_stats(field)
    assert np.array_equal(st[0, 0, 0, 0], [-1, -1, -1])
    assert np.allclose(st[0, 0, 0, 1], [0.0, 2.0, 2.0 / 512])
    x = of.features(field, None, -np.inf)  # c = 0 for a bound that is not finite
    v = _bf16_value(x[0, 0, 0, 0, :3])
    assert np.array_equal(v, np.array([-1, -1, -1], np.float32))


def test_ragged_bricks_use_only_grid_voxels():
    rng = np.random.default_rng(5)
    field = rng.random((1, 9, 10, 11)).astype(np.float32)  # Z=9, Y=10, X=11: 2 bricks per axis
    st = of.brick_stats(field)
    assert st.shape == (1, 2, 2, 2, 3)
    corner = field[0, 8:, 8:, 8:].astype(np.float64)  # 1 x 2 x 3 voxels
    assert np.array_equal(st[0, 1, 1, 1], [corner.min(), corner.max(), corner.mean()])


def test_particle_counts_by_hand():
    X, Y, Z, T = 16, 8, 8, 2
    pts = np.array([
        [[0.0, 0.0, 0.0], [7.99, 7.99, 7.99], [8.0, 0.5, 0.5], [16.0, 1.0, 1.0],
         [-1e-6, 1.0, 1.0], [np.nan, 1.0, 1.0], [-0.0, 0.0, 0.0]],
    ], np.float32)
    xyz = np.repeat(pts, 4, axis=0)  # Tp = 4 steps at rate 2: steps 0,1 -> t 0; 2,3 -> t 1
    cnt = of.brick_counts(xyz, (X, Y, Z), T, rate=2)
    # brick x = 0 holds the points at 0, 7.99 and -0.0; brick x = 1 the one at 8;
    # 16 (= X), a small negative and NaN lie in no voxel
    assert cnt.tolist() == [[[[6, 2]]], [[[6, 2]]]]


def test_previous_step_channels_shift_by_one():
    rng = np.random.default_rng(2)
    field = rng.random((3, 8, 16, 8)).astype(np.float32)
    xyz = rng.random((3, 50, 3)).astype(np.float32) * np.array([8, 16, 8], np.float32)
    x = of.features(field, xyz, 0.1)
    assert np.array_equal(x[1:, ..., 4:8], x[:-1, ..., 0:4])
    assert not x[0, ..., 4:8].any()
    # log1p(count) / 4 channel
    cnt = of.brick_counts(xyz, (8, 16, 8), 3)
    want = of.bf16_bits((np.log1p(cnt).astype(np.float32) * np.float32(0.25)))
    assert np.array_equal(x[..., 3], want)


def test_stats_against_per_voxel_loop():
    rng = np.random.default_rng(11)
    for _ in range(4):
        T, Z, Y, X = rng.integers(1, 3), rng.integers(1, 12), rng.integers(1, 12), rng.integers(1, 12)
        field = rng.normal(size=(T, Z, Y, X)).astype(np.float32)
        field[rng.random(field.shape) < 0.2] = np.nan
        st = of.brick_stats(field)
        D, H, W = math.ceil(Z / 8), math.ceil(Y / 8), math.ceil(X / 8)
        for t in range(T):
            for bz in range(D):
                for by in range(H):
                    for bx in range(W):
                        vals = []
                        for z in range(Z):
                            for y in range(Y):
                                for x in range(X):
                                    v = float(field[t, z, y, x])
                                    if z // 8 == bz and y // 8 == by and x // 8 == bx and v == v:
                                        vals.append(v)
                        if vals:
                            want = [min(vals), max(vals), math.fsum(vals) / len(vals)]
                        else:
                            want = [-1.0, -1.0, -1.0]
                        assert np.allclose(st[t, bz, by, bx], want, rtol=0, atol=1e-12)
