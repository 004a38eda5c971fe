"""The seeded input generator: deterministic, in range, and following its recipe."""
import math

import numpy as np

from paper_1903_12294_amd import synth


def test_deterministic_and_shapes():
    a = synth.make_config(1)
    b = synth.make_config(1)
    for k in ("field", "xyz", "attr", "seeds", "crit"):
        assert np.array_equal(a[k], b[k], equal_nan=True), k
    assert a["field"].shape == (8, 32, 32, 32) and a["field"].dtype == np.float32
    assert a["xyz"].shape == (8, 4096, 3) and a["attr"].shape == (8, 4096)
    assert a["seeds"].shape == (1, 4) and a["seeds"][0, 3] == 0


def test_positions_in_grid_and_attr_is_field_sample():
    inst = synth.make_instance(20, 16, 12, 3, 500, seed=9)
    xyz = inst["xyz"]
    for a, n in enumerate((20, 16, 12)):
        assert (xyz[..., a] >= 0).all() and (xyz[..., a] < n).all()
    # a particle exactly at a voxel centre samples that voxel's value
    f = inst["field"]
    xyzc = np.array([[[3.5, 4.5, 5.5]]], np.float32).repeat(3, axis=0)
    at = synth.sample_attribute(f, xyzc)
    assert np.allclose(at[:, 0], f[:, 5, 4, 3])


def test_abc_rk4_step_matches_fine_integration():
    # one dt=0.05 RK4 step agrees with 100 Euler-free RK4 substeps to ~1e-7
    p0 = np.array([[0.3, 1.7, 4.2]])
    coarse = p0.copy()
    k1 = synth._abc(coarse); k2 = synth._abc(coarse + 0.025 * k1)
    k3 = synth._abc(coarse + 0.025 * k2); k4 = synth._abc(coarse + 0.05 * k3)
    coarse = coarse + (0.05 / 6) * (k1 + 2 * k2 + 2 * k3 + k4)
    fine = p0.copy()
    h = 0.05 / 100
    for _ in range(100):
        k1 = synth._abc(fine); k2 = synth._abc(fine + 0.5 * h * k1)
        k3 = synth._abc(fine + 0.5 * h * k2); k4 = synth._abc(fine + h * k3)
        fine = fine + (h / 6) * (k1 + 2 * k2 + 2 * k3 + k4)
    assert np.abs(coarse - fine).max() < 1e-6
    # steady ABC flow with A=B=C=1 is divergence-free: d/dx(sin z + cos y) = 0 etc.
    x = np.array([[0.1, 0.2, 0.3]])
    eps = 1e-6
    div = sum((synth._abc(x + eps * np.eye(3)[a]) - synth._abc(x - eps * np.eye(3)[a]))[0, a]
              for a in range(3)) / (2 * eps)
    assert abs(div) < 1e-8


def test_blob_peak_near_centre():
    inst = synth.make_instance(40, 40, 40, 2, 0, n_blobs=1, seed=21, n_seeds=1)
    b = inst["blobs"]
    c = np.floor(b.centre(0, 1)).astype(int)
    assert inst["field"][1, c[2], c[1], c[0]] > 0.9 * b.amp[0]


def test_queries_shape():
    inst = synth.make_config(1)
    crit, qs = synth.make_queries(inst, Q=256)
    assert crit.shape == (256, 4) and qs.shape[1] == 5
    assert set(np.unique(qs[:, 4])) == set(range(256))
    assert (crit[:, 0] >= 0.15).all() and (crit[:, 0] <= 0.6).all()
    counts = np.bincount(qs[:, 4], minlength=256)
    assert counts.min() >= 1 and counts.max() <= 16
