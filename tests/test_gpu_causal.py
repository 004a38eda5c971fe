"""GPU parity of forward-only (causal) trajectory coupling: the HIP grower with
MF4D_TRAJ_FORWARD against the oracle's directed breadth-first grow, bit for
bit -- single queries under both schedules and admissibility modes, long
trajectories (several label words), the batched grower, and switching the
mode on one context."""
import numpy as np
import pytest

from oracle import oracle_grow, oracle_grow_queries
from paper_1903_12294_amd import synth
from tests import golden_io

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _grow(g, inst):
    g.set_criteria(*inst["crit"])
    g.set_seeds(np.asarray(inst["seeds"], np.int32).reshape(-1, 4))
    g.grow()
    fm = g.read_field_mask()
    pm = g.read_particle_mask() if inst["xyz"].shape[1] > 0 else np.zeros((inst["field"].shape[0], 0), np.uint8)
    return fm, pm, g.stats()


def _load(g, inst):
    dev = torch.device("cuda:0")
    g.load_field(torch.from_numpy(np.ascontiguousarray(inst["field"])).to(dev))
    if inst["xyz"].shape[1] > 0:
        g.load_particles(torch.from_numpy(np.ascontiguousarray(inst["xyz"])).to(dev),
                         torch.from_numpy(np.ascontiguousarray(inst["attr"])).to(dev))


def _assert_forward(inst, tag, tile_t=None, schedule=None, admit=None):
    from paper_1903_12294_amd import Grower
    _need_gpu()
    print(f"[causal] {tag} field {inst['field'].shape} P={inst['xyz'].shape[1]} "
          f"tile_t={tile_t} {schedule} {admit}", flush=True)
    g = Grower(device=0, tile_t=tile_t, schedule=schedule, admit=admit)
    try:
        _load(g, inst)
        g.set_trajectory_mode("forward")
        fm, pm, st = _grow(g, inst)
    finally:
        g.close()
    ofm, opm, ost = oracle_grow(inst["field"], inst["xyz"], inst["attr"], inst["crit"], inst["seeds"],
                                forward_only=True)
    assert np.array_equal(fm, ofm), f"{tag}: field mask differs"
    assert np.array_equal(pm, opm), f"{tag}: particle mask differs ({int(pm.sum())} vs {int(opm.sum())})"
    assert st["members_field"] == ost["members_field"]
    assert st["members_particle"] == ost["members_particle"]
    return ost


@pytest.mark.parametrize("schedule", ["persistent", "launch"])
@pytest.mark.parametrize("case", golden_io.all_cases(), ids=lambda c: c["name"])
def test_golden_fixtures_forward(case, schedule):
    _assert_forward(dict(case), case["name"], schedule=schedule)


@pytest.mark.parametrize("seed", range(12))
def test_random_small_ragged_forward(seed):
    from tests.test_oracle_pins import _random_instance
    rng = np.random.default_rng(3000 + seed)
    X, Y, Z = (int(v) for v in rng.integers(1, 50, 3))
    T = int(rng.integers(1, 20))
    P = int(rng.integers(0, 300))
    inst = _random_instance(rng, X, Y, Z, T, P, 5)
    _assert_forward(inst, f"random{seed}", tile_t=[4, 8, 16][seed % 3],
                    schedule=["persistent", "launch"][(seed // 3) % 2],
                    admit=["tiles", "all"][(seed // 6) % 2])


@pytest.mark.parametrize("schedule", ["persistent", "launch"])
@pytest.mark.parametrize("variant", ["field", "noise"])
def test_32cube_workload_forward(variant, schedule):
    inst = synth.make_config(1, **(dict(attr_mode="noise") if variant == "noise" else {}))
    ost = _assert_forward(inst, f"32^3x8-{variant}", schedule=schedule)
    _, opm, _ = oracle_grow(inst["field"], inst["xyz"], inst["attr"], inst["crit"], inst["seeds"])
    assert ost["members_particle"] < int(opm.sum())  # the direction matters on this input


@pytest.mark.parametrize("schedule", ["persistent", "launch"])
@pytest.mark.parametrize("T", [67, 130])
def test_long_trajectories_forward(T, schedule):
    """Runs of admissible steps crossing 64-step label words: the carry goes
    upward only."""
    inst = synth.make_instance(40, 24, 16, T, 1500, n_blobs=4, seed=T, n_seeds=4, tau_f=0.3,
                               tau_p=0.15, attr_mode="noise")
    _assert_forward(inst, f"long T={T}", schedule=schedule)


def test_mode_switch_on_one_context():
    from paper_1903_12294_amd import Grower
    from paper_1903_12294_amd._lib import MF4DError
    _need_gpu()
    inst = synth.make_config(1, attr_mode="noise")
    args = (inst["field"], inst["xyz"], inst["attr"], inst["crit"], inst["seeds"])
    g = Grower(device=0)
    try:
        _load(g, inst)
        for mode in ("both", "forward", "both", "forward"):
            g.set_trajectory_mode(mode)
            with pytest.raises(MF4DError):
                g.read_particle_mask()  # the mode change dropped the labels
            fm, pm, _ = _grow(g, inst)
            ofm, opm, _ = oracle_grow(*args, forward_only=mode == "forward")
            assert np.array_equal(fm, ofm) and np.array_equal(pm, opm), mode
        with pytest.raises(MF4DError):
            g._check(g.lib.mf4d_set_trajectory_mode(g.ctx, 2))
    finally:
        g.close()


@pytest.mark.parametrize("seed", range(3))
def test_batched_forward(seed):
    from paper_1903_12294_amd import Grower
    from tests.test_gpu_batched import _planes_to_masks
    from tests.test_oracle_pins import _random_instance
    _need_gpu()
    rng = np.random.default_rng(700 + seed)
    X, Y, Z = (int(v) for v in rng.integers(3, 30, 3))
    T = int(rng.integers(2, 12)) if seed < 2 else 70
    P = int(rng.integers(20, 200))
    inst = _random_instance(rng, X, Y, Z, T, P, 1)
    Q = int(rng.integers(1, 60))
    vals = np.array([0.25, 0.5, 0.75, 1.0, np.inf, -np.inf], np.float32)
    crit = np.stack([vals[rng.integers(0, 4, Q)], vals[rng.integers(2, 5, Q)],
                     vals[rng.integers(0, 4, Q)], vals[rng.integers(3, 5, Q)]], 1).astype(np.float32)
    n = int(rng.integers(Q, 3 * Q + 1))
    qseeds = np.stack([rng.integers(0, X, n), rng.integers(0, Y, n), rng.integers(0, Z, n),
                       rng.integers(0, T, n), rng.integers(0, Q, n)], 1).astype(np.int32)
    print(f"[causal] batched{seed} {X}x{Y}x{Z}x{T} P={P} Q={Q}", flush=True)
    g = Grower(device=0)
    try:
        g.load_field(inst["field"])
        g.load_particles(inst["xyz"], inst["attr"])
        g.set_trajectory_mode("forward")
        g.set_queries(crit, qseeds)
        fp, pp, _ = g.grow_batched()
    finally:
        g.close()
    res = oracle_grow_queries(inst["field"], inst["xyz"], inst["attr"], crit, qseeds, forward_only=True)
    for q, (ofm, opm, _) in res.items():
        f, p = _planes_to_masks(fp, pp, inst["field"].shape, T, P, q)
        assert np.array_equal(f, golden_io.unpack_field(ofm, inst["field"].shape)), f"query {q}: field plane"
        assert np.array_equal(p, opm), f"query {q}: particle plane"
