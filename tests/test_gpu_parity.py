"""GPU parity: the HIP grower (called through the C ABI) against the CPU oracle,
bit for bit, on the same seeded inputs."""
import numpy as np
import pytest

from oracle import check_invariants, oracle_grow
from paper_1903_12294_amd import synth
from tests import golden_io

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _grow_gpu(inst, tile_t=None, device_inputs=True, crit=None, seeds=None, schedule=None,
             admit=None):
    from paper_1903_12294_amd import Grower
    _need_gpu()
    g = Grower(device=0, tile_t=tile_t, schedule=schedule, admit=admit)
    try:
        if device_inputs:
            dev = torch.device("cuda:0")
            g.load_field(torch.from_numpy(np.ascontiguousarray(inst["field"])).to(dev))
            if inst["xyz"] is not None and inst["xyz"].shape[1] > 0:
                g.load_particles(torch.from_numpy(np.ascontiguousarray(inst["xyz"])).to(dev),
                                 torch.from_numpy(np.ascontiguousarray(inst["attr"])).to(dev))
        else:
            g.load_field(inst["field"])
            if inst["xyz"] is not None and inst["xyz"].shape[1] > 0:
                g.load_particles(inst["xyz"], inst["attr"])
        g.set_criteria(*(inst["crit"] if crit is None else crit))
        g.set_seeds(np.asarray(inst["seeds"] if seeds is None else seeds, np.int32).reshape(-1, 4))
        st = g.grow()
        fm = g.read_field_mask()
        P = 0 if inst["xyz"] is None else inst["xyz"].shape[1]
        pm = g.read_particle_mask() if P > 0 else np.zeros((inst["field"].shape[0], 0), np.uint8)
        st = g.stats()
    finally:
        g.close()
    return fm, pm, st


def _assert_parity(inst, tag="", **kw):
    print(f"[parity] {tag} field {inst['field'].shape} P={inst['xyz'].shape[1]} {kw}", flush=True)
    fm, pm, st = _grow_gpu(inst, **kw)
    ofm, opm, ost = oracle_grow(inst["field"], inst["xyz"], inst["attr"], inst["crit"],
                                inst["seeds"])
    assert np.array_equal(fm, ofm), f"{tag}: field mask differs " \
        f"({int(np.unpackbits(fm.view(np.uint8)).sum())} vs {ost['members_field']} members)"
    assert np.array_equal(pm, opm), f"{tag}: particle mask differs " \
        f"({int(pm.sum())} vs {ost['members_particle']})"
    assert st["members_field"] == ost["members_field"]
    assert st["members_particle"] == ost["members_particle"]
    assert st["seeds_dropped"] == ost["seeds_dropped"]
    return st, ost


@pytest.mark.parametrize("admit", ["tiles", "all"])
@pytest.mark.parametrize("schedule", ["persistent", "launch"])
@pytest.mark.parametrize("case", golden_io.all_cases(), ids=lambda c: c["name"])
def test_golden_fixtures_on_gpu(case, schedule, admit):
    inst = dict(case)
    _assert_parity(inst, tag=case["name"], schedule=schedule, admit=admit)


@pytest.mark.parametrize("seed", range(24))
def test_random_small_ragged(seed):
    from tests.test_oracle_pins import _random_instance
    rng = np.random.default_rng(1000 + seed)
    X, Y, Z = (int(v) for v in rng.integers(1, 70, 3))
    T = int(rng.integers(1, 20))
    P = int(rng.integers(0, 300))
    inst = _random_instance(rng, X, Y, Z, T, P, 5)
    _assert_parity(inst, tag=f"random{seed}", tile_t=[4, 8, 16][seed % 3],
                   schedule=["persistent", "launch"][(seed // 3) % 2],
                   admit=["tiles", "all"][(seed // 6) % 2])


@pytest.mark.parametrize("schedule", ["persistent", "launch"])
@pytest.mark.parametrize("tile_t", [4, 8, 16])
@pytest.mark.parametrize("variant", ["field", "noise", "stress_tau"])
def test_config1(tile_t, variant, schedule):
    kw = dict(attr_mode="noise") if variant == "noise" else (
        dict(tau_p_offset=-0.15) if variant == "stress_tau" else {})
    inst = synth.make_config(1, **kw)
    _assert_parity(inst, tag=f"cfg1-{variant}", tile_t=tile_t, schedule=schedule)


def test_config1_host_inputs():
    inst = synth.make_config(1)
    _assert_parity(inst, tag="cfg1-host", device_inputs=False)


@pytest.mark.parametrize("shape", [(45, 37, 29, 11, 3000), (100, 9, 70, 5, 5000),
                                   (33, 64, 17, 67, 2000)])
def test_ragged_multi_tile(shape):
    X, Y, Z, T, P = shape
    inst = synth.make_instance(X, Y, Z, T, P, n_blobs=5, seed=sum(shape), n_seeds=4,
                               tau_f=0.3, tau_p=0.2)
    _assert_parity(inst, tag=f"ragged{shape}")


@pytest.mark.parametrize("admit", ["tiles", "all"])
@pytest.mark.parametrize("schedule", ["persistent", "launch"])
@pytest.mark.parametrize("variant", ["field", "noise"])
def test_config2(variant, schedule, admit):
    inst = synth.make_config(2, attr_mode=variant)
    st, ost = _assert_parity(inst, tag=f"cfg2-{variant}", schedule=schedule, admit=admit)
    print(f"[cfg2] rounds {st['rounds']} visits {st['tile_visits']} depth {ost['depth']}")


def test_config2_invariants_and_all_admissible():
    inst = synth.make_config(1)
    crit = np.array([-np.inf, np.inf, -np.inf, np.inf], np.float32)
    fm, pm, _ = _grow_gpu(inst, crit=crit)
    ofm, opm, _ = oracle_grow(inst["field"], inst["xyz"], inst["attr"], crit, inst["seeds"])
    assert np.array_equal(fm, ofm) and np.array_equal(pm, opm)
    fm, pm, _ = _grow_gpu(inst)
    Mf = golden_io.unpack_field(fm, inst["field"].shape)
    inv = check_invariants(inst["field"], inst["xyz"], inst["attr"], inst["crit"], inst["seeds"],
                           Mf, pm.astype(bool))
    assert all(inv.values()), inv


def test_empty_seeds_and_dropped():
    inst = synth.make_config(1)
    fm, pm, st = _grow_gpu(inst, seeds=np.zeros((0, 4), np.int32))
    assert not fm.any() and not pm.any() and st["rounds"] == 0
    crit = np.array([np.inf, np.inf, np.inf, np.inf], np.float32)
    fm, pm, st = _grow_gpu(inst, crit=crit)
    assert not fm.any() and st["seeds_dropped"] == len(inst["seeds"])


def test_errors_leave_state_unchanged():
    from paper_1903_12294_amd import Grower, MF4DError
    from paper_1903_12294_amd import _lib
    _need_gpu()
    inst = synth.make_config(1)
    g = Grower(device=0)
    try:
        with pytest.raises(MF4DError) as e:
            g.grow()
        assert e.value.code == _lib.MF4D_ERR_STATE
        g.load_field(inst["field"])
        g.load_particles(inst["xyz"], inst["attr"])
        g.set_criteria(*inst["crit"])
        g.set_seeds(inst["seeds"])
        with pytest.raises(MF4DError) as e:
            g.set_seeds(np.array([[32, 0, 0, 0]], np.int32))
        assert e.value.code == _lib.MF4D_ERR_RANGE
        with pytest.raises(MF4DError) as e:
            g.set_criteria(np.nan, 1, 0, 1)
        assert e.value.code == _lib.MF4D_ERR_ARG
        with pytest.raises(MF4DError) as e:
            g.load_particles(inst["xyz"][:4], inst["attr"][:4])
        assert e.value.code == _lib.MF4D_ERR_ARG
        g.grow()
        fm = g.read_field_mask()
        with pytest.raises(MF4DError) as e:
            g.read_field_mask(np.zeros(3, np.uint32))
        assert e.value.code == _lib.MF4D_ERR_ARG
    finally:
        g.close()
    ofm, _, _ = oracle_grow(inst["field"], inst["xyz"], inst["attr"], inst["crit"], inst["seeds"])
    assert np.array_equal(fm, ofm)


@pytest.mark.parametrize("schedule", ["persistent", "launch"])
def test_round_cap_then_resume(schedule):
    from paper_1903_12294_amd import Grower, MF4DError
    from paper_1903_12294_amd import _lib
    _need_gpu()
    inst = synth.make_config(1, attr_mode="noise")
    ofm, opm, _ = oracle_grow(inst["field"], inst["xyz"], inst["attr"], inst["crit"],
                              inst["seeds"])
    g = Grower(device=0, tile_t=4, schedule=schedule)
    try:
        g.load_field(inst["field"])
        g.load_particles(inst["xyz"], inst["attr"])
        g.set_criteria(*inst["crit"])
        g.set_seeds(inst["seeds"])
        g.set_max_rounds(1)
        with pytest.raises(MF4DError) as e:
            g.grow()
        assert e.value.code == _lib.MF4D_ERR_NOT_CONVERGED
        fm = g.read_field_mask()
        pm = g.read_particle_mask()
        Mf = golden_io.unpack_field(fm, inst["field"].shape)
        inv = check_invariants(inst["field"], inst["xyz"], inst["attr"], inst["crit"],
                               inst["seeds"], Mf, pm.astype(bool))
        # a valid partial result: admissible, seeded, connected -- but not closed yet
        assert inv["I1"] and inv["I2"] and inv["I4"] and not inv["I3"]
        assert not (fm & ~ofm).any() and not (pm & ~opm).any()
        g.set_max_rounds(0)
        g.grow_resume()
        assert np.array_equal(g.read_field_mask(), ofm)
        assert np.array_equal(g.read_particle_mask(), opm)
    finally:
        g.close()


@pytest.mark.parametrize("schedule", ["persistent", "launch"])
def test_repeat_grows_identical(schedule):
    inst = synth.make_config(2, attr_mode="noise")
    from paper_1903_12294_amd import Grower
    _need_gpu()
    g = Grower(device=0, schedule=schedule)
    try:
        g.load_field(inst["field"])
        g.load_particles(inst["xyz"], inst["attr"])
        g.set_criteria(*inst["crit"])
        g.set_seeds(inst["seeds"])
        outs = []
        for _ in range(5):
            g.grow()
            outs.append((g.read_field_mask().copy(), g.read_particle_mask().copy()))
    finally:
        g.close()
    for f, p in outs[1:]:
        assert np.array_equal(f, outs[0][0]) and np.array_equal(p, outs[0][1])


def test_criteria_change_between_grows():
    """Labels and admissibility of tiles that stop being candidates must not
    leak into the next grow (tiles are skipped, not cleared)."""
    from paper_1903_12294_amd import Grower
    _need_gpu()
    inst = synth.make_config(1, attr_mode="noise")
    g = Grower(device=0)
    try:
        g.load_field(inst["field"])
        g.load_particles(inst["xyz"], inst["attr"])
        g.set_seeds(inst["seeds"])
        for crit in ([0.1, np.inf, 0.1, np.inf], [0.5, np.inf, 0.5, np.inf],
                     [0.3, 0.6, 0.2, 0.9], [0.05, np.inf, 0.05, np.inf], [0.3, np.inf, 0.3, np.inf]):
            crit = np.array(crit, np.float32)
            g.set_criteria(*crit)
            g.grow()
            fm, pm = g.read_field_mask(), g.read_particle_mask()
            ofm, opm, _ = oracle_grow(inst["field"], inst["xyz"], inst["attr"], crit, inst["seeds"])
            assert np.array_equal(fm, ofm) and np.array_equal(pm, opm), crit
    finally:
        g.close()


@pytest.mark.parametrize("tau_p", [0.70, 0.75, 0.9])
def test_coupled_list_staging_many_iterations(tau_p):
    """Enough particle-steps (64 x 300,000) that each block of the particle
    admissibility pass runs many iterations, with an independent-noise
    attribute whose threshold puts an iteration's coupled entries near, above
    and below what a block stages (flushes and direct writes mixed)."""
    inst = synth.make_instance(64, 64, 64, 64, 300000, n_blobs=8, seed=17, n_seeds=8,
                               tau_f=0.3, tau_p=tau_p, attr_mode="noise")
    for schedule in ("persistent", "launch"):
        _assert_parity(inst, tag=f"staging tau_p={tau_p} {schedule}", schedule=schedule)


@pytest.mark.parametrize("schedule", ["persistent", "launch"])
@pytest.mark.parametrize("T", [67, 130])
def test_long_trajectories(T, schedule):
    """More than 64 steps per particle (two or three label words): runs of
    admissible steps cross word boundaries (independent-noise attribute, 85%
    admissible), so the close phase carries across words."""
    inst = synth.make_instance(40, 24, 16, T, 1500, n_blobs=4, seed=T, n_seeds=4, tau_f=0.3,
                               tau_p=0.15, attr_mode="noise")
    _assert_parity(inst, tag=f"long T={T} {schedule}", schedule=schedule)


@pytest.mark.parametrize("schedule", ["persistent", "launch"])
def test_phase_timing_fills_device_times(schedule):
    """With phase timing on, a grow (and a capped grow then its resume)
    reports device times of its phases, and the masks are the oracle's;
    with it off the times read 0."""
    from paper_1903_12294_amd import Grower
    from paper_1903_12294_amd._lib import MF4DError
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    inst = synth.make_config(1)
    ofm, opm, _ = oracle_grow(inst["field"], inst["xyz"], inst["attr"], inst["crit"], inst["seeds"])
    g = Grower(device=0, schedule=schedule)
    try:
        g.load_field(inst["field"])
        g.load_particles(inst["xyz"], inst["attr"])
        g.set_criteria(*inst["crit"])
        g.set_seeds(inst["seeds"])
        g.set_phase_timing(True)
        st = g.grow()
        assert st["ms_total"] > 0 and st["ms_rounds"] > 0 and st["ms_admit"] > 0
        assert np.array_equal(g.read_field_mask(), ofm) and np.array_equal(g.read_particle_mask(), opm)
        g.set_max_rounds(1)
        with pytest.raises(MF4DError):
            g.grow()
        g.set_max_rounds(0)
        st = g.grow_resume()
        assert st["ms_rounds"] > 0
        assert np.array_equal(g.read_field_mask(), ofm)
        g.set_phase_timing(False)
        st = g.grow()
        assert st["ms_total"] == 0
        assert np.array_equal(g.read_field_mask(), ofm) and np.array_equal(g.read_particle_mask(), opm)
        assert g.stats()["members_particle"] == int(opm.sum())
    finally:
        g.close()
