"""GPU parity of the per-seed component ids (mf4d_grow_seed_ids) against the
oracle's one-grow-per-seed definition, element for element, under both
trajectory modes."""
import numpy as np
import pytest

from oracle import oracle_grow, oracle_seed_ids
from paper_1903_12294_amd import synth
from tests import golden_io

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _ids_gpu(inst, mode, device_out=False, schedule=None):
    from paper_1903_12294_amd import Grower
    _need_gpu()
    dev = torch.device("cuda:0")
    T, Z, Y, X = inst["field"].shape
    P = inst["xyz"].shape[1]
    g = Grower(device=0, schedule=schedule)
    try:
        g.load_field(torch.from_numpy(np.ascontiguousarray(inst["field"])).to(dev))
        if P:
            g.load_particles(torch.from_numpy(np.ascontiguousarray(inst["xyz"])).to(dev),
                             torch.from_numpy(np.ascontiguousarray(inst["attr"])).to(dev))
        g.set_criteria(*inst["crit"])
        g.set_seeds(np.asarray(inst["seeds"], np.int32).reshape(-1, 4))
        g.set_trajectory_mode(mode)
        if device_out:
            fo = torch.full((T, Z, Y, X), 9, dtype=torch.int32, device=dev)
            po = torch.full((T, P), 9, dtype=torch.int32, device=dev)
            _, _, n = g.grow_seed_ids(fo, po)
            fid, pid = fo.cpu().numpy(), po.cpu().numpy()
        else:
            fid, pid, n = g.grow_seed_ids()
    finally:
        g.close()
    return fid, pid, n


def _assert_ids(inst, tag, mode="both", **kw):
    print(f"[seed-ids] {tag} field {inst['field'].shape} P={inst['xyz'].shape[1]} "
          f"S={len(inst['seeds'])} {mode} {kw}", flush=True)
    fid, pid, n = _ids_gpu(inst, mode, **kw)
    ofid, opid = oracle_seed_ids(inst["field"], inst["xyz"], inst["attr"], inst["crit"], inst["seeds"],
                                 forward_only=mode == "forward")
    assert np.array_equal(fid, ofid), f"{tag}: {int((fid != ofid).sum())} field ids differ"
    assert np.array_equal(pid, opid), f"{tag}: {int((pid != opid).sum())} particle ids differ"
    assert n <= len(inst["seeds"])
    return fid, pid, n


@pytest.mark.parametrize("mode", ["both", "forward"])
@pytest.mark.parametrize("case", golden_io.all_cases(), ids=lambda c: c["name"])
def test_golden_fixtures(case, mode):
    _assert_ids(dict(case), case["name"], mode)


@pytest.mark.parametrize("seed", range(10))
def test_random_small_ragged(seed):
    from tests.test_oracle_pins import _random_instance
    rng = np.random.default_rng(4000 + seed)
    X, Y, Z = (int(v) for v in rng.integers(1, 40, 3))
    T = int(rng.integers(1, 16))
    P = int(rng.integers(0, 250))
    S = int(rng.integers(0, 9))
    inst = _random_instance(rng, X, Y, Z, T, P, S)
    if S >= 2:
        inst["seeds"][-1] = inst["seeds"][0]  # a duplicate
    _assert_ids(inst, f"random{seed}", ["both", "forward"][seed % 2],
                device_out=seed % 3 == 0, schedule=["persistent", "launch"][(seed // 2) % 2])


@pytest.mark.parametrize("mode", ["both", "forward"])
def test_32cube_workload_many_seeds(mode):
    """64 seeds on the 32^3 x 8 workload with a narrower field band (f >= 0.5,
    which splits the blobs into separate components): its own seed, 48
    admissible voxels and 15 random ones.  Fewer grows than seeds, and more
    than one id in use."""
    inst = synth.make_config(1, attr_mode="noise")
    inst["crit"] = np.array([0.5, np.inf, inst["crit"][2], inst["crit"][3]], np.float32)
    f = inst["field"]
    rng = np.random.default_rng(9)
    adm = np.argwhere(f >= np.float32(0.5))
    pick = adm[rng.choice(len(adm), 48, replace=False)][:, ::-1].astype(np.int32)
    rnd = np.stack([rng.integers(0, 32, 15), rng.integers(0, 32, 15), rng.integers(0, 32, 15),
                    rng.integers(0, 8, 15)], 1).astype(np.int32)
    inst["seeds"] = np.concatenate([np.asarray(inst["seeds"], np.int32).reshape(-1, 4), pick, rnd])
    fid, pid, n = _assert_ids(inst, "32^3x8 x 64 seeds", mode, device_out=True)
    assert n < 64 and len(np.unique(fid[fid >= 0])) > 1
    # the labelled nodes are the union grow
    fm, pm, _ = oracle_grow(inst["field"], inst["xyz"], inst["attr"], inst["crit"], inst["seeds"],
                            forward_only=mode == "forward")
    V = inst["field"].size
    bits = np.unpackbits(fm.view(np.uint8), bitorder="little")[:V].astype(bool)
    assert np.array_equal(fid.ravel() >= 0, bits) and np.array_equal(pid >= 0, pm != 0)


def test_state_after_ids():
    from paper_1903_12294_amd import Grower
    from paper_1903_12294_amd._lib import MF4DError
    _need_gpu()
    inst = synth.make_config(1)
    g = Grower(device=0)
    try:
        g.load_field(inst["field"])
        g.load_particles(inst["xyz"], inst["attr"])
        with pytest.raises(MF4DError):
            g.grow_seed_ids()  # no criteria
        g.set_criteria(*inst["crit"])
        g.set_seeds(inst["seeds"])
        g.grow_seed_ids()
        with pytest.raises(MF4DError):
            g.read_field_mask()  # the ids leave no grown labels
        g.grow()
        fm, pm = g.read_field_mask(), g.read_particle_mask()
        ofm, opm, _ = oracle_grow(inst["field"], inst["xyz"], inst["attr"], inst["crit"], inst["seeds"])
        assert np.array_equal(fm, ofm) and np.array_equal(pm, opm)
        g.set_seeds(np.zeros((0, 4), np.int32))
        fid, pid, n = g.grow_seed_ids()
        assert n == 0 and (fid == -1).all() and (pid == -1).all()
    finally:
        g.close()
