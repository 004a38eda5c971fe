"""GPU: the Jacobi debugging schedule.  Synchronous sweeps add, from the
labels before the sweep alone, every admissible node one edge away; starting
from the admissible seeds, the sweep that adds nothing is number D + 1, D
the largest breadth-first level of the grown set (the oracle's depth).  So
the sweep count pins the schedule independently of the masks, which must
equal the oracle's as under every schedule."""
import numpy as np
import pytest

from oracle import oracle_grow
from paper_1903_12294_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _run(inst, rate=1, mode="both", cap=0):
    from paper_1903_12294_amd import Grower
    g = Grower(device=0, schedule="jacobi")
    try:
        g.load_field(inst["field"])
        if inst["xyz"] is not None:
            g.load_particles(inst["xyz"], inst["attr"], rate=rate)
        g.set_criteria(*inst["crit"])
        g.set_seeds(inst["seeds"])
        g.set_trajectory_mode(mode)
        st = g.grow()
        fm = g.read_field_mask()
        pm = g.read_particle_mask() if inst["xyz"] is not None else None
    finally:
        g.close()
    return st, fm, pm


def _random_case(seed, X, Y, Z, T, P, rate=1):
    rng = np.random.default_rng(seed)
    field = rng.random((T, Z, Y, X), dtype=np.float32)
    Tp = T * rate
    xyz = (rng.random((Tp, P, 3)) * np.array([X, Y, Z])).astype(np.float32)
    attr = rng.random((Tp, P), dtype=np.float32)
    seeds = np.stack([rng.integers(0, X, 6), rng.integers(0, Y, 6), rng.integers(0, Z, 6),
                      rng.integers(0, T, 6)], 1).astype(np.int32)
    return {"field": field, "xyz": xyz, "attr": attr, "crit": (0.35, np.inf, 0.3, np.inf), "seeds": seeds}


@pytest.mark.parametrize("name", ["config1", "config1-noise", "random", "random-rate3", "random-forward"])
def test_jacobi_sweeps_are_depth_plus_one(name):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rate, mode = 1, "both"
    if name == "config1":
        inst = synth.make_config(1)
    elif name == "config1-noise":
        inst = synth.make_config(1, attr_mode="noise")
    elif name == "random":
        inst = _random_case(1, 37, 19, 11, 6, 300)
    elif name == "random-rate3":
        rate = 3
        inst = _random_case(2, 40, 16, 9, 5, 200, rate=3)
    else:
        mode = "forward"
        inst = _random_case(3, 33, 17, 10, 7, 250)
    print(f"[jacobi] {name}", flush=True)
    st, fm, pm = _run(inst, rate=rate, mode=mode)
    ofm, opm, ost = oracle_grow(inst["field"], inst["xyz"], inst["attr"], inst["crit"], inst["seeds"],
                                rate=rate, forward_only=mode == "forward")
    assert np.array_equal(fm, ofm)
    assert np.array_equal(pm, opm)
    assert st["rounds"] == ost["depth"] + 1, (st["rounds"], ost["depth"])
    assert ost["depth"] > 3


def test_jacobi_cap_then_resume():
    """A cap of k sweeps leaves exactly the nodes within k edges of the seeds
    (a subset of the result), and resuming reaches the result."""
    from paper_1903_12294_amd import Grower
    from paper_1903_12294_amd._lib import MF4DError
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    inst = synth.make_config(1)
    ofm, opm, ost = oracle_grow(inst["field"], inst["xyz"], inst["attr"], inst["crit"], inst["seeds"])
    g = Grower(device=0, schedule="jacobi")
    try:
        g.load_field(inst["field"])
        g.load_particles(inst["xyz"], inst["attr"])
        g.set_criteria(*inst["crit"])
        g.set_seeds(inst["seeds"])
        g.set_max_rounds(2)
        with pytest.raises(MF4DError):
            g.grow()
        part = g.read_field_mask()
        assert np.array_equal(part & ofm, part) and not np.array_equal(part, ofm)
        g.set_max_rounds(0)
        st = g.grow_resume()
        assert np.array_equal(g.read_field_mask(), ofm)
        assert np.array_equal(g.read_particle_mask(), opm)
        assert st["rounds"] == ost["depth"] + 1
    finally:
        g.close()
