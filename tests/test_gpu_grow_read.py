"""GPU: mf4d_grow_read (the grow with both read-outs queued behind its rounds)
against the oracle and against mf4d_grow followed by the two read calls:
both schedules, every tile depth, eager and lazy admissibility, grows that
need several chunks of queued rounds (gated read-outs that must stay no-ops
until the last chunk), a round cap (masks as the cap left the labels, then a
resume), one read-out skipped, criteria changed between calls, and the
schedulers that read out after the grow instead (score-ordered, Jacobi,
phase timing).  Output buffers start filled with ones, so a read-out that
did not run shows."""
import numpy as np
import pytest

from oracle import oracle_grow
from paper_1903_12294_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _grower(inst, **kw):
    from paper_1903_12294_amd import Grower
    g = Grower(device=0, **kw)
    g.load_field(inst["field"])
    g.load_particles(inst["xyz"], inst["attr"])
    g.set_criteria(*inst["crit"])
    g.set_seeds(inst["seeds"])
    return g


def _buffers(g):
    dev = torch.device("cuda:0")
    fm = torch.full((g.field_words(),), -1, dtype=torch.int32, device=dev)
    pm = torch.full((g.Tp, g.P), 0xFF, dtype=torch.uint8, device=dev)
    return fm, pm


def _host(fm, pm):
    torch.cuda.synchronize()
    return fm.cpu().numpy().view(np.uint32), pm.cpu().numpy()


def _oracle(inst, crit=None):
    ofm, opm, ost = oracle_grow(inst["field"], inst["xyz"], inst["attr"],
                                inst["crit"] if crit is None else crit, inst["seeds"])
    return ofm, opm, ost


@pytest.mark.parametrize("schedule,tile_t,admit", [
    ("launch", 4, "tiles"), ("launch", 8, "all"), ("launch", 16, "tiles"),
    ("persistent", 4, "all"), ("persistent", 8, "tiles"), ("persistent", 16, "tiles"),
])
@pytest.mark.parametrize("cfg,mode", [(1, "noise"), (2, "noise"), (2, "field")])
def test_grow_read_equals_oracle(cfg, mode, schedule, tile_t, admit):
    _need_gpu()
    inst = synth.make_config(cfg, attr_mode=mode)
    ofm, opm, ost = _oracle(inst)
    print(f"[grow_read] config {cfg} {mode} {schedule} bt={tile_t} {admit}", flush=True)
    g = _grower(inst, tile_t=tile_t, schedule=schedule, admit=admit)
    try:
        fm, pm = _buffers(g)
        for rep in range(3):  # the first grow of a context queues 4 rounds per chunk
            fm.fill_(-1)
            pm.fill_(0xFF)
            st = g.grow_read(fm, pm)
            hf, hp = _host(fm, pm)
            assert np.array_equal(hf, ofm), rep
            assert np.array_equal(hp, opm), rep
            full = g.stats()
            assert full["members_field"] == ost["members_field"]
            assert full["members_particle"] == ost["members_particle"]
        # (round and visit counts depend on the order in which concurrent
        # sweeps see each other's bits; the masks do not)
        assert st["rounds"] > 0 and st["tile_visits"] > 0
    finally:
        g.close()


def test_grow_read_over_several_chunks():
    """A fresh context queues 4 rounds per chunk: a grow of more rounds runs
    gated read-outs that must do nothing until the fixed point."""
    _need_gpu()
    inst = synth.make_config(1, attr_mode="noise")
    ofm, opm, _ = _oracle(inst)
    g = _grower(inst, tile_t=4, schedule="launch")
    try:
        fm, pm = _buffers(g)
        st = g.grow_read(fm, pm)
        assert st["rounds"] > 4, st["rounds"]
        hf, hp = _host(fm, pm)
        assert np.array_equal(hf, ofm) and np.array_equal(hp, opm)
    finally:
        g.close()


@pytest.mark.parametrize("schedule", ["launch", "persistent"])
def test_grow_read_round_cap_then_resume(schedule):
    from paper_1903_12294_amd import MF4DError, _lib
    _need_gpu()
    inst = synth.make_config(1, attr_mode="noise")
    ofm, opm, _ = _oracle(inst)
    g = _grower(inst, tile_t=4, schedule=schedule)
    ref = _grower(inst, tile_t=4, schedule=schedule)
    try:
        fm, pm = _buffers(g)
        for cap in (1, 2, 3):
            g.set_max_rounds(cap)
            ref.set_max_rounds(cap)
            fm.fill_(-1)
            pm.fill_(0xFF)
            with pytest.raises(MF4DError) as e:
                g.grow_read(fm, pm)
            assert e.value.code == _lib.MF4D_ERR_NOT_CONVERGED
            with pytest.raises(MF4DError):
                ref.grow()
            hf, hp = _host(fm, pm)
            assert np.array_equal(hf, ref.read_field_mask()), cap
            assert np.array_equal(hp, ref.read_particle_mask()), cap
            assert not (hf & ~ofm).any() and not (hp & ~opm).any()
        g.set_max_rounds(0)
        g.grow_resume()
        assert np.array_equal(g.read_field_mask(), ofm)
        assert np.array_equal(g.read_particle_mask(), opm)
    finally:
        g.close()
        ref.close()


def test_grow_read_one_output_and_criteria_changes():
    _need_gpu()
    inst = synth.make_config(1, attr_mode="noise")
    g = _grower(inst, schedule="launch")
    try:
        fm, pm = _buffers(g)
        for k, crit in enumerate(([0.1, np.inf, 0.1, np.inf], [0.5, np.inf, 0.5, np.inf],
                                  [0.3, 0.6, 0.2, 0.9], [0.3, np.inf, 0.3, np.inf])):
            crit = np.array(crit, np.float32)
            g.set_criteria(*crit)
            ofm, opm, _ = _oracle(inst, crit)
            fm.fill_(-1)
            pm.fill_(0xFF)
            if k % 2 == 0:
                g.grow_read(fm, None)
                hf, hp = _host(fm, pm)
                assert np.array_equal(hf, ofm) and (hp == 0xFF).all(), crit
            else:
                g.grow_read(None, pm)
                hf, hp = _host(fm, pm)
                assert np.array_equal(hp, opm) and (hf == 0xFFFFFFFF).all(), crit
            # the separate read calls see the same labels afterwards
            assert np.array_equal(g.read_field_mask(), ofm)
            assert np.array_equal(g.read_particle_mask(), opm)
    finally:
        g.close()


@pytest.mark.parametrize("variant", ["heuristic", "jacobi", "timing"])
def test_grow_read_with_read_after_grow(variant):
    _need_gpu()
    inst = synth.make_config(1, attr_mode="noise")
    ofm, opm, _ = _oracle(inst)
    g = _grower(inst, schedule="launch")
    try:
        if variant == "heuristic":
            g.set_scheduler("heuristic")
        elif variant == "jacobi":
            g.set_schedule("jacobi")
        else:
            g.set_phase_timing(True)
        fm, pm = _buffers(g)
        st = g.grow_read(fm, pm)
        hf, hp = _host(fm, pm)
        assert np.array_equal(hf, ofm) and np.array_equal(hp, opm)
        if variant == "timing":
            assert st["ms_rounds"] > 0
    finally:
        g.close()


def test_grow_read_rejects_bad_buffers():
    from paper_1903_12294_amd import MF4DError
    _need_gpu()
    inst = synth.make_config(1)
    g = _grower(inst)
    try:
        dev = torch.device("cuda:0")
        with pytest.raises(MF4DError):
            g.grow_read(torch.zeros(g.field_words() - 1, dtype=torch.int32, device=dev), None)
        with pytest.raises(MF4DError):
            g.grow_read(None, torch.zeros(g.Tp * g.P - 1, dtype=torch.uint8, device=dev))
        with pytest.raises(ValueError):
            g.grow_read(np.zeros(g.field_words(), np.uint32), None)
    finally:
        g.close()


def test_grow_read_without_statistics():
    """stats=False passes no statistics buffer; the masks and the statistics
    read afterwards are those of the grow."""
    _need_gpu()
    inst = synth.make_config(1, attr_mode="noise")
    ofm, opm, ost = _oracle(inst)
    g = _grower(inst, schedule="launch")
    try:
        fm, pm = _buffers(g)
        assert g.grow_read(fm, pm, stats=False) is None
        hf, hp = _host(fm, pm)
        assert np.array_equal(hf, ofm) and np.array_equal(hp, opm)
        st = g.stats()
        assert st["members_field"] == ost["members_field"]
        assert st["members_particle"] == ost["members_particle"]
    finally:
        g.close()
