"""GPU: asynchronous read-outs (mf4d_set_read_async).  A run of grow_read
calls with changing criteria, each into its own output buffers, alternates
the two label sets while earlier read-outs may still be writing; after
read_wait every buffer holds its own grow's masks (against the oracle).
Calls in between (a synchronous read of the same labels, statistics, a
capped grow and its resume, clearing the labels, switching the mode off)
are ordered after the read-outs still running."""
import numpy as np
import pytest

from oracle import oracle_grow
from paper_1903_12294_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CRITS = ([0.3, np.inf, 0.3, np.inf], [0.1, np.inf, 0.1, np.inf], [0.5, np.inf, 0.5, np.inf],
         [0.3, 0.6, 0.2, 0.9], [0.05, np.inf, 0.05, np.inf], [0.3, np.inf, 0.3, np.inf])


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _grower(inst, **kw):
    from paper_1903_12294_amd import Grower
    g = Grower(device=0, **kw)
    g.load_field(inst["field"])
    g.load_particles(inst["xyz"], inst["attr"])
    g.set_seeds(inst["seeds"])
    return g


def _bufs(g):
    dev = torch.device("cuda:0")
    return (torch.full((g.field_words(),), -1, dtype=torch.int32, device=dev),
            torch.full((g.Tp, g.P), 0xFF, dtype=torch.uint8, device=dev))


@pytest.mark.parametrize("schedule,tile_t", [("launch", 16), ("launch", 4), ("persistent", 8)])
def test_async_runs_equal_oracle(schedule, tile_t):
    _need_gpu()
    inst = synth.make_config(1, attr_mode="noise")
    want = [oracle_grow(inst["field"], inst["xyz"], inst["attr"], np.array(c, np.float32), inst["seeds"])
            for c in CRITS]
    g = _grower(inst, tile_t=tile_t, schedule=schedule)
    try:
        g.set_read_async(True)
        outs = []
        for rep in range(2):
            for c in CRITS:
                g.set_criteria(*np.array(c, np.float32))
                fm, pm = _bufs(g)
                g.grow_read(fm, pm)
                outs.append((fm, pm))
        g.read_wait()
        torch.cuda.synchronize()
        for i, (fm, pm) in enumerate(outs):
            ofm, opm, _ = want[i % len(CRITS)]
            assert np.array_equal(fm.cpu().numpy().view(np.uint32), ofm), i
            assert np.array_equal(pm.cpu().numpy(), opm), i
        st = g.stats()  # settles the member counts of the last grow
        assert st["members_field"] == want[-1][2]["members_field"]
        assert st["members_particle"] == want[-1][2]["members_particle"]
    finally:
        g.close()


def test_async_calls_in_between():
    from paper_1903_12294_amd import MF4DError
    _need_gpu()
    inst = synth.make_config(1, attr_mode="noise")
    crit = np.array(CRITS[0], np.float32)
    ofm, opm, _ = oracle_grow(inst["field"], inst["xyz"], inst["attr"], crit, inst["seeds"])
    g = _grower(inst, tile_t=4, schedule="launch")
    try:
        g.set_criteria(*crit)
        g.set_read_async(True)
        fm, pm = _bufs(g)
        g.grow_read(fm, pm)
        # a synchronous read of the same labels, queued while the read-outs run
        assert np.array_equal(g.read_field_mask(), ofm)
        assert np.array_equal(g.read_particle_mask(), opm)
        torch.cuda.synchronize()
        assert np.array_equal(fm.cpu().numpy().view(np.uint32), ofm)
        # a capped grow: the masks as the cap left them, then the resume
        g.set_max_rounds(1)
        fm2, pm2 = _bufs(g)
        with pytest.raises(MF4DError):
            g.grow_read(fm2, pm2)
        g.set_max_rounds(0)
        g.grow_resume()
        assert np.array_equal(g.read_field_mask(), ofm)
        assert np.array_equal(g.read_particle_mask(), opm)
        torch.cuda.synchronize()
        part = fm2.cpu().numpy().view(np.uint32)
        assert not (part & ~ofm).any() and (part != 0).any()
        # clearing the labels after an asynchronous grow
        fm3, pm3 = _bufs(g)
        g.grow_read(fm3, pm3)
        g.reset_labels()
        torch.cuda.synchronize()
        assert np.array_equal(fm3.cpu().numpy().view(np.uint32), ofm)
        assert np.array_equal(pm3.cpu().numpy(), opm)
        # mode off: grow_read is stream-ordered again
        g.set_read_async(False)
        fm4, pm4 = _bufs(g)
        g.grow_read(fm4, pm4)
        assert np.array_equal(fm4.cpu().numpy().view(np.uint32), ofm)
        assert np.array_equal(pm4.cpu().numpy(), opm)
    finally:
        g.close()


def test_async_then_verification_round():
    """A score-ordered scheduler's verification pull tests every tile that
    holds an admissible voxel-step; label words of other tiles are left from
    earlier grows (or from the other label set) and must not join."""
    _need_gpu()
    inst = synth.make_config(1, attr_mode="noise")
    g = _grower(inst, tile_t=8, schedule="launch")
    try:
        g.set_read_async(True)
        for c in ([0.1, np.inf, 0.1, np.inf], [0.05, np.inf, 0.05, np.inf]):
            g.set_criteria(*np.array(c, np.float32))
            fm, pm = _bufs(g)
            g.grow_read(fm, pm)
        g.set_scheduler("heuristic")
        crit = np.array([0.5, np.inf, 0.5, np.inf], np.float32)
        g.set_criteria(*crit)
        ofm, opm, _ = oracle_grow(inst["field"], inst["xyz"], inst["attr"], crit, inst["seeds"])
        st = g.grow()
        assert st["verify_rounds"] == 1
        assert np.array_equal(g.read_field_mask(), ofm)
        assert np.array_equal(g.read_particle_mask(), opm)
    finally:
        g.close()
