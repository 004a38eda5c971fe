"""GPU: mf4d_grow_submit / mf4d_grow_finish.  Two contexts loaded with the
same data keep two grows in flight with changing criteria, each into its own
buffers, against the oracle; a fresh context's first grow needs more rounds
than its first queued chunk; a round cap and its resume; a call in between
completes the submitted grow and keeps its result; the state errors; the
configurations that grow at once on submit."""
import numpy as np
import pytest

from oracle import oracle_grow
from paper_1903_12294_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CRITS = ([0.3, np.inf, 0.3, np.inf], [0.1, np.inf, 0.1, np.inf], [0.5, np.inf, 0.5, np.inf],
         [0.3, 0.6, 0.2, 0.9], [0.05, np.inf, 0.05, np.inf])


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _grower(inst, stream=None, **kw):
    from paper_1903_12294_amd import Grower
    g = Grower(device=0, stream=stream, **kw)
    g.load_field(inst["field"])
    g.load_particles(inst["xyz"], inst["attr"])
    g.set_criteria(*inst["crit"])
    g.set_seeds(inst["seeds"])
    return g


def _bufs(g):
    dev = torch.device("cuda:0")
    out = (torch.full((g.field_words(),), -1, dtype=torch.int32, device=dev),
           torch.full((g.Tp, g.P), 0xFF, dtype=torch.uint8, device=dev))
    torch.cuda.synchronize()  # filled before another stream writes them
    return out


def _host(fm, pm):
    torch.cuda.synchronize()
    return fm.cpu().numpy().view(np.uint32), pm.cpu().numpy()


@pytest.mark.parametrize("tile_t", [4, 16])
def test_two_contexts_in_flight_equal_oracle(tile_t):
    _need_gpu()
    inst = synth.make_config(1, attr_mode="noise")
    want = [oracle_grow(inst["field"], inst["xyz"], inst["attr"], np.array(c, np.float32), inst["seeds"])
            for c in CRITS]
    streams = [torch.cuda.Stream(device=0) for _ in range(2)]
    gs = [_grower(inst, stream=s.cuda_stream, tile_t=tile_t) for s in streams]
    try:
        coupled = []  # each criterion's coupled steps, from a grow on its own
        for c in CRITS:
            gs[0].set_criteria(*np.array(c, np.float32))
            coupled.append(gs[0].grow()["coupled_steps"])
        outs, pending = [], [None, None]
        for i in range(3 * len(CRITS)):
            k = i & 1
            g = gs[k]
            if pending[k] is not None:
                j, fm, pm = pending[k]
                st = g.grow_finish()
                outs.append((j, fm, pm, st))
            g.set_criteria(*np.array(CRITS[i % len(CRITS)], np.float32))
            fm, pm = _bufs(g)
            g.grow_submit(fm, pm)
            pending[k] = (i, fm, pm)
        for k in range(2):
            j, fm, pm = pending[k]
            outs.append((j, fm, pm, gs[k].grow_finish()))
        assert len(outs) == 3 * len(CRITS)
        for j, fm, pm, st in outs:
            ofm, opm, ost = want[j % len(CRITS)]
            hf, hp = _host(fm, pm)
            assert np.array_equal(hf, ofm), j
            assert np.array_equal(hp, opm), j
            assert st["coupled_steps"] == coupled[j % len(CRITS)], j  # this grow's statistics
    finally:
        for g in gs:
            g.close()


def test_first_chunk_too_short_and_round_cap():
    from paper_1903_12294_amd import MF4DError, _lib
    _need_gpu()
    inst = synth.make_config(1, attr_mode="noise")
    ofm, opm, ost = oracle_grow(inst["field"], inst["xyz"], inst["attr"], inst["crit"], inst["seeds"])
    g = _grower(inst, tile_t=4)
    ref = _grower(inst, tile_t=4)
    try:
        # a fresh context queues 4 rounds first; this grow needs more
        fm, pm = _bufs(g)
        g.grow_submit(fm, pm)
        st = g.grow_finish()
        assert st["rounds"] > 4, st["rounds"]
        hf, hp = _host(fm, pm)
        assert np.array_equal(hf, ofm) and np.array_equal(hp, opm)
        full = g.stats()
        assert full["members_field"] == ost["members_field"]
        assert full["members_particle"] == ost["members_particle"]
        for cap in (1, 3):
            g.set_max_rounds(cap)
            ref.set_max_rounds(cap)
            fm, pm = _bufs(g)
            g.grow_submit(fm, pm)
            with pytest.raises(MF4DError) as e:
                g.grow_finish()
            assert e.value.code == _lib.MF4D_ERR_NOT_CONVERGED
            with pytest.raises(MF4DError):
                ref.grow()
            hf, hp = _host(fm, pm)
            assert np.array_equal(hf, ref.read_field_mask()), cap
            assert np.array_equal(hp, ref.read_particle_mask()), cap
        g.set_max_rounds(0)
        g.grow_resume()
        assert np.array_equal(g.read_field_mask(), ofm)
        assert np.array_equal(g.read_particle_mask(), opm)
    finally:
        g.close()
        ref.close()


def test_call_in_between_completes_the_grow_and_state_errors():
    from paper_1903_12294_amd import MF4DError, _lib
    _need_gpu()
    inst = synth.make_config(1, attr_mode="noise")
    ofm, opm, ost = oracle_grow(inst["field"], inst["xyz"], inst["attr"], inst["crit"], inst["seeds"])
    g = _grower(inst, tile_t=8)
    try:
        with pytest.raises(MF4DError) as e:
            g.grow_finish()
        assert e.value.code == _lib.MF4D_ERR_STATE
        fm, pm = _bufs(g)
        g.grow_submit(fm, pm)
        with pytest.raises(MF4DError) as e:
            g.grow_submit(fm, pm)
        assert e.value.code == _lib.MF4D_ERR_STATE
        # reading the labels completes the submitted grow first
        assert np.array_equal(g.read_field_mask(), ofm)
        assert np.array_equal(g.read_particle_mask(), opm)
        st = g.grow_finish()  # its kept result
        assert st["rounds"] > 0
        hf, hp = _host(fm, pm)
        assert np.array_equal(hf, ofm) and np.array_equal(hp, opm)
        # new criteria set before finishing apply to the next grow only
        fm, pm = _bufs(g)
        g.grow_submit(fm, pm)
        crit2 = np.array(CRITS[1], np.float32)
        g.set_criteria(*crit2)
        g.grow_finish()
        hf, hp = _host(fm, pm)
        assert np.array_equal(hf, ofm) and np.array_equal(hp, opm)
        ofm2, opm2, _ = oracle_grow(inst["field"], inst["xyz"], inst["attr"], crit2, inst["seeds"])
        fm, pm = _bufs(g)
        g.grow_submit(fm, pm)
        g.grow_finish()
        hf, hp = _host(fm, pm)
        assert np.array_equal(hf, ofm2) and np.array_equal(hp, opm2)
    finally:
        g.close()


@pytest.mark.parametrize("variant", ["heuristic", "persistent", "timing", "async"])
def test_configurations_that_grow_on_submit(variant):
    _need_gpu()
    inst = synth.make_config(1, attr_mode="noise")
    ofm, opm, _ = oracle_grow(inst["field"], inst["xyz"], inst["attr"], inst["crit"], inst["seeds"])
    g = _grower(inst, tile_t=8, schedule="persistent" if variant == "persistent" else "launch")
    try:
        if variant == "heuristic":
            g.set_scheduler("heuristic")
        elif variant == "timing":
            g.set_phase_timing(True)
        elif variant == "async":
            g.set_read_async(True)
            g.grow_read(*_bufs(g))  # leaves read-outs deferred
        fm, pm = _bufs(g)
        g.grow_submit(fm, pm)
        st = g.grow_finish()
        assert st["rounds"] > 0
        hf, hp = _host(fm, pm)
        assert np.array_equal(hf, ofm) and np.array_equal(hp, opm)
    finally:
        g.close()
