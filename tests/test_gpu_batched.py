"""GPU parity of the batched grower: every query plane equals the oracle's
single-query grow with that query's criteria and seeds."""
import numpy as np
import pytest

from oracle import oracle_grow_queries
from paper_1903_12294_amd import synth
from tests import golden_io

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _planes_to_masks(fplanes, pplanes, shape, T, P, q):
    fbits = ((fplanes[:, q >> 5] >> np.uint32(q & 31)) & 1).astype(bool).reshape(shape)
    pbits = ((pplanes[:, :, q >> 5] >> np.uint32(q & 31)) & 1).astype(np.uint8).reshape(T, P)
    return fbits, pbits


def _run(inst, crit, qseeds, device_out=True, tile=None):
    from paper_1903_12294_amd import Grower
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    g = Grower(device=0)
    try:
        if tile:
            g.set_batched_tile(*tile)
        g.load_field(inst["field"])
        if inst["xyz"].shape[1] > 0:
            g.load_particles(inst["xyz"], inst["attr"])
        g.set_queries(crit, qseeds)
        X, Y, Z = inst["dims"] if "dims" in inst else inst["field"].shape[::-1][:3]
        T = inst["field"].shape[0]
        P = inst["xyz"].shape[1]
        V = inst["field"].size
        if device_out:
            fpl = torch.zeros((V, 8), dtype=torch.int32, device="cuda:0")
            ppl = torch.zeros((T, max(P, 1), 8), dtype=torch.int32, device="cuda:0") if P else None
            _, _, st = g.grow_batched(fpl, ppl)
            fp = fpl.cpu().numpy().view(np.uint32)
            pp = ppl.cpu().numpy().view(np.uint32) if P else np.zeros((T, 0, 8), np.uint32)
        else:
            fp, pp, st = g.grow_batched()
    finally:
        g.close()
    return fp, pp, st


def _check(inst, crit, qseeds, queries=None, device_out=True, tile=None):
    fp, pp, st = _run(inst, crit, qseeds, device_out, tile)
    T, P = inst["field"].shape[0], inst["xyz"].shape[1]
    Q = len(crit)
    res = oracle_grow_queries(inst["field"], inst["xyz"], inst["attr"], crit, qseeds,
                              queries=queries)
    for q, (ofm, opm, ost) in res.items():
        f, p = _planes_to_masks(fp, pp, inst["field"].shape, T, P, q)
        of = golden_io.unpack_field(ofm, inst["field"].shape)
        assert np.array_equal(f, of), f"query {q}: field plane differs ({f.sum()} vs {of.sum()})"
        assert np.array_equal(p, opm), f"query {q}: particle plane differs"
    # planes past Q stay empty
    for q in range(Q, min(256, Q + 40)):
        f, p = _planes_to_masks(fp, pp, inst["field"].shape, T, P, q)
        assert not f.any() and not p.any()
    return st


@pytest.mark.parametrize("tile", [None, (4, 4, 4, 8)])
@pytest.mark.parametrize("seed", range(6))
def test_random_small_queries(seed, tile):
    from tests.test_oracle_pins import _random_instance
    rng = np.random.default_rng(500 + seed)
    X, Y, Z = (int(v) for v in rng.integers(3, 40, 3))
    T = int(rng.integers(1, 12))
    P = int(rng.integers(0, 200))
    inst = _random_instance(rng, X, Y, Z, T, P, 1)
    Q = int(rng.integers(1, 80))
    vals = np.array([0.25, 0.5, 0.75, 1.0, np.inf, -np.inf], np.float32)
    crit = np.stack([vals[rng.integers(0, 4, Q)], vals[rng.integers(2, 5, Q)],
                     vals[rng.integers(0, 4, Q)], vals[rng.integers(3, 5, Q)]], 1).astype(np.float32)
    n = int(rng.integers(Q, 3 * Q + 1))
    qseeds = np.stack([rng.integers(0, X, n), rng.integers(0, Y, n), rng.integers(0, Z, n),
                       rng.integers(0, T, n), rng.integers(0, Q, n)], 1).astype(np.int32)
    print(f"[batched] random{seed} {X}x{Y}x{Z}x{T} P={P} Q={Q} tile {tile}", flush=True)
    _check(inst, crit, qseeds, device_out=(seed % 2 == 0), tile=tile)


@pytest.mark.parametrize("tile", [None, (4, 4, 4, 8)])
def test_field_only_queries(tile):
    """No particles: rounds of sweeps alone, each round's list built anew."""
    from tests.test_oracle_pins import _random_instance
    rng = np.random.default_rng(77)
    inst = _random_instance(rng, 24, 20, 17, 9, 0, 1)
    Q = 40
    vals = np.array([0.25, 0.5, 0.75, 1.0, np.inf], np.float32)
    crit = np.stack([vals[rng.integers(0, 3, Q)], vals[rng.integers(2, 5, Q)],
                     np.full(Q, -np.inf, np.float32), np.full(Q, np.inf, np.float32)], 1).astype(np.float32)
    qseeds = np.stack([rng.integers(0, 24, 3 * Q), rng.integers(0, 20, 3 * Q), rng.integers(0, 17, 3 * Q),
                       rng.integers(0, 9, 3 * Q), rng.integers(0, Q, 3 * Q)], 1).astype(np.int32)
    st = _check(inst, crit, qseeds, tile=tile)
    assert st["rounds"] > 1


@pytest.mark.parametrize("tile", [None, (4, 4, 4, 8)])
def test_config1_256_queries(tile):
    inst = synth.make_config(1)
    crit, qseeds = synth.make_queries(inst, Q=256)
    _check(inst, crit, qseeds, tile=tile)


def test_config1_noise_attr_256_queries():
    inst = synth.make_config(1, attr_mode="noise")
    crit, qseeds = synth.make_queries(inst, Q=256, seed=9)
    _check(inst, crit, qseeds)


def test_config4_sampled_queries():
    """Config 4: config 2's data, 256 queries; 24 planes checked against the oracle."""
    inst = synth.make_config(2)
    crit, qseeds = synth.make_queries(inst, Q=256)
    qs = list(np.random.default_rng(3).choice(256, 24, replace=False))
    st = _check(inst, crit, qseeds, queries=qs)
    print(f"[batched] cfg4 rounds {st['rounds']} visits {st['tile_visits']}", flush=True)
