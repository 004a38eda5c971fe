"""GPU parity at the full workload sizes, element by element against the
oracle:
  256^3 x 64 field with 4,194,304 particles x 64 steps (64 crossing blobs, 32
  seeds, thresholds 0.25 / 0.25) under both round schedules and both
  admissibility modes, at the tile depth and schedule the benchmark times and
  at the default tile depth;
  the same data with the trained activity predictor (learned scheduler);
  128^3 x 32 with 262,144 particles and 256 concurrent queries (1-16 seeds
  each, thresholds from U[0.15, 0.6]): every one of the 256 planes against
  its own oracle grow, run on all host cores.
Masks are compared on the device as packed words."""
import json
import os

import numpy as np
import pytest

from oracle import oracle_grow, oracle_grow_queries
from paper_1903_12294_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PREDICTOR = os.path.join(ROOT, "paper_1903_12294_amd", "predictor.npy")


@pytest.fixture(scope="module")
def scale():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("[fullsize] generating the 256^3 x 64 workload", flush=True)
    inst = synth.make_config(3)
    print("[fullsize] oracle grow", flush=True)
    ofm, opm, ost = oracle_grow(inst["field"], inst["xyz"], inst["attr"], inst["crit"], inst["seeds"])
    dev = torch.device("cuda:0")
    yield {"inst": inst, "ofm": torch.from_numpy(ofm.view(np.int32)).to(dev),
           "opm": torch.from_numpy(opm).to(dev), "ost": ost,
           "field": torch.from_numpy(inst["field"]).to(dev),
           "xyz": torch.from_numpy(inst["xyz"]).to(dev), "attr": torch.from_numpy(inst["attr"]).to(dev)}
    torch.cuda.empty_cache()


def _grow_scale(scale, tile_t, schedule, admit, scheduler=None):
    from paper_1903_12294_amd import Grower
    inst = scale["inst"]
    T, P = inst["T"], inst["P"]
    V = inst["field"].size
    g = Grower(device=0, tile_t=tile_t, schedule=schedule, admit=admit)
    try:
        g.load_field(scale["field"])
        g.load_particles(scale["xyz"], scale["attr"])
        g.set_criteria(*inst["crit"])
        g.set_seeds(inst["seeds"])
        if scheduler is not None:
            g.set_scheduler(*scheduler)
        fm = torch.empty((V + 31) // 32, dtype=torch.int32, device="cuda:0")
        pm = torch.empty((T, P), dtype=torch.uint8, device="cuda:0")
        st = g.grow()
        g.read_field_mask(fm)
        g.read_particle_mask(pm)
        torch.cuda.synchronize()
    finally:
        g.close()
    return fm, pm, st


@pytest.mark.parametrize("tile_t,schedule,admit", [
    (16, "launch", "tiles"), (16, "persistent", "tiles"), (8, "persistent", "tiles"),
    (8, "launch", "all"),
])
def test_config3_masks_equal_oracle(scale, tile_t, schedule, admit):
    print(f"[fullsize] 256^3x64 tile_t={tile_t} {schedule} {admit}", flush=True)
    fm, pm, st = _grow_scale(scale, tile_t, schedule, admit)
    assert torch.equal(fm, scale["ofm"])
    assert torch.equal(pm, scale["opm"])
    assert st["rounds"] > 0


def test_config5_learned_masks_equal_oracle(scale):
    if not os.path.exists(PREDICTOR):
        pytest.skip("no trained predictor weights in the tree")
    meta = json.load(open(os.path.splitext(PREDICTOR)[0] + ".json"))
    params = np.load(PREDICTOR)
    for schedule in ("launch", "persistent"):
        print(f"[fullsize] 256^3x64 learned {schedule}", flush=True)
        fm, pm, st = _grow_scale(scale, 16, schedule, "tiles",
                                 scheduler=("learned", params, float(meta["logit_threshold"])))
        assert torch.equal(fm, scale["ofm"]), schedule
        assert torch.equal(pm, scale["opm"]), schedule
        assert st["verify_rounds"] == 1
    print("[fullsize] 256^3x64 heuristic priority", flush=True)
    fm, pm, st = _grow_scale(scale, 16, "launch", "tiles", scheduler=("heuristic",))
    assert torch.equal(fm, scale["ofm"]) and torch.equal(pm, scale["opm"])
    assert st["verify_rounds"] == 1 and st["priority_visits"] > 0


def _pack_plane(bits_u8):
    """Little-endian packing of a flat 0/1 byte tensor into int32 words."""
    n = bits_u8.numel()
    pad = (-n) % 32
    b = torch.nn.functional.pad(bits_u8.to(torch.int64), (0, pad)).view(-1, 32)
    w = (b << torch.arange(32, device=b.device, dtype=torch.int64)).sum(1)
    return w.to(torch.int64)


def test_config4_every_plane_equals_oracle():
    from paper_1903_12294_amd import Grower
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    inst = synth.make_config(2)
    crit, qseeds = synth.make_queries(inst, Q=256, seed=4)
    T, P = inst["T"], inst["P"]
    V = inst["field"].size
    dev = torch.device("cuda:0")
    # the default tile and the 4 x 4 x 4 x 8 tile (its sweep takes the
    # in-wave cube route)
    runs = []
    g = Grower(device=0)
    try:
        g.load_field(inst["field"])
        g.load_particles(inst["xyz"], inst["attr"])
        g.set_queries(crit, qseeds)
        for shape in (None, (4, 4, 4, 8)):
            print(f"[fullsize] 128^3x32 x 256 queries: batched grow, tile {shape}", flush=True)
            if shape:
                g.set_batched_tile(*shape)
            fp = torch.empty((V, 8), dtype=torch.int32, device=dev)
            pp = torch.empty((T, P, 8), dtype=torch.int32, device=dev)
            _, _, st = g.grow_batched(fp, pp)
            torch.cuda.synchronize()
            runs.append((shape, fp, pp, st))
    finally:
        g.close()
    threads = min(16, os.cpu_count() or 1)
    print(f"[fullsize] 256 oracle grows on {threads} threads", flush=True)
    res = oracle_grow_queries(inst["field"], inst["xyz"], inst["attr"], crit, qseeds, threads=threads)
    assert sorted(res) == list(range(256))
    for shape, fp, pp, st in runs:
        for q in range(256):
            ofm, opm, _ = res[q]
            plane_f = ((fp[:, q >> 5] >> (q & 31)) & 1).to(torch.uint8)
            got_f = _pack_plane(plane_f)
            want_f = torch.from_numpy(ofm.astype(np.int64)).to(dev)
            assert torch.equal(got_f, want_f), f"tile {shape}, query {q}: field plane differs"
            plane_p = ((pp[..., q >> 5] >> (q & 31)) & 1).to(torch.uint8)
            assert torch.equal(plane_p, torch.from_numpy(opm).to(dev)), \
                f"tile {shape}, query {q}: particle plane differs"
        print(f"[fullsize] tile {shape}: all 256 planes equal; {st['rounds']} rounds", flush=True)
