"""GPU parity with particles stored at their own temporal rate (r particle
steps per field step, mf4d_load_particles_rate) and on planar 2D + t grids:
the grower (both schedules and trajectory modes), the batched grower, the
segment read-out, per-seed ids and the clustering against the oracle at the
same rate, bit for bit."""
import ctypes

import numpy as np
import pytest

from oracle import oracle_grow, oracle_grow_queries, oracle_seed_ids
from oracle import segments as oseg
from oracle import slic as oslic
from paper_1903_12294_amd import synth
from tests import golden_io

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _load(g, inst, rate):
    dev = torch.device("cuda:0")
    g.load_field(torch.from_numpy(np.ascontiguousarray(inst["field"])).to(dev))
    if inst["xyz"].shape[1] > 0:
        g.load_particles(torch.from_numpy(np.ascontiguousarray(inst["xyz"])).to(dev),
                         torch.from_numpy(np.ascontiguousarray(inst["attr"])).to(dev), rate=rate)


def _rate_instance(seed, X, Y, Z, T, P, r, Tp=None):
    from tests.test_oracle_pins import _random_instance
    rng = np.random.default_rng(seed)
    Tp = r * T if Tp is None else Tp
    parts = _random_instance(rng, X, Y, Z, Tp, P, 0)
    inst = _random_instance(rng, X, Y, Z, T, 0, 5)
    inst["xyz"], inst["attr"] = parts["xyz"], parts["attr"]
    return inst


def _assert_grow(inst, r, tag, schedule=None, mode="both", tile_t=None):
    from paper_1903_12294_amd import Grower
    _need_gpu()
    P = inst["xyz"].shape[1]
    print(f"[rate] {tag} field {inst['field'].shape} Tp={inst['xyz'].shape[0]} P={P} r={r} "
          f"{schedule} {mode} tile_t={tile_t}", flush=True)
    g = Grower(device=0, schedule=schedule, tile_t=tile_t)
    try:
        _load(g, inst, r)
        g.set_trajectory_mode(mode)
        g.set_criteria(*inst["crit"])
        g.set_seeds(np.asarray(inst["seeds"], np.int32).reshape(-1, 4))
        g.grow()
        fm = g.read_field_mask()
        pm = g.read_particle_mask()
        seg = g.read_particle_segments()
        st = g.stats()
    finally:
        g.close()
    ofm, opm, ost = oracle_grow(inst["field"], inst["xyz"], inst["attr"], inst["crit"], inst["seeds"],
                                forward_only=mode == "forward", rate=r)
    assert np.array_equal(fm, ofm), f"{tag}: field mask differs"
    assert np.array_equal(pm, opm), f"{tag}: particle mask differs ({int(pm.sum())} vs {int(opm.sum())})"
    assert np.array_equal(seg, oseg.mask_segments(opm)), f"{tag}: segments differ"
    assert st["members_particle"] == ost["members_particle"]
    return ost


@pytest.mark.parametrize("seed", range(12))
def test_random_rates(seed):
    rng = np.random.default_rng(5000 + seed)
    X, Y, Z = (int(v) for v in rng.integers(1, 40, 3))
    T = int(rng.integers(1, 10))
    r = int(rng.integers(2, 6))
    Tp = int(rng.integers(1, r * T + 1))
    P = int(rng.integers(1, 300))
    inst = _rate_instance(seed, X, Y, Z, T, P, r, Tp)
    _assert_grow(inst, r, f"random{seed}", schedule=["persistent", "launch"][seed % 2],
                 mode=["both", "forward"][(seed // 2) % 2], tile_t=[4, 8, 16][seed % 3])


@pytest.mark.parametrize("schedule", ["persistent", "launch"])
@pytest.mark.parametrize("mode", ["both", "forward"])
def test_long_trajectories_at_rate_4(schedule, mode):
    """130 particle steps over 33 field steps: three label words per particle."""
    inst = synth.make_instance(40, 24, 16, 33, 1500, n_blobs=4, seed=33, n_seeds=4, tau_f=0.3,
                               tau_p=0.15, attr_mode="noise", rate=4)
    inst["xyz"], inst["attr"] = inst["xyz"][:130], inst["attr"][:130]
    _assert_grow(inst, 4, "long Tp=130 r=4", schedule=schedule, mode=mode)


def test_one_field_step():
    inst = _rate_instance(77, 20, 10, 6, 1, 200, 5)
    _assert_grow(inst, 5, "T=1 Tp=5")


@pytest.mark.parametrize("mode", ["both", "forward"])
def test_planar_2d_plus_t_workload(mode):
    """A planar city-like grid (128 x 128 x 1, 12 field steps) with 3,000
    particles at 4 steps per field step."""
    inst = synth.make_instance(128, 128, 1, 12, 3000, n_blobs=8, seed=7, n_seeds=4, tau_f=0.3,
                               tau_p=0.3, rate=4)
    ost = _assert_grow(inst, 4, "planar 128^2x1x12 r=4", mode=mode)
    assert ost["members_particle"] > 0


def test_rate_one_matches_plain_load():
    from paper_1903_12294_amd import Grower
    _need_gpu()
    inst = synth.make_config(1)
    outs = []
    for use_rate in (False, True):
        g = Grower(device=0)
        try:
            g.load_field(inst["field"])
            if use_rate:
                g._check(g.lib.mf4d_load_particles_rate(
                    g.ctx, inst["xyz"].ctypes.data_as(ctypes.c_void_p),
                    inst["attr"].ctypes.data_as(ctypes.c_void_p), inst["P"], inst["T"], 1, 0))
                g.P, g.Tp = inst["P"], inst["T"]
            else:
                g.load_particles(inst["xyz"], inst["attr"])
            g.set_criteria(*inst["crit"])
            g.set_seeds(inst["seeds"])
            g.grow()
            outs.append((g.read_field_mask(), g.read_particle_mask()))
        finally:
            g.close()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_rate_errors():
    from paper_1903_12294_amd import Grower
    from paper_1903_12294_amd._lib import MF4DError
    _need_gpu()
    inst = _rate_instance(3, 8, 8, 8, 3, 16, 2)
    g = Grower(device=0)
    try:
        g.load_field(inst["field"])
        with pytest.raises(MF4DError):
            g.load_particles(inst["xyz"], inst["attr"], rate=1)  # 6 steps over 3 field steps at rate 1
        with pytest.raises(MF4DError):
            g.load_particles(inst["xyz"][:6], inst["attr"][:6], rate=0)
        xyz7 = np.concatenate([inst["xyz"], inst["xyz"][:1]])
        attr7 = np.concatenate([inst["attr"], inst["attr"][:1]])
        with pytest.raises(MF4DError):
            g.load_particles(xyz7, attr7, rate=2)  # 7 > 2 * 3
        g.load_particles(inst["xyz"], inst["attr"], rate=2)
    finally:
        g.close()


@pytest.mark.parametrize("seed", range(2))
def test_batched_at_rate(seed):
    from paper_1903_12294_amd import Grower
    from tests.test_gpu_batched import _planes_to_masks
    _need_gpu()
    rng = np.random.default_rng(800 + seed)
    X, Y, Z = (int(v) for v in rng.integers(3, 30, 3))
    T, r = int(rng.integers(2, 8)), int(rng.integers(2, 5))
    Tp = int(rng.integers(1, r * T + 1))
    P = int(rng.integers(20, 200))
    inst = _rate_instance(seed + 40, X, Y, Z, T, P, r, Tp)
    Q = int(rng.integers(1, 40))
    vals = np.array([0.25, 0.5, 0.75, 1.0, np.inf, -np.inf], np.float32)
    crit = np.stack([vals[rng.integers(0, 4, Q)], vals[rng.integers(2, 5, Q)],
                     vals[rng.integers(0, 4, Q)], vals[rng.integers(3, 5, Q)]], 1).astype(np.float32)
    n = int(rng.integers(Q, 3 * Q + 1))
    qseeds = np.stack([rng.integers(0, X, n), rng.integers(0, Y, n), rng.integers(0, Z, n),
                       rng.integers(0, T, n), rng.integers(0, Q, n)], 1).astype(np.int32)
    print(f"[rate] batched{seed} {X}x{Y}x{Z}x{T} Tp={Tp} r={r} P={P} Q={Q}", flush=True)
    g = Grower(device=0)
    try:
        g.load_field(inst["field"])
        g.load_particles(inst["xyz"], inst["attr"], rate=r)
        g.set_queries(crit, qseeds)
        fp, pp, _ = g.grow_batched()
    finally:
        g.close()
    res = oracle_grow_queries(inst["field"], inst["xyz"], inst["attr"], crit, qseeds, rate=r)
    for q, (ofm, opm, _) in res.items():
        f, p = _planes_to_masks(fp, pp, inst["field"].shape, Tp, P, q)
        assert np.array_equal(f, golden_io.unpack_field(ofm, inst["field"].shape)), f"query {q}: field plane"
        assert np.array_equal(p, opm), f"query {q}: particle plane"


def test_seed_ids_at_rate():
    from paper_1903_12294_amd import Grower
    _need_gpu()
    inst = synth.make_instance(48, 40, 1, 10, 800, n_blobs=6, seed=11, n_seeds=6, tau_f=0.45,
                               tau_p=0.3, rate=3)
    g = Grower(device=0)
    try:
        _load(g, inst, 3)
        g.set_criteria(*inst["crit"])
        g.set_seeds(inst["seeds"])
        fid, pid, _ = g.grow_seed_ids()
    finally:
        g.close()
    ofid, opid = oracle_seed_ids(inst["field"], inst["xyz"], inst["attr"], inst["crit"], inst["seeds"], rate=3)
    assert np.array_equal(fid, ofid) and np.array_equal(pid, opid)


@pytest.mark.parametrize("r,k", [(2, (4, 2, 2, 2)), (3, (3, 2, 1, 3))])
def test_clustering_at_rate(r, k):
    from paper_1903_12294_amd import Grower
    from tests.test_gpu_slic import _case
    _need_gpu()
    T, Z, Y, X, P = 6, 8, 8, 16, 90
    field, _, _ = _case(60 + r, T, Z, Y, X, 0)
    _, xyz, attr = _case(61 + r, T * r - 1, Z, Y, X, P, spread=1.2, nan=True)
    w, cf, eps, it, eps_m = (1.0, 2.0, 2.0), 0.5, 1e-4, 6, 0.05
    print(f"[rate] clustering r={r} k={k}", flush=True)
    g = Grower(device=0)
    try:
        _load(g, dict(field=field, xyz=xyz, attr=attr), r)
        g.slic_set_params(k, w[0], w[1], w[2], cf, eps, it)
        n_it = g.slic_run()
        fl, pl = g.slic_read_labels()
        cen, cnt = g.slic_read_centres()
        g.slic_merge(eps_m)
        feat, fst = g.slic_read_features()
        seg = g.slic_read_segments()
    finally:
        g.close()
    ofl, opl, ocen, ocnt, oit = oslic.slic(field, xyz, attr, k, w, cf, eps, it, rate=r)
    assert n_it == oit
    assert np.array_equal(fl, ofl) and np.array_equal(pl, opl)
    assert np.array_equal(cnt, ocnt) and cen.tobytes() == ocen.tobytes()
    ofeat = oslic.merge_centres(ocen, ocnt, eps_m)
    assert np.array_equal(feat, ofeat)
    ost = oslic.feature_stats(field, xyz, attr, ofl, opl, ofeat, rate=r)
    exact = [0, 1, 2, 3] + list(range(6, 14))
    assert fst[:, exact].tobytes() == ost[:, exact].tobytes()
    assert np.allclose(fst[:, 4:6], ost[:, 4:6], rtol=1e-9, atol=1e-12)
    assert np.array_equal(seg, oseg.feature_segments(oseg.point_features(opl, ofeat)))
