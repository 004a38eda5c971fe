"""GPU tests of the brick-activity predictor: its forward pass and gradients
against the fp64 reference (oracle/nn_ref.py), its training, and the grower
staying bit-exact whatever the predictor says."""
import numpy as np
import pytest

from oracle import nn_ref, oracle_grow
from paper_1903_12294_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _bf16_round(a):
    return torch.from_numpy(np.asarray(a, np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


# A kernel's pre-activation carries the rounding of fp32 accumulation over at
# most 43 terms (7 or 14 matrix instructions of 32 products, three operand
# pieces each): at most 43 * 2^-24 = 2.6e-6 of the sum of the terms'
# magnitudes.  A ReLU decision on a pre-activation closer to zero than that
# could go either way, so the inputs are chosen (seeded, on the CPU, in fp64)
# with every hidden pre-activation further from zero than 3e-6 of its
# magnitude sum; then both sides take every ReLU decision alike and the
# gradients are compared element by element.
RELU_MARGIN = 3e-6


def _make_case(shape, seed):
    from paper_1903_12294_amd.learned import init_params, split_params
    rng = np.random.default_rng(seed)
    flat = (init_params(seed) + 0.02 * rng.normal(size=10833)).astype(np.float32)
    parts = split_params(flat)
    ref_params = [(_bf16_round(p) if i % 2 == 0 else np.asarray(p, np.float64)) for i, p in enumerate(parts)]
    N, D, H, W = shape
    x8 = rng.normal(size=(N, D, H, W, 8)).astype(np.float32)
    y = (rng.random(shape) < 0.3).astype(np.uint8)
    return flat, ref_params, x8, y


def _relu_margin(ref_params, x):
    """Smallest |z| / sum |terms| over the hidden pre-activations (fp64)."""
    w1, b1, w2, b2, _, _ = ref_params
    z1 = nn_ref.conv3d(x, w1, b1)
    s1 = nn_ref.conv3d(np.abs(x), np.abs(w1), np.abs(b1))
    a1 = np.maximum(z1, 0)
    z2 = nn_ref.conv3d(a1, w2, b2)
    s2 = nn_ref.conv3d(a1, np.abs(w2), np.abs(b2))
    return min(float((np.abs(z1) / s1).min()), float((np.abs(z2) / s2).min()))


def _well_posed_case(shape):
    for seed in range(200):
        flat, ref_params, x8, y = _make_case(shape, seed)
        x_ref = _bf16_round(x8)
        if _relu_margin(ref_params, x_ref) > RELU_MARGIN:
            return flat, ref_params, x8, x_ref, y
    raise AssertionError(f"no seed below 200 gives a ReLU margin above {RELU_MARGIN} at {shape}")


@pytest.mark.parametrize("shape", [(4, 8, 8, 8), (4, 9, 10, 19), (5, 8, 12, 8), (6, 8, 8, 16)])
def test_forward_and_gradients_match_fp64_reference(shape):
    """Logits (the inference path: bf16 activations) within 2e-2 of the
    logit scale; loss, every weight and bias gradient and the input gradient
    (the training path: fp32 activations and layer gradients) element by
    element within 2e-2 of the pure fp64 reference (oracle/nn_ref.py) plus
    1e-4 of the tensor's largest magnitude, on grids of at least 8 x 8 x 8 x 4
    brick-steps.  The reference keeps every intermediate in fp64; weights and
    inputs are the bf16 values both sides use."""
    from paper_1903_12294_amd.learned import Net, join_params
    _need_gpu()
    flat, ref_params, x8, x_ref, y = _well_posed_case(shape)
    print(f"[grad] {shape}", flush=True)
    x = np.zeros(shape + (16,), np.float32)
    x[..., :8] = x8
    xt = torch.from_numpy(x).to(torch.bfloat16).to("cuda:0").contiguous()
    yt = torch.from_numpy(y).to("cuda:0")
    net = Net(0)
    try:
        net.set_params(flat)
        assert np.array_equal(net.get_params(), flat)
        logits = net.forward(xt).cpu().numpy().astype(np.float64)
        g, dx, loss = net.backward(xt, yt, 2.5)
        g = g.cpu().numpy().astype(np.float64)
        dx = dx.cpu().numpy().astype(np.float64)
    finally:
        net.close()
    z, cache = nn_ref.forward(ref_params, x_ref)
    loss_ref, dz = nn_ref.bce_loss(z, y, 2.5)
    grads_ref = nn_ref.backward(ref_params, cache, dz)
    # the input gradient: the first layer's input-gradient convolution of the
    # first layer's output gradient
    xr, z1, a1, z2, a2 = cache
    w1, _, w2, _, w3, _ = ref_params
    da2, _, _ = nn_ref.conv3d_backward(a2, w3, dz[..., None])
    da1, _, _ = nn_ref.conv3d_backward(a1, w2, da2 * (z2 > 0))
    dx_ref, _, _ = nn_ref.conv3d_backward(xr, w1, da1 * (z1 > 0))
    assert np.abs(logits - z).max() < 2e-2 * (np.abs(z).max() + 1e-6)
    assert abs(loss - loss_ref) < 1e-4 * abs(loss_ref), (loss, loss_ref)
    got = [gg for gg in _split_flat(g)] + [dx[..., :8]]
    want = [np.asarray(r, np.float64) for r in grads_ref] + [dx_ref]
    names = ["dW1", "db1", "dW2", "db2", "dW3", "db3", "dX"]
    for name, a, b in zip(names, got, want):
        a = a.reshape(b.shape)
        tol = 2e-2 * np.abs(b) + 1e-4 * np.abs(b).max()
        bad = np.abs(a - b) > tol
        assert not bad.any(), (name, int(bad.sum()), float((np.abs(a - b) / (tol + 1e-300)).max()))
    assert not dx[..., 8:].any()


def _split_flat(g):
    from paper_1903_12294_amd.learned import split_params
    return [np.asarray(p, np.float64) for p in split_params(g)]


def test_training_reduces_loss():
    from paper_1903_12294_amd.learned import Net, init_params, make_dataset, train
    _need_gpu()
    data = make_dataset([11, 12], config=1)
    net = Net(0)
    try:
        net.set_params(init_params(3))
        hist = train(net, data, epochs=40, lr=3e-3)
    finally:
        net.close()
    assert hist[-1] < 0.7 * hist[0], hist


@pytest.mark.parametrize("variant", ["field", "noise"])
def test_learned_schedule_is_exact(variant):
    from paper_1903_12294_amd import Grower
    from paper_1903_12294_amd.learned import Net, init_params, set_predictor
    _need_gpu()
    inst = synth.make_config(2, attr_mode=variant)
    ofm, opm, _ = oracle_grow(inst["field"], inst["xyz"], inst["attr"], inst["crit"], inst["seeds"])
    net = Net(0)
    g = Grower(device=0)
    try:
        g.load_field(inst["field"])
        g.load_particles(inst["xyz"], inst["attr"])
        g.set_criteria(*inst["crit"])
        g.set_seeds(inst["seeds"])
        nan_params = np.full(10833, np.nan, np.float32)
        for params, thr in [(init_params(1), 0.0), (init_params(2), -np.inf),
                            (init_params(2), np.inf), (nan_params, 0.0)]:
            net.set_params(params)
            set_predictor(g, net, thr)
            for schedule in ("persistent", "launch"):
                g.set_schedule(schedule)
                g.grow()
                assert np.array_equal(g.read_field_mask(), ofm), (thr, schedule)
                assert np.array_equal(g.read_particle_mask(), opm), (thr, schedule)
        set_predictor(g, None)
        g.grow()
        assert np.array_equal(g.read_field_mask(), ofm)
    finally:
        g.close()
        net.close()


def test_labels_are_members_per_brick():
    from paper_1903_12294_amd import Grower
    from paper_1903_12294_amd.learned import labels
    from tests import golden_io
    _need_gpu()
    inst = synth.make_config(1)
    g = Grower(device=0)
    try:
        g.load_field(inst["field"])
        g.load_particles(inst["xyz"], inst["attr"])
        g.set_criteria(*inst["crit"])
        g.set_seeds(inst["seeds"])
        g.grow()
        y = labels(g).cpu().numpy()
        Mf = golden_io.unpack_field(g.read_field_mask(), inst["field"].shape)
    finally:
        g.close()
    T, Z, Y, X = Mf.shape
    exp = Mf.reshape(T, Z // 8, 8, Y // 8, 8, X // 8, 8).any(axis=(2, 4, 6))
    assert np.array_equal(y.astype(bool), exp)


def test_trained_predictor_reads_fewer_tiles_and_stays_exact():
    """What the trained network gains over the grower without it, on a
    held-out variant (data seed 2000, not among the training seeds): fewer
    field tiles read (up front plus deferred), identical masks."""
    import json
    import os
    from paper_1903_12294_amd import Grower
    from paper_1903_12294_amd.learned import Net, init_params, set_predictor
    _need_gpu()
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    path = os.path.join(root, "paper_1903_12294_amd", "predictor.npy")
    if not os.path.exists(path):
        pytest.skip("no trained predictor weights in the tree")
    meta = json.load(open(os.path.splitext(path)[0] + ".json"))
    c = synth.CONFIGS[2]
    inst = synth.make_instance(c["X"], c["Y"], c["Z"], c["T"], c["P"], n_blobs=c["n_blobs"],
                               seed=2000, n_seeds=c["n_seeds"], tau_f=c["tau"], tau_p=c["tau"],
                               crossing=c["crossing"])
    ofm, opm, _ = oracle_grow(inst["field"], inst["xyz"], inst["attr"], inst["crit"], inst["seeds"])
    net = Net(0)
    g = Grower(device=0)
    try:
        g.load_field(inst["field"])
        g.load_particles(inst["xyz"], inst["attr"])
        g.set_criteria(*inst["crit"])
        g.set_seeds(inst["seeds"])
        g.set_admit_mode("tiles")
        base = g.grow()
        assert np.array_equal(g.read_field_mask(), ofm)
        res = {}
        for name, params, thr in [("trained", np.load(path), float(meta["logit_threshold"])),
                                  ("untrained", init_params(0), 0.0)]:
            net.set_params(params)
            set_predictor(g, net, thr)
            st = g.grow()
            assert np.array_equal(g.read_field_mask(), ofm), name
            assert np.array_equal(g.read_particle_mask(), opm), name
            res[name] = st
        set_predictor(g, None)
    finally:
        g.close()
        net.close()
    tr = res["trained"]
    reads = tr["tiles_tested"] + tr["tiles_deferred_read"]
    print(f"tiles read: without predictor {base['tiles_tested']}, trained {tr['tiles_tested']} up front "
          f"+ {tr['tiles_deferred_read']} deferred, untrained {res['untrained']['tiles_tested']} + "
          f"{res['untrained']['tiles_deferred_read']}")
    assert tr["tiles_tested"] < base["tiles_tested"]
    assert reads < base["tiles_tested"]


@pytest.mark.parametrize("variant", ["field", "noise"])
def test_score_ordered_schedulers_are_exact(variant):
    """The score-ordered schedulers (priority pass over the candidate tiles in
    descending score, plain rounds, a verification round that sweeps every
    tile holding an admissible voxel-step and pulls every coupled step) give
    the oracle's masks under both round schedules, with the heuristic score,
    an untrained and a NaN-weighted network, and report the verification
    round (which changes nothing: exactly one verification round)."""
    from paper_1903_12294_amd import Grower
    from paper_1903_12294_amd.learned import init_params
    _need_gpu()
    inst = synth.make_config(2, attr_mode=variant)
    ofm, opm, _ = oracle_grow(inst["field"], inst["xyz"], inst["attr"], inst["crit"], inst["seeds"])
    g = Grower(device=0)
    try:
        g.load_field(inst["field"])
        g.load_particles(inst["xyz"], inst["attr"])
        g.set_criteria(*inst["crit"])
        g.set_seeds(inst["seeds"])
        g.set_scheduler("plain")
        base = g.grow()
        assert base["verify_rounds"] == 0 and base["priority_visits"] == 0
        cases = [("heuristic", None, None), ("learned", init_params(4), 0.0),
                 ("learned", init_params(5), -np.inf), ("learned", np.full(10833, np.nan, np.float32), 0.0)]
        for kind, params, thr in cases:
            if params is None:
                g.set_scheduler(kind)
            else:
                g.set_scheduler(kind, params, thr)
            for schedule in ("persistent", "launch"):
                print(f"[ordered] {variant} {kind} thr={thr} {schedule}", flush=True)
                g.set_schedule(schedule)
                st = g.grow()
                assert np.array_equal(g.read_field_mask(), ofm), (kind, thr, schedule)
                assert np.array_equal(g.read_particle_mask(), opm), (kind, thr, schedule)
                assert st["verify_rounds"] == 1, st
                if kind == "heuristic" or thr == -np.inf:
                    assert st["priority_visits"] > 0
        g.set_scheduler("plain")
        st = g.grow()
        assert st["verify_rounds"] == 0
        assert np.array_equal(g.read_field_mask(), ofm)
    finally:
        g.close()
