"""GPU: the predictor's inputs (per-brick field statistics and particle counts
at t and t - 1, centred on the field lower bound, bfloat16) against the plain
reference oracle/features.py, element by element, on ragged grids with NaN
samples, unbinned particles and particle rates."""
import numpy as np
import pytest

from oracle import features as of

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _case(seed, dims, T, P, rate, nan_frac):
    rng = np.random.default_rng(seed)
    X, Y, Z = dims
    field = rng.random((T, Z, Y, X)).astype(np.float32)
    field[rng.random(field.shape) < nan_frac] = np.nan
    if Z > 8 and Y > 8 and X > 8:
        field[:, :8, :8, :8] = np.nan  # a brick with no value at every step
    Tp = T * rate
    xyz = (rng.random((Tp, P, 3)) * np.array([X + 2, Y + 2, Z + 2]) - 1).astype(np.float32)
    xyz[rng.random((Tp, P)) < 0.05] = np.nan
    attr = rng.random((Tp, P)).astype(np.float32)
    return field, xyz, attr


def _compare(got, want, stats):
    """Channels 0, 1, 4, 5 (min, max) and 8..15 bit-exact; the counts'
    log1p within one bfloat16 step (log1pf); the means within the error of a
    float32 sum of up to 512 values, centred, plus one bfloat16 step."""
    assert got.shape == want.shape
    for ch in (0, 1, 4, 5):
        assert np.array_equal(got[..., ch], want[..., ch]), ch
    assert not got[..., 8:].any()
    for ch in (3, 7):
        d = np.abs(got[..., ch].astype(np.int64) - want[..., ch].astype(np.int64))
        assert d.max() <= 1, ch
    gv = (got.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    wv = (want.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    mag = np.maximum(np.abs(stats[..., 0]), np.abs(stats[..., 1]))
    prev = np.zeros_like(mag)
    prev[1:] = mag[:-1]
    for ch, m in ((2, mag), (6, prev)):
        tol = 2.0 ** -8 * np.abs(wv[..., ch]) + 1e-4 * m + 1e-30
        assert np.all(np.abs(gv[..., ch] - wv[..., ch]) <= tol), ch


@pytest.mark.parametrize("seed,dims,T,P,rate,f_lo", [
    (1, (37, 21, 13), 5, 300, 1, 0.3),
    (2, (24, 17, 9), 3, 500, 3, 0.25),
    (3, (8, 8, 8), 2, 0, 1, -np.inf),
    (4, (40, 30, 20), 4, 2000, 2, 0.5),
])
def test_features_match_oracle(seed, dims, T, P, rate, f_lo):
    from paper_1903_12294_amd import Grower
    from paper_1903_12294_amd.learned import brick_dims, features
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    field, xyz, attr = _case(seed, dims, T, P, rate, 0.1)
    print(f"features case seed={seed} dims={dims} T={T} P={P} rate={rate}", flush=True)
    g = Grower(device=0)
    try:
        g.load_field(field)
        if P:
            g.load_particles(xyz, attr, rate=rate)
        g.set_criteria(f_lo, np.inf, 0.2, np.inf)
        assert brick_dims(g) == of.brick_dims(*dims, T)
        got = features(g).view(torch.int16).cpu().numpy().view(np.uint16)
    finally:
        g.close()
    want = of.features(field, xyz if P else None, f_lo, rate=rate)
    _compare(got, want, of.brick_stats(field))
