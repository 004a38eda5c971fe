"""Pins of the fp64 predictor reference (oracle/nn_ref.py): against scipy's
n-d correlation, and against central finite differences."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import nn_ref


def test_conv3d_single_channel_is_ndimage_correlate():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 5, 6, 7, 1))
    w = rng.normal(size=(1, 1, 3, 3, 3))
    out = nn_ref.conv3d(x, w, np.array([0.25]))
    for n in range(2):
        exp = ndimage.correlate(x[n, ..., 0], w[0, 0], mode="constant", cval=0.0) + 0.25
        assert np.allclose(out[n, ..., 0], exp, atol=1e-12)


def test_conv3d_channels_sum_of_correlations():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(1, 4, 5, 3, 3))
    w = rng.normal(size=(2, 3, 3, 3, 3))
    out = nn_ref.conv3d(x, w, np.zeros(2))
    for co in range(2):
        exp = sum(ndimage.correlate(x[0, ..., ci], w[co, ci], mode="constant") for ci in range(3))
        assert np.allclose(out[0, ..., co], exp, atol=1e-12)


def _fd(f, arr, idx, h=1e-6):
    old = arr[idx]
    arr[idx] = old + h
    fp = f()
    arr[idx] = old - h
    fm = f()
    arr[idx] = old
    return (fp - fm) / (2 * h)


def test_conv3d_backward_finite_differences():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(2, 3, 4, 5, 3))
    w = rng.normal(size=(4, 3, 3, 3, 3))
    b = rng.normal(size=4)
    g = rng.normal(size=(2, 3, 4, 5, 4))
    f = lambda: float((nn_ref.conv3d(x, w, b) * g).sum())
    dx, dw, db = nn_ref.conv3d_backward(x, w, g)
    for idx in [(0, 0, 0, 0, 0), (1, 2, 3, 4, 2), (0, 1, 2, 2, 1)]:
        assert abs(_fd(f, x, idx) - dx[idx]) < 1e-6 * max(1, abs(dx[idx]))
    for idx in [(0, 0, 0, 0, 0), (3, 2, 2, 1, 0), (1, 1, 1, 1, 1)]:
        assert abs(_fd(f, w, idx) - dw[idx]) < 1e-6 * max(1, abs(dw[idx]))
    for i in range(4):
        assert abs(_fd(f, b, (i,)) - db[i]) < 1e-6 * max(1, abs(db[i]))


def test_network_gradient_finite_differences():
    rng = np.random.default_rng(3)
    params = nn_ref.init_params(rng, cin=8, hidden=16)
    params = [p + 0.05 * rng.normal(size=p.shape) for p in params]
    x = rng.normal(size=(2, 4, 3, 5, 8))
    y = (rng.random((2, 4, 3, 5)) < 0.3).astype(np.float64)

    def loss():
        z, _ = nn_ref.forward(params, x)
        return nn_ref.bce_loss(z, y, 3.0)[0]

    z, cache = nn_ref.forward(params, x)
    _, dz = nn_ref.bce_loss(z, y, 3.0)
    grads = nn_ref.backward(params, cache, dz)
    for pi, idx in [(0, (3, 2, 1, 0, 2)), (1, (5,)), (2, (7, 11, 2, 2, 0)), (3, (9,)),
                    (4, (0, 13, 1, 1, 1)), (5, (0,))]:
        fd = _fd(loss, params[pi], idx)
        assert abs(fd - grads[pi][idx]) < 1e-6 * max(1e-3, abs(fd)), (pi, idx, fd, grads[pi][idx])


def test_bce_gradient_and_value():
    z = np.array([-3.0, -0.2, 0.0, 0.7, 4.0])
    y = np.array([0.0, 1.0, 1.0, 0.0, 1.0])
    loss, dz = nn_ref.bce_loss(z, y, 2.0)
    s = 1 / (1 + np.exp(-z))
    exp = np.mean(-(2.0 * y * np.log(s) + (1 - y) * np.log(1 - s)))
    assert abs(loss - exp) < 1e-12
    for i in range(5):
        zz = z.copy()
        fd = _fd(lambda: nn_ref.bce_loss(zz, y, 2.0)[0], zz, (i,))
        assert abs(fd - dz[i]) < 1e-8


def test_adam_first_step_is_signed_lr():
    p = [np.array([1.0, -2.0, 0.5])]
    g = [np.array([0.3, -4.0, 1e-3])]
    m = [np.zeros(3)]
    v = [np.zeros(3)]
    p1, m1, v1 = nn_ref.adam_step(p, g, m, v, 1, lr=0.01, eps=0.0)
    assert np.allclose(p1[0], p[0] - 0.01 * np.sign(g[0]))


def test_bf16_round_matches_torch_bfloat16():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(9)
    a = np.concatenate([rng.normal(size=2000) * 10.0 ** rng.integers(-30, 30, 2000),
                        [0.0, -0.0, np.inf, -np.inf, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8,
                         3.3895313892515355e38, 1e-40, -1e-42]]).astype(np.float32)
    exp = torch.from_numpy(a).to(torch.bfloat16).to(torch.float64).numpy()
    got = nn_ref.bf16_round(a)
    assert np.array_equal(got, exp)
    assert np.isnan(nn_ref.bf16_round(np.array([np.nan], np.float32))[0])


def test_bf16_storage_is_identity_on_representable_values():
    # activations and gradients that are already bfloat16 values (small
    # integers here) pass the storage rounding unchanged
    rng = np.random.default_rng(4)
    params = [np.round(p * 4) for p in nn_ref.init_params(rng, cin=2, hidden=2)]
    params = [p * 0 + np.clip(p, -2, 2) for p in params]
    x = rng.integers(-2, 3, size=(1, 3, 3, 3, 2)).astype(np.float64)
    z, c = nn_ref.forward(params, x)
    zb, cb = nn_ref.forward(params, x, bf16_storage=True)
    assert np.array_equal(z, zb)
    g = nn_ref.backward(params, c, np.sign(z))
    gb = nn_ref.backward(params, cb, np.sign(z), bf16_storage=True)
    for a, b in zip(g, gb):
        assert np.array_equal(a, b)
