"""fp64 reference of the brick-activity predictor (forward, backward, loss).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Network over a grid of bricks, applied to each timestep's 3D brick grid
independently: conv3d(Cin -> 16, 3x3x3, zero "same" padding) -> ReLU ->
conv3d(16 -> 16) -> ReLU -> conv3d(16 -> 1) -> sigmoid.  Loss: binary cross
entropy with a weight on positive targets, averaged over positions.

Written as direct sums over the 27 kernel offsets (no im2col, no FFT) so that
it can be checked by eye; pinned by central finite differences in
tests/test_nn_ref.py.

Layouts: activations [N, D, H, W, C] (N = timesteps, channels last);
weights [Cout, Cin, 3, 3, 3] (kz, ky, kx); biases [Cout].
"""
from __future__ import annotations

import numpy as np

OFFSETS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def _shift(x, dz, dy, dx):
    """y[n, z, y, x, c] = x[n, z + dz, y + dy, x + dx, c], zero outside."""
    out = np.zeros_like(x)
    N, D, H, W, C = x.shape
    zs = slice(max(0, -dz), D - max(0, dz))
    ys = slice(max(0, -dy), H - max(0, dy))
    xs = slice(max(0, -dx), W - max(0, dx))
    zd = slice(max(0, dz), D + min(0, dz))
    yd = slice(max(0, dy), H + min(0, dy))
    xd = slice(max(0, dx), W + min(0, dx))
    out[:, zs, ys, xs, :] = x[:, zd, yd, xd, :]
    return out


def conv3d(x, w, b):
    """out[n,z,y,x,co] = b[co] + sum_{ci,k} w[co,ci,k] * x[n, (z,y,x)+off(k), ci]."""
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    out = np.zeros(x.shape[:4] + (w.shape[0],), np.float64)
    for k, (dz, dy, dx) in enumerate(OFFSETS):
        xs = _shift(x, dz, dy, dx)
        wk = w[:, :, dz + 1, dy + 1, dx + 1]  # [Cout, Cin]
        out += xs @ wk.T
    return out + np.asarray(b, np.float64)


def conv3d_backward(x, w, dout):
    """Gradients of sum(dout * conv3d(x, w, b)) w.r.t. x, w and b."""
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    dout = np.asarray(dout, np.float64)
    dx = np.zeros_like(x)
    dw = np.zeros_like(w)
    for k, (dz, dy, dx_) in enumerate(OFFSETS):
        xs = _shift(x, dz, dy, dx_)
        wk = w[:, :, dz + 1, dy + 1, dx_ + 1]
        # dw[co, ci] = sum_n dout[n, co] * xs[n, ci]
        dw[:, :, dz + 1, dy + 1, dx_ + 1] = (dout.reshape(-1, dout.shape[-1]).T @
                                             xs.reshape(-1, xs.shape[-1]))
        # dx[p + off] += dout[p] @ wk  ->  dx += shift(dout @ wk, -off)
        dx += _shift(dout @ wk, -dz, -dy, -dx_)
    db = dout.reshape(-1, dout.shape[-1]).sum(0)
    return dx, dw, db


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def bf16_round(a):
    """Nearest bfloat16 value of each float32 value (ties to even), as float64;
    NaN stays NaN.  bfloat16 keeps float32's sign, exponent and the top 7
    mantissa bits, so rounding is integer arithmetic on the float32 bits."""
    a32 = np.asarray(a, np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    r = (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16).astype(np.uint32)
    out = r.view(np.float32)
    return np.where(np.isnan(a32), a32, out).astype(np.float64)


def forward(params, x, bf16_storage: bool = False):
    """Returns (logits [N,D,H,W], cache).

    With bf16_storage the hidden activations are rounded to bfloat16 after the
    ReLU and the logits to float32, as when they are stored in those types
    between layers; the arithmetic itself stays fp64."""
    w1, b1, w2, b2, w3, b3 = params
    rnd = bf16_round if bf16_storage else (lambda a: a)
    z1 = conv3d(x, w1, b1)
    a1 = rnd(np.maximum(z1, 0))
    z2 = conv3d(a1, w2, b2)
    a2 = rnd(np.maximum(z2, 0))
    z3 = conv3d(a2, w3, b3)[..., 0]
    if bf16_storage:
        z3 = z3.astype(np.float32).astype(np.float64)
    return z3, (x, z1, a1, z2, a2)


def bce_loss(logits, y, pos_weight):
    """mean over positions of -(w*y*log s + (1-y)*log(1-s)), s = sigmoid(z)."""
    z = np.asarray(logits, np.float64)
    y = np.asarray(y, np.float64)
    # log s = -softplus(-z), log(1-s) = -softplus(z)
    sp_neg = np.logaddexp(0, -z)
    sp_pos = np.logaddexp(0, z)
    loss = pos_weight * y * sp_neg + (1 - y) * sp_pos
    dz = (sigmoid(z) * (pos_weight * y + 1 - y) - pos_weight * y) / z.size
    return loss.mean(), dz


def backward(params, cache, dlogits, bf16_storage: bool = False):
    """Parameter gradients; with bf16_storage each layer's output gradient is
    rounded to bfloat16 before it is used (as when stored in that type)."""
    w1, b1, w2, b2, w3, b3 = params
    x, z1, a1, z2, a2 = cache
    rnd = bf16_round if bf16_storage else (lambda a: a)
    d3 = rnd(np.asarray(dlogits, np.float64))[..., None]
    da2, dw3, db3 = conv3d_backward(a2, w3, d3)
    dz2 = rnd(da2 * (z2 > 0))
    da1, dw2, db2 = conv3d_backward(a1, w2, dz2)
    dz1 = rnd(da1 * (z1 > 0))
    _, dw1, db1 = conv3d_backward(x, w1, dz1)
    return [dw1, db1, dw2, db2, dw3, db3]


def init_params(rng, cin=8, hidden=16):
    """He-style initial weights (fp64)."""
    def w(co, ci):
        return rng.normal(0, np.sqrt(2.0 / (ci * 27)), size=(co, ci, 3, 3, 3))
    return [w(hidden, cin), np.zeros(hidden), w(hidden, hidden), np.zeros(hidden),
            w(1, hidden), np.zeros(1)]


def adam_step(params, grads, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns new params, m, v."""
    out_p, out_m, out_v = [], [], []
    for p, g, mm, vv in zip(params, grads, m, v):
        mm = b1 * mm + (1 - b1) * g
        vv = b2 * vv + (1 - b2) * g * g
        mhat = mm / (1 - b1 ** t)
        vhat = vv / (1 - b2 ** t)
        out_p.append(p - lr * mhat / (np.sqrt(vhat) + eps))
        out_m.append(mm)
        out_v.append(vv)
    return out_p, out_m, out_v
