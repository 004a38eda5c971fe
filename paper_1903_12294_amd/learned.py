"""Brick-activity predictor: Python side of the network kernels in libmf4d.

The network, its gradients and its Adam updates run in the library's HIP
kernels; this module holds the parameter layout, the initial values, the
training loop (which only sequences library calls) and the glue to a Grower.
Tensors are torch device tensors; bf16 inputs are torch.bfloat16.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import MF4D_DEVICE, MF4D_HOST

LAYERS = [(8, 16), (16, 16), (16, 1)]  # (cin, cout)


def _torch():
    import torch
    return torch


def split_params(flat: np.ndarray) -> list:
    """Flat fp32 parameters -> [W1, b1, W2, b2, W3, b3] (W [cout][cin][3][3][3])."""
    out, off = [], 0
    for cin, cout in LAYERS:
        n = cout * cin * 27
        out.append(np.asarray(flat[off:off + n]).reshape(cout, cin, 3, 3, 3))
        off += n
        out.append(np.asarray(flat[off:off + cout]))
        off += cout
    return out


def join_params(parts) -> np.ndarray:
    return np.concatenate([np.asarray(p, np.float32).ravel() for p in parts]).astype(np.float32)


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal weights, zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for cin, cout in LAYERS:
        parts.append(rng.normal(0, np.sqrt(2.0 / (cin * 27)), size=(cout, cin, 3, 3, 3)))
        parts.append(np.zeros(cout))
    return join_params(parts)


class Net:
    """The predictor network on one GPU."""

    def __init__(self, device: int = 0, stream=None):
        self.lib = _lib.load_library()
        torch = _torch()
        if stream is None:
            stream = torch.cuda.current_stream(device).cuda_stream
        self.ptr = ctypes.c_void_p()
        self._check(self.lib.mf4d_net_create(ctypes.byref(self.ptr), device, ctypes.c_void_p(stream)))
        _lib.track(self)
        self.n = self.lib.mf4d_net_num_params()
        self.device = device

    def _check(self, rc):
        if rc != 0:
            raise _lib.MF4DError(rc, (self.lib.mf4d_net_last_error() or b"").decode())

    def close(self):
        if self.ptr:
            self.lib.mf4d_net_destroy(self.ptr)
            self.ptr = ctypes.c_void_p()

    def __del__(self):
        if _lib.finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, flat: np.ndarray):
        flat = np.ascontiguousarray(flat, np.float32)
        assert flat.size == self.n
        self._check(self.lib.mf4d_net_set_params(self.ptr, flat.ctypes.data_as(ctypes.c_void_p),
                                                 MF4D_HOST))

    def get_params(self) -> np.ndarray:
        out = np.zeros(self.n, np.float32)
        self._check(self.lib.mf4d_net_get_params(self.ptr, out.ctypes.data_as(ctypes.c_void_p),
                                                 MF4D_HOST))
        return out

    def forward(self, x):
        torch = _torch()
        N, D, H, W, C = x.shape
        assert C == 16 and x.dtype == torch.bfloat16 and x.is_contiguous()
        out = torch.empty((N, D, H, W), dtype=torch.float32, device=x.device)
        self._check(self.lib.mf4d_net_forward(self.ptr, ctypes.c_void_p(x.data_ptr()), N, D, H, W,
                                              ctypes.c_void_p(out.data_ptr()), MF4D_DEVICE))
        return out

    def grad(self, x, y, pos_weight: float):
        torch = _torch()
        N, D, H, W, _ = x.shape
        g = torch.empty(self.n, dtype=torch.float32, device=x.device)
        loss = ctypes.c_float()
        self._check(self.lib.mf4d_net_grad(self.ptr, ctypes.c_void_p(x.data_ptr()),
                                           ctypes.c_void_p(y.data_ptr()), N, D, H, W,
                                           float(pos_weight), ctypes.c_void_p(g.data_ptr()),
                                           ctypes.byref(loss), MF4D_DEVICE))
        return g, loss.value

    def backward(self, x, y, pos_weight: float):
        """Parameter gradients, input gradient (fp32 [N][D][H][W][16]) and
        loss of the training path (mf4d_nn_backward)."""
        torch = _torch()
        N, D, H, W, _ = x.shape
        g = torch.empty(self.n, dtype=torch.float32, device=x.device)
        dx = torch.empty((N, D, H, W, 16), dtype=torch.float32, device=x.device)
        loss = ctypes.c_float()
        self._check(self.lib.mf4d_nn_backward(self.ptr, ctypes.c_void_p(x.data_ptr()),
                                              ctypes.c_void_p(y.data_ptr()), N, D, H, W,
                                              float(pos_weight), ctypes.c_void_p(g.data_ptr()),
                                              ctypes.c_void_p(dx.data_ptr()), ctypes.byref(loss),
                                              MF4D_DEVICE))
        return g, dx, loss.value

    def train_step(self, x, y, pos_weight: float, lr: float) -> float:
        N, D, H, W, _ = x.shape
        loss = ctypes.c_float()
        self._check(self.lib.mf4d_net_train_step(self.ptr, ctypes.c_void_p(x.data_ptr()),
                                                 ctypes.c_void_p(y.data_ptr()), N, D, H, W,
                                                 float(pos_weight), float(lr), ctypes.byref(loss)))
        return loss.value


def brick_dims(grower) -> tuple:
    d = (ctypes.c_int * 4)()
    grower._check(grower.lib.mf4d_brick_dims(grower.ctx, d))
    return tuple(d)


def features(grower):
    """Network inputs of the grower's data under its current criteria."""
    torch = _torch()
    T, D, H, W = brick_dims(grower)
    x = torch.empty((T, D, H, W, 16), dtype=torch.bfloat16, device=f"cuda:{grower.device}")
    grower._check(grower.lib.mf4d_features(grower.ctx, ctypes.c_void_p(x.data_ptr()), x.numel(),
                                           MF4D_DEVICE))
    return x


def labels(grower):
    """Brick-step labels of the grower's last grow (1 = holds a member)."""
    torch = _torch()
    T, D, H, W = brick_dims(grower)
    y = torch.empty((T, D, H, W), dtype=torch.uint8, device=f"cuda:{grower.device}")
    grower._check(grower.lib.mf4d_brick_labels(grower.ctx, ctypes.c_void_p(y.data_ptr()),
                                               y.numel(), MF4D_DEVICE))
    return y


def set_predictor(grower, net: Net | None, logit_threshold: float = 0.0):
    grower._net_ref = net  # keep it alive while the context uses it
    grower._check(grower.lib.mf4d_set_predictor(grower.ctx, net.ptr if net else None,
                                                float(logit_threshold)))


def make_dataset(variant_seeds, config: int = 2, device: int = 0, log=None):
    """(features, labels) per variant: the config's workload regenerated with
    another data seed, grown by the plain grower on the GPU."""
    from . import synth
    from .grower import Grower
    c = synth.CONFIGS[config]
    out = []
    g = Grower(device=device)
    try:
        for s in variant_seeds:
            inst = synth.make_instance(c["X"], c["Y"], c["Z"], c["T"], c["P"],
                                       n_blobs=c["n_blobs"], seed=int(s), n_seeds=c["n_seeds"],
                                       tau_f=c["tau"], tau_p=c["tau"], crossing=c["crossing"])
            g.load_field(inst["field"])
            g.load_particles(inst["xyz"], inst["attr"])
            g.set_criteria(*inst["crit"])
            g.set_seeds(inst["seeds"])
            g.grow()
            out.append((features(g), labels(g)))
            if log:
                log(f"variant {s}: {int(out[-1][1].sum())} positive brick-steps")
    finally:
        g.close()
    return out


def train(net: Net, data, epochs: int = 20, lr: float = 3e-3, pos_weight: float | None = None,
          log=None) -> list:
    """Adam over the variants, one variant per step, in a fixed order."""
    torch = _torch()
    if pos_weight is None:
        pos = sum(float(y.sum()) for _, y in data)
        tot = sum(y.numel() for _, y in data)
        pos_weight = max(1.0, (tot - pos) / max(pos, 1.0))
    hist = []
    for ep in range(epochs):
        losses = [net.train_step(x, y, pos_weight, lr) for x, y in data]
        hist.append(float(np.mean(losses)))
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.5f}")
    torch.cuda.synchronize()
    return hist
