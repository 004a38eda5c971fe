"""GPU: the allocation-free network forward (mf4d_nn_forward_noalloc), called
through the C ABI, against mf4d_nn_forward on the same inputs: logits equal
bit for bit on two calls in a row (the second smaller, so it runs on the
scratch the first left behind), and a size beyond the static scratch is
refused with MF4D_ERR_RANGE."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _inputs(seed, shape):
    rng = np.random.default_rng(seed)
    x = np.zeros(shape + (16,), np.float32)
    x[..., :8] = rng.normal(size=shape + (8,))
    return torch.from_numpy(x).to(torch.bfloat16).to("cuda:0").contiguous()


def test_noalloc_forward_equals_forward_twice():
    from paper_1903_12294_amd import _lib
    from paper_1903_12294_amd.learned import Net, init_params
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lib = _lib.load_library()
    net = Net(0)
    try:
        net.set_params(init_params(5) + np.float32(0.01))
        for seed, shape in [(1, (4, 16, 64, 64)), (2, (3, 5, 7, 9))]:
            print(f"[noalloc] shape {shape}", flush=True)
            x = _inputs(seed, shape)
            want = net.forward(x)
            got = torch.full(shape, float("nan"), dtype=torch.float32, device="cuda:0")
            N, D, H, W = shape
            rc = lib.mf4d_nn_forward_noalloc(net.ptr, ctypes.c_void_p(x.data_ptr()), N, D, H, W,
                                             ctypes.c_void_p(got.data_ptr()), _lib.MF4D_DEVICE)
            assert rc == 0, lib.mf4d_net_last_error()
            torch.cuda.synchronize()
            assert torch.equal(got, want), shape
        # beyond the scratch: 2^18 + 1 positions
        x = torch.zeros((1, 1, 1, (1 << 18) + 1, 16), dtype=torch.bfloat16, device="cuda:0")
        out = torch.empty((1, 1, 1, (1 << 18) + 1), dtype=torch.float32, device="cuda:0")
        rc = lib.mf4d_nn_forward_noalloc(net.ptr, ctypes.c_void_p(x.data_ptr()), 1, 1, 1, (1 << 18) + 1,
                                         ctypes.c_void_p(out.data_ptr()), _lib.MF4D_DEVICE)
        assert rc == _lib.MF4D_ERR_RANGE
        assert b"scratch" in lib.mf4d_net_last_error()
    finally:
        net.close()
