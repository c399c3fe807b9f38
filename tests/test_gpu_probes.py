"""Bandwidth probes through the C ABI (GPU): the copy and triad kernels
write the right values and report a positive time."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    return torch, torch.device("cuda:0")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


@pytest.mark.parametrize("n", [2, 257, 1 << 20])
def test_copy_and_triad_values(torch_dev, n):
    torch, dev = torch_dev
    from paper_1410_1942_amd import _lib as L
    lib = L.load()
    rng = np.random.default_rng(n)
    # small integers: b + 3 c is exact, so a fused multiply-add and separate
    # operations give the same double
    b = torch.from_numpy(rng.integers(-1000, 1000, n).astype(np.float64)).to(dev)
    c = torch.from_numpy(rng.integers(-1000, 1000, n).astype(np.float64)).to(dev)
    a = torch.full_like(b, np.nan)
    ms = ctypes.c_double()
    assert lib.pcg_triad_probe(_ptr(a), _ptr(b), _ptr(c), n, 3.0, 2, None,
                               ctypes.byref(ms)) == L.OK
    torch.cuda.synchronize()
    assert ms.value > 0.0
    assert torch.equal(a, b + 3.0 * c)
    d = torch.full_like(b, np.nan)
    assert lib.pcg_copy_probe(_ptr(b), _ptr(d), n, 2, None, ctypes.byref(ms)) == L.OK
    torch.cuda.synchronize()
    assert ms.value > 0.0
    assert torch.equal(d, b)


def test_triad_refuses_aliasing(torch_dev):
    torch, dev = torch_dev
    from paper_1410_1942_amd import _lib as L
    lib = L.load()
    b = torch.ones(64, dtype=torch.float64, device=dev)
    ms = ctypes.c_double()
    assert lib.pcg_triad_probe(_ptr(b), _ptr(b), _ptr(b), 64, 1.0, 1, None,
                               ctypes.byref(ms)) == L.EINVAL
