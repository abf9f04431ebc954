"""The measurement probes through the C ABI: the streaming copy moves every
byte, and the FMA throughput probe computes its chains (each thread's output
is the sum of 16 affine recurrences a <- a*b + c, whose closed form after k
steps is b^k a0 + c (1 - b^k) / (1 - b)) and reports 2 flops per FMA."""
import numpy as np
import pytest
import torch

from paper_1410_1764_amd import chemora as C

pytestmark = pytest.mark.gpu


def test_probe_copy_is_exact():
    n = (1 << 20) + 48
    a = torch.rand(n // 8, dtype=torch.float64, device="cuda")
    b = torch.zeros_like(a)
    C.probe_copy(b, a, n)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("precision,dtype,rtol", [(C.FP64, np.float64, 1e-13),
                                                  (C.MIXED, np.float32, 1e-5)])
def test_probe_fma_computes_its_chains(precision, dtype, rtol):
    iters = 37
    out = torch.zeros(C.lib().chemora_probe_fma_bytes() // 8, dtype=torch.float64, device="cuda")
    flops = C.probe_fma(precision, out, iters)
    torch.cuda.synchronize()
    threads = 8192 * 256
    assert flops == 2 * 16 * iters * threads
    itemsize = np.dtype(dtype).itemsize
    got = out.cpu().numpy().view(dtype)[:threads].astype(np.float64)
    b, c = float(dtype(0.999999)), float(dtype(1e-7))
    tid = np.arange(threads) % 256
    q = np.arange(16)
    a0 = ((tid[:, None] + q[None, :]).astype(dtype) * dtype(1e-3)).astype(np.float64)
    bk = b ** iters
    want = (bk * a0 + c * (1 - bk) / (1 - b)).sum(axis=1)
    assert itemsize * threads <= out.numel() * 8
    np.testing.assert_allclose(got, want, rtol=rtol, atol=1e-12)
