"""The library's copy kernel (used between pyramid levels and as the bandwidth
probe of the benchmark), through the C ABI: vector and element paths."""

import sys

import pytest
import torch

from paper_1605_02060_amd import lddmm as L

pytestmark = pytest.mark.gpu
DEV = "cuda"


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("n,offset", [(1 << 20, 0), (1000003, 0), (7, 0), (1 << 16, 1),
                                      (33333, 3), (1, 0)])
def test_copy_is_exact(n, offset):
    say(f"lddmm_copy n={n} offset={offset}")
    g = torch.Generator(device="cpu").manual_seed(n)
    buf = torch.randn(n + offset, generator=g).to(DEV)
    src = buf[offset:]
    dst = torch.full((n + 2,), -7.0, device=DEV)
    L.lddmm_copy(src, dst[1:n + 1])
    torch.cuda.synchronize()
    assert torch.equal(dst[1:n + 1], src)
    assert dst[0].item() == -7.0 and dst[n + 1].item() == -7.0     # nothing written outside


def test_copy_arguments():
    say("lddmm_copy arguments")
    lib = L.load()
    s = torch.cuda.current_stream().cuda_stream
    import ctypes
    assert lib.lddmm_copy(None, None, 0, ctypes.c_void_p(s)) == L.OK
    assert lib.lddmm_copy(None, None, 5, ctypes.c_void_p(s)) == L.EINVAL
    x = torch.zeros(4, device=DEV)
    assert lib.lddmm_copy(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr()), -1,
                          ctypes.c_void_p(s)) == L.EINVAL
