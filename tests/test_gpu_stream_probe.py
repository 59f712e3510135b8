"""The benchmark's streaming probe (libstream_probe.so, not part of the
method) moves the bytes it is timed on: the copies reproduce the source, the
write kernel fills the destination with its pattern, and the read kernel's
per-thread sums add up to the sum of the source, for every unroll and for a
size that is not a multiple of one grid pass."""
import ctypes
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _probe():
    from paper_1301_3423_amd import build as _b
    if not os.path.exists(_b.PROBE_OUT):
        raise RuntimeError("libstream_probe.so is not built")
    f = ctypes.CDLL(_b.PROBE_OUT).stream_probe_ms
    f.restype = ctypes.c_double
    f.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                  ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p]
    return f


@pytest.mark.parametrize("unroll", [1, 2, 4, 8])
def test_probe_kernels_move_the_bytes(unroll):
    import torch
    f = _probe()
    n = (3 << 20) + 4 * 37                      # floats: 12 MiB plus a ragged tail of 37 vectors
    grid = 96
    g = torch.Generator().manual_seed(unroll)
    host = torch.randint(-8, 8, (n,), generator=g).to(torch.float32)   # small integers: exact sums
    src = host.cuda()
    sink = torch.zeros(grid * 256, dtype=torch.float32, device="cuda")
    st = torch.cuda.current_stream()
    for kind in (0, 1):
        dst = torch.zeros_like(src)
        assert f(kind, unroll, grid, src.data_ptr(), dst.data_ptr(), None, 4 * n, 2, st.cuda_stream) > 0
        torch.cuda.synchronize()
        assert torch.equal(dst.cpu(), host), kind
    assert f(2, unroll, grid, src.data_ptr(), None, sink.data_ptr(), 4 * n, 2, st.cuda_stream) > 0
    torch.cuda.synchronize()
    assert float(sink.double().sum()) == float(host.double().sum())
    dst = torch.zeros_like(src)
    assert f(3, unroll, grid, None, dst.data_ptr(), None, 4 * n, 2, st.cuda_stream) > 0
    torch.cuda.synchronize()
    assert np.array_equal(dst.cpu().numpy().reshape(-1, 4), np.tile([1.0, 2.0, 3.0, 4.0], (n // 4, 1)))
