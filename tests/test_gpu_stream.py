"""gsi_stream_rates, the streaming reference of the roofline figures: the copy reproduces its
source (the destination ends equal to it), the source is untouched, times are positive, and
bad arguments are refused before any launch."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_stream_rates_move_the_bytes_they_time():
    from paper_2306_10379_amd import gsi
    L = gsi.load()
    g = np.random.default_rng(5)
    # more pieces than one sweep of the grid (16384 x 256 threads) covers, a ragged count within
    # one sweep, and a single 16-byte piece
    for n in (9_000_002, 3 * (1 << 20) + 2, 2):
        src = torch.as_tensor(g.standard_normal(n), device="cuda")
        keep = src.clone()
        dst = torch.zeros_like(src)
        us = (ctypes.c_double * 3)()
        st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        assert L.gsi_stream_rates(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), n * 8, 2, us,
                                  st) == 0
        assert all(u > 0 for u in us)
        assert torch.equal(dst, src) and torch.equal(src, keep)
    a = torch.zeros(1024, dtype=torch.float64, device="cuda")
    b = torch.zeros_like(a)
    us = (ctypes.c_double * 3)()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for nbytes, reps in ((1024 * 8 - 8, 2), (1024 * 8, 0), (8, 1)):
        assert L.gsi_stream_rates(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), nbytes, reps, us,
                                  st) == gsi.GSI_EINVAL
    assert L.gsi_stream_rates(ctypes.c_void_p(a.data_ptr() + 8), ctypes.c_void_p(b.data_ptr()), 1024, 1, us,
                              st) == gsi.GSI_EINVAL
    r = gsi.stream_rates(1 << 26, 2)
    print(f"stream rates (64 MiB): copy {r['copy']:.0f}, read {r['read']:.0f}, write {r['write']:.0f} GB/s", flush=True)
    assert r["copy"] > 0 and r["read"] > 0 and r["write"] > 0
