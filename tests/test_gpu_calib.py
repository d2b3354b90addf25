"""The HBM read-stream calibration kernel (rp_read_stream): every 16-byte word
of the buffer is read exactly once, so the XOR of the per-thread folds equals
the XOR of all 32-bit words of the buffer, for any grid and unroll; bad
arguments are refused on the host."""
import ctypes

import numpy as np
import pytest

from gpu_helpers import log

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("n16,grid,unroll", [(1, 1, 1), (65536 + 3, 7, 4), (300001, 64, 8), (4096, 5000, 2)])
def test_read_stream_reads_every_word_once(n16, grid, unroll):
    from paper_2311_15429_amd import _lib
    lib = _lib.load()
    words = np.random.default_rng(n16).integers(-2**31, 2**31, size=4 * n16, dtype=np.int64).astype(np.int32)
    buf = torch.from_numpy(words).to("cuda")
    sink = torch.full((grid * 256,), -1, dtype=torch.int32, device="cuda")
    st = lib.rp_read_stream(ctypes.c_void_p(buf.data_ptr()), ctypes.c_size_t(16 * n16),
                            ctypes.c_void_p(sink.data_ptr()), grid, unroll,
                            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0
    torch.cuda.synchronize()
    got = np.bitwise_xor.reduce(sink.cpu().numpy().view(np.uint32))
    want = np.bitwise_xor.reduce(words.view(np.uint32))
    log(f"n16 {n16}, grid {grid}, unroll {unroll}: xor {got:#010x}")
    assert got == want


def test_read_stream_refuses_bad_arguments():
    from paper_2311_15429_amd import _lib
    lib = _lib.load()
    buf = torch.zeros(64, dtype=torch.int32, device="cuda")
    sink = torch.zeros(256, dtype=torch.int32, device="cuda")
    p, q = ctypes.c_void_p(buf.data_ptr()), ctypes.c_void_p(sink.data_ptr())
    assert lib.rp_read_stream(p, ctypes.c_size_t(256), q, 1, 3, None) == 1          # unroll
    assert lib.rp_read_stream(p, ctypes.c_size_t(250), q, 1, 1, None) == 1          # not 16-byte words
    assert lib.rp_read_stream(p, ctypes.c_size_t(256), q, 0, 1, None) == 1          # grid
    assert lib.rp_read_stream(None, ctypes.c_size_t(256), q, 1, 1, None) == 1       # null buffer
    assert lib.rp_read_stream(ctypes.c_void_p(buf.data_ptr() + 4), ctypes.c_size_t(240), q, 1, 1, None) == 1
