"""HBM read-stream calibration through ``rp_read_stream``: the practical read
bandwidth of the device, timed with HIP events on the caller's stream."""
import ctypes

from . import _lib

# (loads in flight per thread, blocks per compute unit) tried; the best is kept
LAUNCHES = ((2, 4), (4, 4), (8, 8), (8, 16), (1, 8))


def read_stream_gbs(nbytes=4 << 30, reps=5, launches=LAUNCHES):
    """Best read bandwidth (GB/s) over `launches`, each the best of `reps`
    timed reads of an `nbytes` device buffer; returns (GB/s, (unroll, blocks per CU))."""
    import torch
    lib = _lib.load()
    dev = torch.cuda.current_device()
    n_cu = torch.cuda.get_device_properties(dev).multi_processor_count
    buf = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    grid_max = max(b for _, b in launches) * n_cu
    sink = torch.empty(grid_max * 256, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    h = ctypes.c_void_p(stream.cuda_stream)
    best, best_cfg = 0.0, None
    for unroll, bpc in launches:
        grid = bpc * n_cu
        for r in range(reps + 1):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            st = lib.rp_read_stream(ctypes.c_void_p(buf.data_ptr()), ctypes.c_size_t(buf.numel() * 4),
                                    ctypes.c_void_p(sink.data_ptr()), grid, unroll, h)
            if st != 0:
                raise _lib.RpotError(st, "rp_read_stream failed")
            e1.record(stream)
            e1.synchronize()
            if r == 0:
                continue                      # first launch of a shape: not timed
            gbs = buf.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9
            if gbs > best:
                best, best_cfg = gbs, (unroll, bpc)
    del buf, sink
    return best, best_cfg
