"""ctypes view of libinrf_peaks.so (include/inrf_peaks.h): the benchmark's
measurement kernels, a streaming HBM read and a matrix-core loop.  PyTorch
provides the buffers, stream and events; the kernels are the library's."""
from __future__ import annotations

import ctypes
import os
from ctypes import c_int32, c_int64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libinrf_peaks.so")
EXPORTED = ["inrf_peaks_last_error", "inrf_peak_read_sink_size", "inrf_peak_hbm_read", "inrf_peak_mfma_waves",
            "inrf_peak_mfma"]
FLOP_PER_MFMA = {"fp32": 2048, "fp16": 16384, "bf16": 16384}
PRECISION = {"fp32": 0, "fp16": 1, "bf16": 2}

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2303_04086_amd.build.build()")
        _lib = ctypes.CDLL(LIB_PATH)
        _lib.inrf_peaks_last_error.restype = ctypes.c_char_p
        _lib.inrf_peak_read_sink_size.restype = c_int32
        _lib.inrf_peak_hbm_read.restype = c_int32
        _lib.inrf_peak_hbm_read.argtypes = [c_void_p, c_int64, c_int32, c_void_p, c_void_p]
        _lib.inrf_peak_mfma_waves.restype = c_int64
        _lib.inrf_peak_mfma_waves.argtypes = [c_int32]
        _lib.inrf_peak_mfma.restype = c_int32
        _lib.inrf_peak_mfma.argtypes = [c_int32, c_int32, c_int64, c_void_p, c_void_p]
    return _lib


def _check(st):
    if st != 0:
        raise RuntimeError(lib().inrf_peaks_last_error().decode())


def _timed(torch, fn, trials):
    """Best of `trials` event-timed calls (ms), after one untimed call."""
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(trials):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b))
    return best


def hbm_read(torch, gib: int = 4, reps: int = 2, trials: int = 5) -> dict:
    """Streaming read bandwidth of a gib-GiB buffer, GB/s (best of trials)."""
    n = gib << 30
    buf = torch.ones(n // 4, dtype=torch.int32, device="cuda")
    sink = torch.empty(lib().inrf_peak_read_sink_size(), dtype=torch.int32, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    ms = _timed(torch, lambda: _check(lib().inrf_peak_hbm_read(buf.data_ptr(), n, reps, sink.data_ptr(), s)), trials)
    del buf
    return {"GBps": round(reps * n / (ms / 1e3) / 1e9, 1), "bytes": reps * n, "ms": round(ms, 3)}


def mfma(torch, precision: str, waves_per_simd: int = 2, iters: int = 0, trials: int = 3) -> dict:
    """Matrix-core throughput of the network's instruction, TFLOP/s."""
    waves = int(lib().inrf_peak_mfma_waves(waves_per_simd))
    if waves < 0:
        raise RuntimeError(lib().inrf_peaks_last_error().decode())
    iters = iters or (100_000 if precision == "fp32" else 300_000)
    sink = torch.empty(waves, dtype=torch.float32, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    ms = _timed(torch, lambda: _check(lib().inrf_peak_mfma(PRECISION[precision], waves_per_simd, iters,
                                                           sink.data_ptr(), s)), trials)
    flop = waves * iters * 4 * FLOP_PER_MFMA[precision]
    return {"TFLOPs": round(flop / (ms / 1e3) / 1e12, 1), "waves": waves, "ms": round(ms, 3)}
