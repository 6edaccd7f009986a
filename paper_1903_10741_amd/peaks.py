"""Python binding of libffspeaks.so (include/ffs_peaks.h): the device peaks the
rooflines divide by, measured on the GPU at hand."""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libffspeaks.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built: run __graft_entry__.build()")
_lib = ctypes.CDLL(LIB_PATH)
for _f in (_lib.ffs_peak_valu_int32, _lib.ffs_peak_mfma_bf16):
    _f.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(ctypes.c_float),
                   ctypes.c_void_p]
    _f.restype = ctypes.c_int


def _run(fn, blocks, iters, dtype):
    sink = torch.zeros(blocks, dtype=dtype, device="cuda")
    ms = ctypes.c_float()
    rc = fn(int(blocks), int(iters), ctypes.c_void_p(sink.data_ptr()), ctypes.byref(ms),
            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    if rc != 0:
        raise RuntimeError(f"{fn.__name__} failed with {rc}")
    return ms.value / 1e3


def ffs_peak_valu_int32(blocks, iters):
    """(seconds, int32 lane-ops per second) of one launch."""
    s = _run(_lib.ffs_peak_valu_int32, blocks, iters, torch.int32)
    return s, blocks * 256 * iters * 64 / s


def ffs_peak_mfma_bf16(blocks, iters):
    """(seconds, bf16 matrix-core FLOP per second) of one launch."""
    s = _run(_lib.ffs_peak_mfma_bf16, blocks, iters, torch.float32)
    return s, blocks * 4 * iters * 4 * (32 * 32 * 16 * 2) / s


def exported_symbols():
    return ["ffs_peak_valu_int32", "ffs_peak_mfma_bf16"]
