"""Values as the library stores them at 16 bits, each real rounded to nearest-even: fields
given as complex64 from their FP32 values; links, given in FP64, once from FP64 at FP16 and from
their FP32 value at BF16."""
import numpy as np


def _bf16(x32):
    u = np.ascontiguousarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def stored(a, prec, links=False):
    """complex128 -> the value held at FP16 (prec 2) or BF16 (prec 3); links=True for the gauge
    field (FP16 rounded directly from FP64), else a field passed as complex64."""
    a = np.asarray(a)
    f = a.astype(np.complex64)
    if prec == 2:
        src = a.astype(np.complex128) if links else f
        return src.real.astype(np.float16).astype(np.float64) + 1j * src.imag.astype(np.float16).astype(np.float64)
    return _bf16(f.real) + 1j * _bf16(f.imag)
