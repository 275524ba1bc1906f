"""Reduced-precision storage formats, as value maps on FP64 numbers (test
infrastructure only).

A field stored in FP32 holds the FP32 rounding of each real number (round to
nearest, ties to even).  A field stored in bfloat16 (1 sign bit, 8 exponent
bits, 7 stored fraction bits: 8 significant bits) holds the bfloat16 rounding
(round to nearest, ties to even) of that FP32 value: an FP64 input reaches
BF16 through FP32, the conversion the library documents for its inputs and
links.  These maps let the oracle evaluate an operator exactly on the values
a reduced-precision evaluation actually reads, so the comparison with such an
evaluation isolates its arithmetic from the rounding of its inputs.
"""
from __future__ import annotations

import numpy as np


def fp32_value(a):
    """Each real part rounded to FP32, returned in FP64 (complex kept)."""
    a = np.asarray(a)
    if np.iscomplexobj(a):
        return fp32_value(a.real) + 1j * fp32_value(a.imag)
    return a.astype(np.float32).astype(np.float64)


def _bf16_of_fp32(f):
    """Round FP32 numbers to 8 significant bits, ties to even, by integer
    arithmetic on their bit patterns (finite inputs)."""
    u = np.ascontiguousarray(f, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = ((u + 0x7FFF + lsb) >> 16) << 16
    return u.astype(np.uint32).view(np.float32)


def bf16_value(a):
    """Each real part stored in bfloat16 via FP32, returned in FP64."""
    a = np.asarray(a)
    if np.iscomplexobj(a):
        return bf16_value(a.real) + 1j * bf16_value(a.imag)
    return _bf16_of_fp32(a.astype(np.float32)).astype(np.float64)


UNIT_ROUNDOFF = {"fp64": 2.0 ** -53, "fp32": 2.0 ** -24, "bf16": 2.0 ** -8}
