"""Rounding of matrix values to 16-bit storage formats, written from the IEEE 754
binary16 and bfloat16 definitions (round to nearest, ties to even).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Reading taken for the half-precision value storage (a future-work item of
Sec. 5): the FP64 value is first rounded to FP32, then to the 16-bit format.
"""

from __future__ import annotations

import numpy as np


def round_to_bf16(x) -> np.ndarray:
    """Round to bfloat16 (8 exponent bits, 7 stored mantissa bits) and return the
    value as float64.  FP32 bits ``u``: add ``0x7FFF + ((u >> 16) & 1)`` and clear the
    low 16 bits (round to nearest even; NaN is not expected in matrix values)."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def round_to_f16(x) -> np.ndarray:
    """Round to IEEE binary16 through FP32, returned as float64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    return f.astype(np.float16).astype(np.float64)


def round_values(S, fmt: str):
    """Copy of the sparse matrix ``S`` with its values rounded to ``fmt``."""
    T = S.copy()
    if fmt == "f32":
        T.data = T.data.astype(np.float32).astype(np.float64)
    elif fmt == "bf16":
        T.data = round_to_bf16(T.data)
    elif fmt == "f16":
        T.data = round_to_f16(T.data)
    elif fmt != "f64":
        raise ValueError(fmt)
    return T
