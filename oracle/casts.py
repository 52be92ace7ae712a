"""Reduced-precision casts (oracle).

TEST INFRASTRUCTURE: only tests, the smoke check and the benchmark's CPU
baseline may use this module.

bfloat16 keeps the top 16 bits of a single-precision word (Section "Casting
between single-precision and bfloat16"), so widening a bfloat16 back to single
precision is exact: append 16 zero bits.  The paper does not state the
rounding mode of the narrowing cast; round-to-nearest-even is the reading used
here, and the paper's template-conversion statistics (Table 1: |relative
difference| <= 0.39 %, mean ~ 0) fix it against truncation (which would bias
every value downwards by up to 0.78 %).
"""
from __future__ import annotations

import numpy as np


def bf16_bits(x) -> np.ndarray:
    """RNE narrowing of float32 values to bfloat16 bit patterns (uint16)."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) & 0xFFFF
    nan = np.isnan(f)
    r = np.where(nan, (u >> 16) | 0x40, r)          # keep NaN quiet
    return r.astype(np.uint16)


def bf16_widen(bits) -> np.ndarray:
    """bfloat16 bit patterns -> float32 by appending 16 zero bits (exact)."""
    b = np.ascontiguousarray(bits, dtype=np.uint16).astype(np.uint32) << 16
    return b.view(np.float32)


def to_bf16(x) -> np.ndarray:
    """float32 -> nearest bfloat16 value (RNE), returned as float32."""
    return bf16_widen(bf16_bits(x))


def bf16_truncate(x) -> np.ndarray:
    """Truncating narrowing (drop the low 16 bits); used only to show that the
    paper's statistics reject it."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    return ((f.view(np.uint32) >> 16) << 16).view(np.float32)
