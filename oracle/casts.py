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


# ---------------------------------------------------------------------------
# FP8 e4m3 (the OCP "e4m3fn" encoding: 1 sign, 4 exponent bits with bias 7,
# 3 mantissa bits, no infinities, S.1111.111 is NaN, largest finite 448,
# smallest normal 2^-6, subnormals in steps of 2^-9).  The paper has no FP8
# form; this is the reduced-precision form below bfloat16 that gfx950 stores
# natively.  Defined by its value table, rounded to nearest with ties to the
# even code, by exhaustive search (plain, slow, obviously correct).
# ---------------------------------------------------------------------------

def e4m3_value(code: int) -> float:
    """Value of one e4m3 code (NaN for the two NaN codes)."""
    code = int(code) & 0xFF
    s = -1.0 if code & 0x80 else 1.0
    e = (code >> 3) & 0xF
    m = code & 0x7
    if e == 15 and m == 7:
        return float("nan")
    if e == 0:
        return s * (m / 8.0) * 2.0 ** -6
    return s * (1.0 + m / 8.0) * 2.0 ** (e - 7)


E4M3_TABLE = np.array([e4m3_value(c) for c in range(256)])
E4M3_MAX = 448.0


def e4m3_bits(x) -> np.ndarray:
    """Nearest e4m3 code of each value (ties to the even code); |x| above the
    rounding range of 448 and NaN give the NaN code 0x7F (sign kept)."""
    xs = np.asarray(x, dtype=np.float64).ravel()
    pos = np.array([c for c in range(0x7F)])          # finite non-negative codes 0x00..0x7E
    vals = E4M3_TABLE[pos]
    out = np.empty(xs.size, dtype=np.uint8)
    for i, v in enumerate(xs):
        sign = 0x80 if (np.signbit(v) and not np.isnan(v)) else 0
        a = abs(v)
        if np.isnan(v) or a >= 464.0:                 # 464 = midpoint of 448 and the next step
            out[i] = 0x7F | sign
            continue
        d = np.abs(vals - a)
        best = np.flatnonzero(d == d.min())
        c = best[0] if best.size == 1 else [b for b in best if b % 2 == 0][0]
        out[i] = int(pos[c]) | sign
    return out.reshape(np.shape(x))


def e4m3_decode(bits) -> np.ndarray:
    return E4M3_TABLE[np.asarray(bits, dtype=np.uint8)]


def to_e4m3(x) -> np.ndarray:
    """Round to the nearest e4m3 value (float64 result)."""
    return e4m3_decode(e4m3_bits(x))
