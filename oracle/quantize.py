"""Scoring-row number formats, from their definitions (test infrastructure).

The float path scores candidates on reduced-precision copies of the points
(the measured configurations ask for bfloat16 rows, and FP8 E4M3 rows with
one scale per row); stored distances are float32.  These are the plain
definitions the GPU's ingest is checked against:

* bfloat16: the 16 high bits of an IEEE float32 after rounding the float32
  to 8 significand bits, round to nearest, ties to even.
* FP8 E4M3 (OCP 8-bit floating point, "E4M3"): sign bit, 4 exponent bits
  with bias 7, 3 mantissa bits; exponent field 0 encodes subnormals
  m/8 * 2^-6; there are no infinities, 0x7f / 0xff are NaN, so the largest
  finite magnitude is 1.75 * 2^8 = 448.  Encoding = the nearest finite
  value (ties: even mantissa code); magnitudes beyond 448 take 448; the
  sign bit is the input's, also when the magnitude rounds to zero.
* Row scale: s = max_j |x_j| / 448 in float32 (0 for a zero row) and codes
  E4M3(x_j / s), both divisions in float32, so that the integer codes are
  decided in the kernel's precision.
"""

from __future__ import annotations

import numpy as np


def bf16_bits(x: np.ndarray) -> np.ndarray:
    """float32 -> bfloat16 bit patterns (uint16), round to nearest even.

    Written from the definition: keep the high 16 bits, and round up when
    the dropped 16 bits exceed half an ulp, or equal it with an odd kept
    part.  Finite inputs only.
    """
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    hi = u >> 16
    lo = u & 0xFFFF
    up = (lo > 0x8000) | ((lo == 0x8000) & ((hi & 1) == 1))
    return (hi + up.astype(np.uint64)).astype(np.uint16)


def bf16_value(bits: np.ndarray) -> np.ndarray:
    return (np.asarray(bits, dtype=np.uint32) << 16).view(np.float32)


def e4m3_value(code: int) -> float:
    """Value of an E4M3 code by the format's definition (NaN for 0x7f/0xff)."""
    s = -1.0 if code & 0x80 else 1.0
    e = (code >> 3) & 0xF
    m = code & 0x7
    if e == 0xF and m == 0x7:
        return float("nan")
    if e == 0:
        return s * (m / 8.0) * 2.0 ** -6
    return s * (1.0 + m / 8.0) * 2.0 ** (e - 7)


def e4m3_table() -> tuple[np.ndarray, np.ndarray]:
    """Non-negative finite codes 0x00..0x7e and their values (ascending)."""
    codes = np.arange(0x7F, dtype=np.int64)
    vals = np.array([e4m3_value(int(c)) for c in codes], dtype=np.float64)
    return codes, vals


def e4m3_codes(v: np.ndarray) -> np.ndarray:
    """Nearest finite E4M3 code of each float32 value (ties to even code)."""
    v = np.asarray(v, dtype=np.float32).astype(np.float64)
    codes, vals = e4m3_table()
    a = np.abs(v)
    # nearest by brute force over the 127 magnitudes (exact in float64)
    diff = np.abs(a[..., None] - vals)                  # [..., 127]
    best = diff.min(axis=-1, keepdims=True)
    tie = diff == best
    # among the nearest, prefer the even code (the set has at most two)
    even = tie & ((codes & 1) == 0)
    pick = np.where(even.any(axis=-1), even.argmax(axis=-1), tie.argmax(axis=-1))
    out = codes[pick].astype(np.uint8)
    # the sign is kept when the magnitude rounds to zero (IEEE rounding of
    # a negative value gives negative zero)
    sign = np.signbit(v).astype(np.uint8) << 7
    return out | sign


def fp8_rows(x: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Per-row scale s = max |x| / 448 (float32) and codes E4M3(x / s)."""
    x = np.asarray(x, dtype=np.float32)
    mx = np.abs(x).max(axis=1).astype(np.float32)
    s = (mx / np.float32(448.0)).astype(np.float32)
    safe = np.where(s > 0, s, np.float32(1.0)).astype(np.float32)
    q = (x / safe[:, None]).astype(np.float32)
    codes = e4m3_codes(q)
    codes[s == 0] = 0
    return codes, s
