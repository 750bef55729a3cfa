"""Block-scaled FP8 (E4M3) quantization of range-finder operands, for
checking the FP8 range finder.

TEST INFRASTRUCTURE ONLY: imported by the tests and the checker scripts,
never by the library.  It shares no code with the GPU path.

Formats, as the Open Compute Project's 8-bit floating point and
microscaling (MX) specifications define them:

* E4M3: sign, 4 exponent bits (bias 7), 3 mantissa bits.  Normal values
  (1 + m/8) 2^(e - 7) for exponent field e = 1..15 (e = 15 with m = 7 is NaN,
  so the largest finite value is 448); subnormals (m/8) 2^-6.  No infinities.
* E8M0 scale: an unsigned byte b standing for 2^(b - 127).
* A block is 32 consecutive elements along the contraction index; all share
  one scale.

The reading taken here (the method itself only asks for per-block scaling
and a refinement step):
* the value is first rounded to FP32 (operands in FP64 included), then the
  block scale is 2^(E - 7) with E = floor(log2(max |v|)) over the block, so
  the block maximum lands in [128, 256) and no element saturates; an all-zero
  block takes scale 2^0;
* each element is v / scale rounded to the nearest E4M3 value, ties to even
  mantissa; values below the smallest subnormal half-way point become zero.
"""
from __future__ import annotations

import numpy as np

BLOCK = 32
E4M3_MAX = 448.0


def e4m3_values() -> np.ndarray:
    """The value of every code 0..255 (NaN for the two NaN codes)."""
    v = np.empty(256)
    for code in range(256):
        s = -1.0 if code & 0x80 else 1.0
        e = (code >> 3) & 0xF
        m = code & 7
        if e == 15 and m == 7:
            v[code] = np.nan
        elif e == 0:
            v[code] = s * (m / 8.0) * 2.0 ** -6
        else:
            v[code] = s * (1.0 + m / 8.0) * 2.0 ** (e - 7)
    return v


_VALUES = e4m3_values()
# finite non-negative values in increasing order, with their codes
_POS_CODES = np.array([c for c in range(0x7F)], dtype=np.int64)     # 0x00..0x7E
_POS_VALUES = _VALUES[_POS_CODES]


def encode_e4m3(x: np.ndarray) -> np.ndarray:
    """Nearest E4M3 code of each |x| <= 448 (ties to the even code, i.e. the
    even mantissa), sign kept; by direct search of the value table."""
    x = np.asarray(x, dtype=np.float64)
    a = np.abs(x)
    if np.any(a > E4M3_MAX):
        raise ValueError("value outside the E4M3 range")
    idx = np.searchsorted(_POS_VALUES, a)            # first value >= a
    idx = np.clip(idx, 1, len(_POS_VALUES) - 1)
    lo, hi = _POS_VALUES[idx - 1], _POS_VALUES[idx]
    below = (a - lo) < (hi - a)
    above = (a - lo) > (hi - a)
    tie_even = (_POS_CODES[idx - 1] & 1) == 0
    pick_lo = below | (~above & tie_even)
    code = np.where(pick_lo, _POS_CODES[idx - 1], _POS_CODES[idx])
    code = np.where(a == 0.0, 0, code)
    sign = np.where(np.signbit(x) & (code != 0), 0x80, 0)
    return (code | sign).astype(np.uint8)


def decode_e4m3(codes: np.ndarray) -> np.ndarray:
    return _VALUES[np.asarray(codes, dtype=np.int64)]


def block_scale_exponents(v32: np.ndarray) -> np.ndarray:
    """Scale exponent of each block of 32 along the last axis (length a
    multiple of 32): floor(log2(max |v|)) - 7, or 0 for an all-zero block."""
    b = np.abs(v32.reshape(v32.shape[:-1] + (-1, BLOCK))).max(axis=-1).astype(np.float64)
    e = np.zeros(b.shape, dtype=np.int64)
    nz = b > 0
    e[nz] = np.floor(np.log2(b[nz])).astype(np.int64) - 7
    return e


def quantize_rows(a: np.ndarray):
    """Block-scaled E4M3 of a 2-D array along its rows (blocks of 32
    consecutive columns, zero-padded to a multiple of 32).  Returns (codes,
    scale exponents, dequantized values of the original shape)."""
    a = np.asarray(a)
    r, c = a.shape
    cp = -(-c // BLOCK) * BLOCK
    v = np.zeros((r, cp), dtype=np.float32)
    v[:, :c] = a.astype(np.float32)
    e = block_scale_exponents(v)
    scale = np.repeat(np.ldexp(1.0, e), BLOCK, axis=-1)
    codes = encode_e4m3(v.astype(np.float64) / scale)
    deq = decode_e4m3(codes) * scale
    return codes, e, deq[:, :c]


def product(a: np.ndarray, x: np.ndarray) -> np.ndarray:
    """a @ x with both operands block-quantized along the contraction index
    (rows of a, columns of x), accumulated in FP64."""
    _, _, aq = quantize_rows(a)
    _, _, xq = quantize_rows(np.asarray(x).T)
    return aq @ xq.T
