"""Pins of the checker's block-scaled FP8 (E4M3) quantizer (oracle/fp8.py)
against the format's definition (Open Compute Project 8-bit floating point:
bias 7, 3 mantissa bits, largest finite 448, subnormals m/8 2^-6, NaN at
S.1111.111) and the microscaling convention of one power-of-two scale per
block of 32 elements."""
import numpy as np
import pytest

from oracle import fp8


def test_decode_known_codes():
    v = fp8.e4m3_values()
    assert v[0x38] == 1.0
    assert v[0x40] == 2.0
    assert v[0x7E] == 448.0                        # largest finite: 1.75 2^8
    assert v[0x08] == 2.0 ** -6                    # smallest normal
    assert v[0x01] == 2.0 ** -9                    # smallest subnormal
    assert v[0x07] == 7 * 2.0 ** -9
    assert np.isnan(v[0x7F]) and np.isnan(v[0xFF])
    assert v[0xB8] == -1.0 and v[0x80] == 0.0 and np.signbit(v[0x80])
    finite = v[np.isfinite(v)]
    assert len(finite) == 254


def test_encode_roundtrip_every_finite_code():
    v = fp8.e4m3_values()
    codes = np.array([c for c in range(256) if np.isfinite(v[c]) and c != 0x80])
    assert np.array_equal(fp8.encode_e4m3(v[codes]), codes.astype(np.uint8))


@pytest.mark.parametrize("x,code", [
    (1.0625, 0x38),            # half way 1 .. 1.125: tie to the even mantissa (1)
    (1.1875, 0x3A),            # half way 1.125 .. 1.25: tie to 1.25
    (1.06, 0x38), (1.07, 0x39),
    (0.5 * 2.0 ** -9, 0x00),   # half the smallest subnormal: tie to zero
    (0.75 * 2.0 ** -9, 0x01),
    (7.5 * 2.0 ** -9, 0x08),   # half way between the last subnormal and 2^-6
    (440.0, 0x7E), (-3.0, 0xC4),
])
def test_encode_rounding(x, code):
    assert int(fp8.encode_e4m3(np.array([x]))[0]) == code


def test_encode_rejects_out_of_range():
    with pytest.raises(ValueError):
        fp8.encode_e4m3(np.array([449.0]))


def test_block_scales():
    v = np.zeros((1, 96), dtype=np.float32)
    v[0, 5] = 200.0            # block 0: max in [128, 256): scale 2^0
    v[0, 40] = -1.0            # block 1: max 1: scale 2^-7
    e = fp8.block_scale_exponents(v)                # block 2: all zero: 2^0
    assert e.tolist() == [[0, -7, 0]]


def test_quantization_error_bound():
    """Relative error at most 2^-4 (half a unit of the 3-bit mantissa) for
    elements in the normal range of their block, absolute at most half the
    smallest subnormal times the scale below it."""
    rng = np.random.default_rng(3)
    a = (rng.standard_normal((40, 250)) * np.exp(rng.uniform(-6, 6, (40, 1)))).astype(np.float32)
    codes, e, deq = fp8.quantize_rows(a)
    cp = codes.shape[1]
    scale = np.repeat(np.ldexp(1.0, e), 32, axis=1)[:, :250]
    v = a.astype(np.float64)
    normal = np.abs(v) / scale >= 2.0 ** -6
    assert np.all(np.abs(deq - v)[normal] <= 2.0 ** -4 * np.abs(v)[normal])
    assert np.all(np.abs(deq - v)[~normal] <= 2.0 ** -10 * scale[~normal] + 1e-300)
    # the block maximum lands in [128, 256) after scaling, so nothing saturates
    amax = np.abs(np.pad(v, ((0, 0), (0, cp - 250)))).reshape(40, -1, 32).max(axis=2)
    ratio = amax / np.ldexp(1.0, e)
    assert np.all((ratio >= 128) & (ratio < 256))


def test_product_exact_on_small_integers():
    """Integers |a| <= 16 and |x| <= 4 are exact in E4M3 under any power-of-two
    block scale that keeps them in range, so the quantized product is a @ x."""
    rng = np.random.default_rng(5)
    a = rng.integers(-16, 17, size=(37, 75)).astype(np.float64)
    x = rng.integers(-4, 5, size=(75, 9)).astype(np.float64)
    assert np.array_equal(fp8.product(a, x), a @ x)
