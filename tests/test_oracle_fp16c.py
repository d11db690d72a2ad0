"""Pins of the FP16C oracle (oracle/fp16c.py) against numpy's IEEE binary16
and against the format's own definition, exhaustively over the 65536 codes."""
import numpy as np

from oracle import fp16c as C


def test_codes_are_ordered_and_round_trip():
    pos = C.decode(np.arange(0x8000))
    assert pos[0] == 0.0 and pos[-1] == C.MAX_VALUE
    assert np.all(np.diff(pos) > 0)
    codes = np.arange(0x10000).astype(np.uint16)
    assert np.array_equal(C.encode(C.decode(codes)), codes)
    assert np.array_equal(C.decode(codes[0x8000:]), -pos)


def test_normal_and_subnormal_spacing():
    v = C.decode(np.arange(0x8000))
    steps = np.diff(v)
    assert np.all(steps[:0x800] == 2.0 ** -25)               # subnormals and the first normal
    for e in range(1, 16):                                    # 2^11 codes per binade
        blk = steps[e * 0x800:(e + 1) * 0x800 - 1]
        assert np.all(blk == 2.0 ** (e - 15 - 11))


def test_midpoints_round_to_the_even_code():
    c = np.arange(0x7FFF)
    lo, hi = C.decode(c), C.decode(c + 1)
    mid = 0.5 * (lo + hi)
    even = np.where(c % 2 == 0, c, c + 1)
    assert np.array_equal(C.encode(mid).astype(np.int64), even)
    assert np.array_equal(C.encode(np.nextafter(mid, 0)).astype(np.int64), c)
    assert np.array_equal(C.encode(np.nextafter(mid, 3)).astype(np.int64), c + 1)
    assert np.array_equal(C.encode(-mid).astype(np.int64), even | 0x8000)


def test_every_binary16_value_below_two_is_exact():
    h = np.arange(0x10000).astype(np.uint16).view(np.float16).astype(np.float64)
    h = h[np.isfinite(h) & (np.abs(h) < 2.0)]
    assert np.array_equal(C.round_fp16c(h), h)


def test_rounding_error_is_half_that_of_binary16():
    """The format's point: one more significand bit halves the relative
    rounding error of binary16 on normal values (2^-12 against 2^-11)."""
    rng = np.random.default_rng(5)
    x = np.exp2(rng.uniform(-14, 0.99, 200000)) * rng.choice([-1.0, 1.0], 200000)
    e16c = np.abs(C.round_fp16c(x) - x) / np.abs(x)
    e16 = np.abs(x.astype(np.float16).astype(np.float64) - x) / np.abs(x)
    assert e16c.max() <= 2.0 ** -12
    assert 0.99 * 2.0 ** -11 < e16.max() <= 2.0 ** -11
    assert 0.45 < e16c.mean() / e16.mean() < 0.55


def test_subnormals_and_saturation():
    sub16 = np.arange(1, 1024) * 2.0 ** -24                   # binary16 subnormals
    assert np.array_equal(C.round_fp16c(sub16), sub16)
    assert C.encode(2.0 ** -26) == 0                          # half the step: tie to even (0)
    assert C.encode(3 * 2.0 ** -26) == 2                      # 1.5 steps: tie to even (2)
    assert C.encode(5.0) == 0x7FFF and C.encode(-5.0) == 0xFFFF
    assert C.encode(-0.0) == 0x8000 and C.decode(np.uint16(0x8000)) == 0.0
