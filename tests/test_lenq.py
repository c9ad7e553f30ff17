"""One-byte lengths (section II-B): the device reads a byte q as the float
q / 180 through two FMAs instead of a division.  Checked here in exact
rational arithmetic for all 256 bytes: the result is q / 180 correctly
rounded to FP32, which is how the oracle dequantizes."""
from fractions import Fraction

import numpy as np


def rn32(x: Fraction) -> Fraction:
    """x rounded to the nearest FP32 value, ties to even (normal range)."""
    if x == 0:
        return Fraction(0)
    s = -1 if x < 0 else 1
    a = abs(x)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    ulp = Fraction(2) ** (e - 23)
    m = a / ulp
    n = m.numerator // m.denominator
    rem = m - n
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and n % 2 == 1):
        n += 1
    return s * n * ulp


def test_rn32_agrees_with_numpy():
    rng = np.random.default_rng(0)
    for v in rng.random(200) * 3.0:
        assert float(rn32(Fraction(float(v)))) == float(np.float32(v))


def test_two_fma_dequantization_is_correctly_rounded():
    c = rn32(Fraction(1, 180))
    for q in range(256):
        x = Fraction(q)
        r = rn32(x * c)
        e = rn32(-r * 180 + x)  # fma: one rounding
        got = rn32(e * c + r)   # fma: one rounding
        assert got == rn32(Fraction(q, 180)), q
        assert float(got) == float(np.float32(q) / np.float32(180.0)), q
