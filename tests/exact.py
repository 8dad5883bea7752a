"""Exact-arithmetic helpers for tests: correctly rounded FP32/BF16 from rationals.

Independent of the C oracle: a value is carried as a Python Fraction and
rounded to the nearest FP32 (or BF16) number, ties to even, with gradual
underflow and overflow to infinity, by integer arithmetic on the rational.
"""
from fractions import Fraction

import numpy as np


def frac(x) -> Fraction:
    return Fraction(float(x))


def _round_to_grid(q: Fraction, sig_bits: int, emin: int, emax: int) -> float:
    """Nearest number with `sig_bits` significant bits (ties to even) whose
    exponent is >= emin (gradual underflow) and <= emax (else +-inf)."""
    if q == 0:
        return 0.0
    s = -1 if q < 0 else 1
    a = abs(q)
    # exponent e with 2^e <= a < 2^(e+1)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    e = max(e, emin)
    ulp = Fraction(2) ** (e - (sig_bits - 1))
    m = a / ulp
    fl = m.numerator // m.denominator
    rem = m - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    r = fl * ulp
    if r >= Fraction(2) ** (emax + 1):
        return s * float("inf")
    return s * float(r)


def fl32(q: Fraction) -> np.float32:
    """Correctly rounded FP32 value of a rational."""
    return np.float32(_round_to_grid(q, 24, -126, 127))


def bf16_nearest(q: Fraction) -> float:
    """Correctly rounded BF16 value of a rational (overflow to +-inf)."""
    return _round_to_grid(q, 8, -126, 127)


def fma32(a, b, c) -> np.float32:
    return fl32(frac(a) * frac(b) + frac(c))


def add32(a, b) -> np.float32:
    return fl32(frac(a) + frac(b))
