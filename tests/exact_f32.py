"""Exact rational evaluation with IEEE-754 binary32 rounding, for pinning the
oracle's FP32 operation chains.

Every operation is carried out exactly on ``fractions.Fraction`` values and
then rounded once to the nearest binary32 value, ties to the even
significand (IEEE-754 roundTiesToEven).  A fused multiply-add rounds the
exact a*b + c once; an unfused one rounds the product and then the sum.
Nothing here calls the oracle or numpy's float32 arithmetic, so a mismatch
with the oracle points at the oracle.
"""
from fractions import Fraction

_MIN_EXP = -126      # smallest normal binary32 exponent
_MANT = 23           # stored significand bits


def round_f32(q):
    """Nearest binary32 value to the rational q (ties to even), as a Python
    float (exact: every binary32 value is a binary64 value)."""
    q = Fraction(q)
    if q == 0:
        return 0.0
    neg = q < 0
    a = -q if neg else q
    # exponent e with 2^e <= a < 2^(e+1)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    while Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    e = max(e, _MIN_EXP)  # below the normal range the spacing stays 2^-149
    ulp = Fraction(2) ** (e - _MANT)
    m = a / ulp
    fl = m.numerator // m.denominator
    rem = m - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    r = fl * ulp
    if r >= Fraction(2) ** 128:
        r = float("inf")
        return -r if neg else r
    return float(-r if neg else r)


def F(x):
    """Exact rational value of a float (binary32 values pass through binary64 exactly)."""
    return Fraction(float(x))


def fma(a, b, c):
    """binary32 fused multiply-add: a*b + c rounded once."""
    return round_f32(F(a) * F(b) + F(c))


def mul(a, b):
    return round_f32(F(a) * F(b))


def add(a, b):
    return round_f32(F(a) + F(b))


def div(a, b):
    return round_f32(F(a) / F(b))
