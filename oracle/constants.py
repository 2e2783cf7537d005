"""Derive the bit patterns of the constants used by the oracle's ssa_log.

TEST INFRASTRUCTURE: run by hand (``python -m oracle.constants``) and by the
test suite, which checks that oracle/ssa.c holds exactly these values.

  SQRT2  = RN(sqrt 2)
  LN2_HI = ln 2 rounded to nearest at 32 significant bits, so that E*LN2_HI
           is exact for every exponent |E| <= 2^21
  LN2_LO = RN(ln 2 - LN2_HI)
Rounding to binary64 is done on exact rationals (fractions), not via float().
"""
from fractions import Fraction
import struct

import mpmath


def _rn_double(q: Fraction) -> float:
    """Round a positive or negative rational to the nearest binary64 (ties to
    even), exactly."""
    if q == 0:
        return 0.0
    sign = -1 if q < 0 else 1
    q = abs(q)
    e = q.numerator.bit_length() - q.denominator.bit_length()
    # normalise so that 2^52 <= q * 2^(52-e) < 2^53
    while Fraction(2) ** e > q:
        e -= 1
    while Fraction(2) ** (e + 1) <= q:
        e += 1
    scaled = q * Fraction(2) ** (52 - e)
    n = scaled.numerator // scaled.denominator
    rem = scaled - n
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and n % 2 == 1):
        n += 1
    return sign * float(Fraction(n) * Fraction(2) ** (e - 52))


def _bits(d: float) -> int:
    return struct.unpack("<Q", struct.pack("<d", d))[0]


def derive(digits: int = 60):
    mpmath.mp.dps = digits
    ln2 = Fraction(mpmath.nstr(mpmath.log(2), digits, min_fixed=-1, max_fixed=1))
    sqrt2 = Fraction(mpmath.nstr(mpmath.sqrt(2), digits, min_fixed=-1, max_fixed=1))
    # ln2 in [1/2, 1): 32 significant bits -> multiple of 2^-32
    scaled = ln2 * 2 ** 32
    n = scaled.numerator // scaled.denominator
    if scaled - n >= Fraction(1, 2):
        n += 1
    hi = Fraction(n, 2 ** 32)
    lo = _rn_double(ln2 - hi)
    return {"SQRT2": _bits(_rn_double(sqrt2)), "LN2_HI": _bits(float(hi)),
            "LN2_LO": _bits(lo)}


if __name__ == "__main__":
    for k, v in derive().items():
        print("%-7s 0x%016X" % (k, v))
