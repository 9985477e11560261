"""Exact floating-point rounding for the oracle (test infrastructure only).

The paper's notation (Section 2.1) uses ``single`` (binary32, round to nearest
even), ``single_up`` and ``single_down`` (binary32 with rounding toward +inf and
-inf), and asks for the squared norms "with rounding-up" (Algorithms 1 and 2).
Every one of those operations is a correctly rounded result of an exact real
operand, so the oracle computes the operand exactly (a ``Fraction``, or an
integer times a power of two) and rounds it with ``round_rational`` or
``round_dyadic`` below.  Nothing here depends on the host's FPU
rounding mode.

The fast base-2 logarithm of the paper (a vendor math-library routine with an
absolute error of at most 4*u32 on [1, 2), Section 2.3 and Section 4) is
replaced by the correctly rounded binary32 log2 (``log2_rn32``), whose error is
at most half an ulp, i.e. at most 2**-25 on [1, 2]: it satisfies the only
property the paper's proof uses, and it is uniquely defined, so a GPU
implementation can be checked against it bit for bit.
"""
from __future__ import annotations

import decimal
import math
from fractions import Fraction

import numpy as np

# (precision p, minimum normal exponent, maximum exponent) of IEEE 754 formats.
BINARY64 = (53, -1022, 1023)
BINARY32 = (24, -126, 127)

# Unit roundoff of binary32; the paper writes u_32 without defining it.
U32 = Fraction(1, 2**24)

INF = float("inf")


def _pow2(e: int) -> Fraction:
    return Fraction(2) ** e if e >= 0 else Fraction(1, 2 ** (-e))


def floor_log2(x: Fraction) -> int:
    """The integer e with 2**e <= x < 2**(e+1), for a rational x > 0."""
    if x <= 0:
        raise ValueError("floor_log2 needs x > 0")
    e = x.numerator.bit_length() - x.denominator.bit_length()
    if _pow2(e) > x:
        e -= 1
    assert _pow2(e) <= x < _pow2(e + 1)
    return e


def round_rational(x, fmt=BINARY64, mode: str = "RN"):
    """Round the exact rational ``x`` to the format ``fmt``.

    ``mode`` is one of ``RN`` (nearest, ties to even), ``RU`` (toward +inf),
    ``RD`` (toward -inf) or ``RZ`` (toward zero).  Subnormal results are
    rounded on the subnormal grid.  Returns a ``Fraction`` holding the exact
    value of the result, or ``+inf``/``-inf`` (Python floats) on overflow, as
    IEEE 754 prescribes for each mode.
    """
    x = Fraction(x)
    prec, emin, emax = fmt
    if x == 0:
        return Fraction(0)
    neg = x < 0
    a = -x if neg else x
    e = floor_log2(a)
    q = max(e, emin) - (prec - 1)  # exponent of the last kept bit (the quantum)
    scaled = a / _pow2(q)
    n = scaled.numerator // scaled.denominator
    rem = scaled - n
    if mode == "RN":
        up = rem > Fraction(1, 2) or (rem == Fraction(1, 2) and n % 2 == 1)
    elif mode == "RU":
        up = rem > 0 and not neg
    elif mode == "RD":
        up = rem > 0 and neg
    elif mode == "RZ":
        up = False
    else:
        raise ValueError(mode)
    n += int(up)
    mag = n * _pow2(q)
    maxfinite = (2**prec - 1) * _pow2(emax - prec + 1)
    if mag > maxfinite:
        # Overflow: RN goes to inf; directed modes stop at the largest finite
        # value on the side they do not round toward.
        if mode == "RN" or (mode == "RU" and not neg) or (mode == "RD" and neg):
            return -INF if neg else INF
        mag = maxfinite
    return -mag if neg else mag


def round_dyadic(n: int, e: int, fmt=BINARY64, mode: str = "RN") -> float:
    """Round the exact value n * 2**e (integers n, e) to ``fmt``.

    Same rounding rules as ``round_rational``, specialised to dyadic values
    (every sum and product of binary64 numbers is one); the result is a
    Python float holding the exact rounded value (binary32 results included,
    since binary32 is a subset of binary64), or +-inf.
    """
    prec, emin, emax = fmt
    if n == 0:
        return 0.0
    neg = n < 0
    a = -n if neg else n
    top = e + a.bit_length() - 1          # floor(log2 |value|)
    q = max(top, emin) - (prec - 1)       # exponent of the quantum
    if q <= e:
        mant, q = a << (e - q), q
    else:
        sh = q - e
        mant = a >> sh
        rem = a - (mant << sh)
        half = 1 << (sh - 1)
        if mode == "RN":
            up = rem > half or (rem == half and (mant & 1) == 1)
        elif mode == "RU":
            up = rem != 0 and not neg
        elif mode == "RD":
            up = rem != 0 and neg
        elif mode == "RZ":
            up = False
        else:
            raise ValueError(mode)
        mant += int(up)
    if _exceeds_max(mant, q, fmt):
        # Overflow: RN goes to inf; directed modes stop at the largest finite
        # value on the side they do not round toward.
        if mode == "RN" or (mode == "RU" and not neg) or (mode == "RD" and neg):
            return -INF if neg else INF
        v = math.ldexp(float((1 << prec) - 1), emax - prec + 1)
        return -v if neg else v
    v = math.ldexp(float(mant), q)        # exact: mant <= 2**prec
    return -v if neg else v


def _exceeds_max(mant: int, q: int, fmt) -> bool:
    prec, _, emax = fmt
    # largest finite = (2**prec - 1) * 2**(emax - prec + 1)
    lhs_e, rhs_e = q, emax - prec + 1
    if lhs_e >= rhs_e:
        return mant << (lhs_e - rhs_e) > (1 << prec) - 1
    return mant > ((1 << prec) - 1) << (rhs_e - lhs_e)


def int_exp(x: float):
    """Exact decomposition x = n * 2**e of a finite binary64 value."""
    num, den = float(x).as_integer_ratio()
    return num, -(den.bit_length() - 1)


def to_float(v) -> float:
    """Python float holding the exact value of a binary64 result."""
    if isinstance(v, float):
        return v
    f = float(v)
    assert Fraction(f) == v, "value is not representable in binary64"
    return f


def to_f32(v) -> np.float32:
    """numpy float32 holding the exact value of a binary32 result."""
    if isinstance(v, float):
        return np.float32(v)
    f = np.float32(float(v))
    assert Fraction(float(f)) == v, "value is not representable in binary32"
    return f


def ru64(x) -> float:
    return to_float(round_rational(x, BINARY64, "RU"))


def rn64(x) -> float:
    return to_float(round_rational(x, BINARY64, "RN"))


def ru32(x) -> Fraction:
    """single_up(x): the exact value of the binary32 result as a Fraction."""
    return round_rational(x, BINARY32, "RU")


def rd32(x) -> Fraction:
    """single_down(x): the exact value of the binary32 result as a Fraction."""
    return round_rational(x, BINARY32, "RD")


def rn32(x) -> Fraction:
    """single(x): round to nearest even in binary32."""
    return round_rational(x, BINARY32, "RN")


# ---------------------------------------------------------------------------
# Rounded-up sums of squares (the norm bound of Algorithms 1 and 2)
# ---------------------------------------------------------------------------

def ru_square(a: float) -> float:
    """RU_64(a*a): the square of a binary64 value rounded toward +inf."""
    if not math.isfinite(a):
        return math.nan if math.isnan(a) else INF
    n, e = int_exp(a)
    return round_dyadic(n * n, 2 * e, BINARY64, "RU")


def ru_add(x: float, y: float) -> float:
    """RU_64(x + y) for binary64 x, y (inf propagates, NaN too)."""
    if math.isnan(x) or math.isnan(y):
        return math.nan
    if math.isinf(x) or math.isinf(y):
        return INF
    nx, ex = int_exp(x)
    ny, ey = int_exp(y)
    e = min(ex, ey)
    return round_dyadic((nx << (ex - e)) + (ny << (ey - e)), e, BINARY64, "RU")


# ---------------------------------------------------------------------------
# Base-2 logarithm
# ---------------------------------------------------------------------------

_LOG_PREC = 70  # decimal digits; the error of the decimal result is < 1e-65


def log2_decimal(x: Fraction, prec: int = _LOG_PREC) -> decimal.Decimal:
    """log2(x) for a rational x > 0, to ``prec`` significant decimal digits."""
    with decimal.localcontext() as ctx:
        ctx.prec = prec + 10
        num = decimal.Decimal(x.numerator)
        den = decimal.Decimal(x.denominator)
        v = (num.ln() - den.ln()) / decimal.Decimal(2).ln()
        ctx.prec = prec
        return +v


def log2_rn32(xf: Fraction) -> Fraction:
    """Correctly rounded (nearest-even) binary32 log2 of a binary32 value.

    This is the oracle's stand-in for the fast single-precision log2 of the
    paper (Sections 2.3 and 4).  Its absolute error on [1, 2] is at most
    2**-25, inside the 4*u32 = 2**-22 the paper's proof allows.  log2(x) is
    rational only at powers of two (where decimal returns it exactly), so the
    rounding decision is never a tie; we still assert that the decimal value
    is far from a rounding midpoint compared with its own error.
    """
    xf = Fraction(xf)
    if xf <= 0:
        raise ValueError("log2 of a non-positive value")
    if xf.denominator == 1 and (xf.numerator & (xf.numerator - 1)) == 0:
        return Fraction(xf.numerator.bit_length() - 1)
    if xf.numerator == 1 and (xf.denominator & (xf.denominator - 1)) == 0:
        return Fraction(-(xf.denominator.bit_length() - 1))
    d = Fraction(log2_decimal(xf))
    r = round_rational(d, BINARY32, "RN")
    # Guard: the exact log2 lies within err of d; the rounding of d is the
    # rounding of the exact value unless a midpoint lies within err of d.
    err = Fraction(1, 10**60) * max(1, abs(d))
    lo = round_rational(d - err, BINARY32, "RN")
    hi = round_rational(d + err, BINARY32, "RN")
    assert lo == r == hi, "log2 too close to a binary32 rounding midpoint"
    return r
