"""Step 1 of Ozaki scheme II and the single-precision scaling constants
(test infrastructure only).

Section 2.2, Step 1: pick pairwise coprime moduli p_1..p_N, P = prod p_i,
P_i = P / p_i and q_i = P_i^{-1} mod p_i (Theorem 1, the CRT).
Section 3.1 prints the twenty moduli used by the evaluation.  The paper uses
N < 20 moduli as well (Section 5) without saying which; the reading taken
here is "the first N of the printed list".

Section 2.3 defines P'_accu = single_down(log2(P-1)/2 - 0.5),
P'_fast = single_down(log2(P-1)/2 - 1.5) and
delta = single_up(0.5 / (1 - 4 u32)); Section 4 defines
P'_prop = single_down(log2(P-1)/2 - 0.5), which equals P'_accu.
u32 is not defined in the paper; the reading is the binary32 unit roundoff
2**-24.
"""
from __future__ import annotations

import math
from fractions import Fraction

from . import fp

# The moduli printed in Section 3.1, in printed order.
MODULI = (256, 255, 253, 251, 247, 241, 239, 233, 229, 227,
          223, 217, 211, 199, 197, 193, 191, 181, 179, 173)

N_MIN, N_MAX = 2, len(MODULI)


def moduli(N: int) -> tuple:
    """The first N moduli of the printed list (reading of Section 5's N < 20)."""
    if not N_MIN <= N <= N_MAX:
        raise ValueError(f"N must be in [{N_MIN}, {N_MAX}]")
    return MODULI[:N]


def step1(N: int):
    """Step 1 (Section 2.2): returns (p, P, [P_i], [q_i])."""
    p = moduli(N)
    P = math.prod(p)
    Pi = [P // pi for pi in p]
    qi = [pow(Pi_, -1, pi) for Pi_, pi in zip(Pi, p)]
    return p, P, Pi, qi


def _log2_half_minus(P: int, c: Fraction, mode: str) -> Fraction:
    """single_{mode}(log2(P-1)/2 - c), rounded exactly from a decimal value
    whose error is checked against the distance to the binary32 grid."""
    d = Fraction(fp.log2_decimal(Fraction(P - 1))) / 2 - c
    r = fp.round_rational(d, fp.BINARY32, mode)
    err = Fraction(1, 10**60) * max(1, abs(d))
    assert fp.round_rational(d - err, fp.BINARY32, mode) == r
    assert fp.round_rational(d + err, fp.BINARY32, mode) == r
    return r


def p_prime_prop(N: int) -> Fraction:
    """P'_prop = single_down(log2(P-1)/2 - 0.5) (Section 4)."""
    _, P, _, _ = step1(N)
    return _log2_half_minus(P, Fraction(1, 2), "RD")


def p_prime_accu(N: int) -> Fraction:
    """P'_accu = single_down(log2(P-1)/2 - 0.5) (Section 2.3, accurate mode)."""
    return p_prime_prop(N)


def p_prime_fast(N: int) -> Fraction:
    """P'_fast = single_down(log2(P-1)/2 - 1.5) (Section 2.3, fast mode)."""
    _, P, _, _ = step1(N)
    return _log2_half_minus(P, Fraction(3, 2), "RD")


def delta() -> Fraction:
    """delta = single_up(0.5 / (1 - 4 u32)) (Section 2.3)."""
    return fp.ru32(Fraction(1, 2) / (1 - 4 * fp.U32))


def f32_bits(v: Fraction) -> int:
    """IEEE binary32 bit pattern of an exactly representable value."""
    import struct
    return struct.unpack("<I", struct.pack("<f", float(v)))[0]
