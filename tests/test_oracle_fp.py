"""Pins for the oracle's exact rounding and logarithm (CPU only).

Each check compares the oracle with an independent implementation:
CPython's correctly rounded Fraction->float and int/int division, the host
FPU under fesetround() (tests/fenv_ref.c), and glibc's log2.
"""
import ctypes
import math
import os
import random
import struct
import subprocess
import tempfile
from fractions import Fraction

import numpy as np
import pytest

from oracle import fp

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def fenv():
    d = tempfile.mkdtemp()
    so = os.path.join(d, "fenv_ref.so")
    subprocess.check_call(["gcc", "-O0", "-frounding-math", "-shared", "-fPIC",
                           os.path.join(HERE, "fenv_ref.c"), "-o", so, "-lm"])
    lib = ctypes.CDLL(so)
    lib.ru_square.restype = ctypes.c_double
    lib.ru_square.argtypes = [ctypes.c_double]
    lib.ru_add.restype = ctypes.c_double
    lib.ru_add.argtypes = [ctypes.c_double, ctypes.c_double]
    lib.f64_to_f32.restype = ctypes.c_float
    lib.f64_to_f32.argtypes = [ctypes.c_double, ctypes.c_int]
    lib.ru_norm_chunked.restype = ctypes.c_double
    lib.ru_norm_chunked.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64]
    return lib


def _random_doubles(rng, n):
    out = []
    for _ in range(n):
        kind = rng.random()
        if kind < 0.6:
            out.append(rng.uniform(-1, 1) * 2.0 ** rng.randint(-60, 60))
        elif kind < 0.8:
            out.append(rng.uniform(-1, 1) * 2.0 ** rng.randint(-1074, 1023))
        elif kind < 0.9:   # subnormal
            out.append(rng.randint(1, 2**52 - 1) * 2.0 ** -1074 * rng.choice([-1, 1]))
        else:              # exact small integers / powers of two
            out.append(float(rng.randint(-2**20, 2**20)) * 2.0 ** rng.randint(-30, 30))
    return out


def test_round_rational_rn_matches_cpython():
    """RN of random rationals (normal, subnormal, overflow) equals CPython's
    correctly rounded Fraction.__float__."""
    rng = random.Random(1)
    for _ in range(3000):
        num = rng.randint(-10**40, 10**40)
        den = rng.randint(1, 10**40)
        scale = Fraction(2) ** rng.randint(-1200, 1100)
        x = Fraction(num, den) * scale
        try:
            ref = float(x)
        except OverflowError:
            ref = math.inf if x > 0 else -math.inf
        got = fp.round_rational(x, fp.BINARY64, "RN")
        assert float(got) == ref, x


def test_round_dyadic_matches_cpython_division():
    """round_dyadic RN equals CPython's correctly rounded int / 2**e."""
    rng = random.Random(2)
    for _ in range(5000):
        n = rng.randint(-2**200, 2**200)
        e = rng.randint(-1300, 900)
        try:
            ref = n * 2.0 ** e if e >= 0 and abs(n) < 2**53 else (
                n / (1 << -e) if e < 0 else float(n << e))
        except OverflowError:
            ref = math.inf if n > 0 else -math.inf
        assert fp.round_dyadic(n, e, fp.BINARY64, "RN") == ref


def test_directed_rounding_matches_fenv(fenv):
    """RU squares, RU sums and RU/RD binary64->binary32 conversions equal the
    host FPU's results under FE_UPWARD / FE_DOWNWARD."""
    rng = random.Random(3)
    xs = _random_doubles(rng, 4000)
    for a in xs:
        assert fp.ru_square(a) == fenv.ru_square(a), a
        if abs(a) < 2.0 ** 120 and abs(a) > 2.0 ** -140:
            assert float(fp.ru32(Fraction(a))) == fenv.f64_to_f32(a, 1), a
            assert float(fp.rd32(Fraction(a))) == fenv.f64_to_f32(a, 0), a
    for a, b in zip(xs[::2], xs[1::2]):
        a, b = abs(a), abs(b)
        assert fp.ru_add(a, b) == fenv.ru_add(a, b), (a, b)
    # Overflow of a rounded-up square goes to +inf.
    assert fp.ru_square(2.0 ** 600) == math.inf == fenv.ru_square(2.0 ** 600)
    # Underflow rounds up to the smallest subnormal, never to zero.
    assert fp.ru_square(2.0 ** -600) == 2.0 ** -1074 == fenv.ru_square(2.0 ** -600)


def test_log2_rn32_against_glibc():
    """Correctly rounded binary32 log2 on [1, 2]: equals glibc's binary64
    log2 rounded to binary32 wherever that rounding is unambiguous, and is
    always within half a binary32 ulp (<= 2**-25) of log2."""
    rng = np.random.default_rng(4)
    bits = np.concatenate([
        rng.integers(0x3F800000, 0x40000001, 1500),
        np.arange(0x3F800000, 0x3F800000 + 200),
        np.arange(0x40000000 - 200, 0x40000001),
    ]).astype(np.uint32)
    checked = 0
    for b in bits:
        x = struct.unpack("<f", struct.pack("<I", int(b)))[0]
        L = fp.log2_rn32(Fraction(x))
        y = math.log2(x)
        assert abs(Fraction(y) - L) <= Fraction(1, 2**25) + Fraction(1, 2**50)
        # glibc's binary64 log2 is within 1 binary64 ulp; its binary32 rounding
        # is the correct one unless y is within that error of a midpoint.
        f = float(np.float32(y))
        ulp32 = 2.0 ** (math.frexp(f)[1] - 25) if f != 0 else 2.0 ** -149
        lo_mid, hi_mid = f - ulp32 / 2, f + ulp32 / 2
        if min(abs(y - lo_mid), abs(y - hi_mid)) > 4 * 2.0 ** -52:
            assert float(L) == f
            checked += 1
    assert checked > 1500
    assert fp.log2_rn32(Fraction(1)) == 0
    assert fp.log2_rn32(Fraction(2)) == 1


def test_floor_log2_and_int_exp():
    for x in [1.0, 1.5, 2.0, 3.0, 0.75, 2.0 ** -1074, 1.7976931348623157e308]:
        assert fp.floor_log2(Fraction(x)) == math.frexp(x)[1] - 1
        n, e = fp.int_exp(x)
        assert n * Fraction(2) ** e == Fraction(x)
