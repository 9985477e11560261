"""Pins for Step 1 and the single-precision constants (CPU only)."""
import math
import struct
from fractions import Fraction

import numpy as np
import pytest

from oracle import constants, fp


def _bits(x):
    return struct.unpack("<I", struct.pack("<f", float(x)))[0]


def test_moduli_are_pairwise_coprime_and_fit_int8_products():
    p = constants.MODULI
    assert len(p) == 20 and len(set(p)) == 20
    for i in range(20):
        for j in range(i + 1, 20):
            assert math.gcd(p[i], p[j]) == 1
    # The residues lie in [-128, 127]; |C_t| <= k * 128**2 < 2**31 for k <= 2**17.
    assert 2**17 * 128 * 128 == 2**31


@pytest.mark.parametrize("N", [2, 5, 9, 14, 17, 20])
def test_crt_reconstructs_every_residue_vector(N):
    """Theorem 1: for random x in (-P/2, P/2), sum_t P_t q_t (x mod p_t)
    reduced with rmod(., P) gives back x."""
    from oracle import ozaki2
    p, P, Pi, qi = constants.step1(N)
    rng = np.random.default_rng(N)
    for _ in range(200):
        x = int(rng.integers(0, 2**62)) * int(rng.integers(1, 2**62)) * int(rng.integers(1, 2**40))
        x = x % P - P // 2
        y = sum(Pi[t] * qi[t] * (x % p[t]) for t in range(N))
        assert ozaki2.rmod(y, P) == x


@pytest.mark.parametrize("N", range(2, 21))
def test_p_prime_against_glibc_log2(N):
    """P'_prop = RD32(log2(P-1)/2 - 0.5) and P'_fast = RD32(... - 1.5):
    the decimal-based values agree with glibc's binary64 log2 of the big
    integer P-1 rounded down to binary32 (glibc is independent of the
    oracle's decimal logarithm; the check is skipped only where the binary64
    value is too close to a binary32 grid point to decide)."""
    _, P, _, _ = constants.step1(N)
    y = math.log2(P - 1)  # glibc/CPython, error ~1e-16 relative
    for c, val in ((0.5, constants.p_prime_prop(N)), (1.5, constants.p_prime_fast(N))):
        x = y / 2 - c
        lo = float(np.float32(x))
        if lo > x:
            lo = float(np.nextafter(np.float32(lo), np.float32(-np.inf)))
        grid_dist = min(abs(x - lo), abs(float(np.nextafter(np.float32(lo), np.float32(np.inf))) - x))
        if grid_dist > 1e-12:
            assert float(val) == lo, (N, c)
    assert constants.p_prime_accu(N) == constants.p_prime_prop(N)


def test_delta_closed_form():
    """delta = RU32(0.5 / (1 - 2**-22)).  0.5/(1-2**-22) = 0.5 + 2**-23 + 2**-45
    + ..., strictly between 0.5 + 2 * 2**-24 and 0.5 + 3 * 2**-24 (ulp(0.5)
    = 2**-24 in binary32), so rounding up gives 0.5 + 3 * 2**-24 = 0x3F000003."""
    assert _bits(constants.delta()) == 0x3F000003


def test_p_prime_fast_is_prop_minus_one_within_a_binade():
    """Both constants round log2(P-1)/2 - c down on the binary32 grid; where
    both values lie in one binade the grid shift by exactly 1 is exact."""
    for N in range(2, 21):
        pp, pf = constants.p_prime_prop(N), constants.p_prime_fast(N)
        if math.frexp(float(pp))[1] == math.frexp(float(pf))[1]:
            assert pf == pp - 1
