"""Pins for the oracle's scale exponents (CPU only)."""
import math
import os
import random
from fractions import Fraction

import numpy as np
import pytest

from oracle import constants, fp, scaling
from paper_2606_29129_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))


def test_norm_matches_fpu_upward_rounding(fenv):
    """The chunked rounded-up sum of squares equals the same loop run by the
    host FPU in FE_UPWARD mode, for the paper's distribution and for
    extreme scalings (2**+-300, 3.7e+-100, tiny values with underflowing
    squares)."""
    rng = np.random.default_rng(5)
    cases = []
    for phi in (0.5, 2.0, 4.0):
        v = inputs.ozaki_matrix(1, 300, phi, seed=int(phi * 10))[0]
        cases += [v, v * 2.0 ** 300, v * 2.0 ** -300, v * 3.7e100, v * 3.7e-100]
    cases.append(rng.standard_normal(200) * 2.0 ** -530)   # squares underflow
    cases.append(np.array([2.0 ** -1074, 3 * 2.0 ** -1074, 0.0, -2.0 ** -1000]))
    cases.append(rng.standard_normal(129) * 1e150)          # sum overflows
    for v in cases:
        v = np.ascontiguousarray(v, dtype=np.float64)
        ref = fenv.ru_norm_chunked(v.ctypes.data, v.size, scaling.KC)
        assert scaling.norm_sq_ru(v) == ref


def test_norm_closed_forms():
    """All-ones of length k sums to exactly k; integer vectors with small sums
    are exact; a non-exact sum is an upper bound within (1 + 2**-52)**(k+1)."""
    for k in (1, 63, 64, 65, 1000):
        assert scaling.norm_sq_ru(np.ones(k)) == float(k)
    v = np.arange(-50, 51, dtype=np.float64)
    assert scaling.norm_sq_ru(v) == float(sum(int(x) ** 2 for x in v))
    v = inputs.ozaki_matrix(1, 777, 1.0, seed=9)[0]
    exact = sum(Fraction(float(x)) ** 2 for x in v)
    S = Fraction(scaling.norm_sq_ru(v))
    assert exact <= S <= exact * (1 + Fraction(1, 2**52)) ** (len(v) + 1)


def _emax(S: float, P: int) -> int:
    """Largest e with 2**(2e+1) * S <= P - 1, by exact comparison."""
    x = Fraction(S)

    def ok(e):
        return fp._pow2(2 * e + 1) * x <= P - 1

    e = math.floor((math.log2(P - 1) - 1 - math.log2(S)) / 2)
    while not ok(e):
        e -= 1
    while ok(e + 1):
        e += 1
    return e


@pytest.mark.parametrize("N", [2, 8, 14, 16, 20])
def test_alg2_is_within_one_of_the_exact_maximum(N):
    """Section 4 defines mu_i as the maximal power of two with
    2 mu_i^2 ||a_i||^2 <= P - 1 (up to the 4 u32 slack of the log).  Algorithm 2
    returns that exponent or one less, never more."""
    _, P, _, _ = constants.step1(N)
    pp = constants.p_prime_prop(N)
    rng = random.Random(N)
    for _ in range(150):
        S = rng.uniform(1, 2) * 2.0 ** rng.randint(-300, 300)
        e = scaling.alg2_log2_mu(S, pp)
        em = _emax(S, P)
        assert em - 1 <= e <= em, (S, e, em)


@pytest.mark.parametrize("N", [5, 14, 20])
def test_alg2_scale_invariance_of_exponent(N):
    """Section 4: for S -> 4**s S (a row scaled by 2**s), log2 mu shifts by
    exactly -s as long as Algorithm 2's w = RD32(P' - 0.5 s) is exact, i.e.
    |P' - 0.5 s| < 64 for both s (P' has bits down to 2^-18).  Beyond that
    the binary32 rounding of w can only lower it, so the exponent is the
    shifted one or one less (a smaller, still valid scale)."""
    pp = constants.p_prime_prop(N)
    rng = random.Random(7 + N)
    for _ in range(100):
        S = rng.uniform(1, 2) * 2.0 ** rng.randint(-200, 200)
        e0 = scaling.alg2_log2_mu(S, pp)
        s0 = math.frexp(S)[1] - 1
        for s in (-300, -17, -1, 1, 5, 150):
            S2 = S * 4.0 ** s
            if S2 == 0 or not math.isfinite(S2):
                continue
            e2 = scaling.alg2_log2_mu(S2, pp)
            if abs(pp - 0.5 * s0) < 64 and abs(pp - 0.5 * (s0 + 2 * s)) < 64:
                assert e2 == e0 - s
            else:
                assert e2 in (e0 - s, e0 - s - 1)


def test_alg2_rounding_of_w_breaks_exact_invariance_at_extreme_scale():
    """A witness that Algorithm 2 as printed (w rounded down to binary32) is
    not exactly scale invariant at 4**300: |P' - 0.5 s| ~ 245 needs a binary32
    ulp of 2^-16, coarser than P''s lowest bit, and for this S the rounding
    crosses an integer of w - t."""
    pp = constants.p_prime_prop(14)
    S = float.fromhex("0x1.1e3f12b23acd6p-3")
    assert scaling.alg2_log2_mu(S, pp) == 56
    assert scaling.alg2_log2_mu(S * 4.0 ** 300, pp) == 56 - 300 - 1


def test_alg1_is_not_scale_invariant():
    """Section 3.1, eq. (effective-precision-fast): with the original fast mode
    the bit width of the integer row falls as alpha grows."""
    pf, d = constants.p_prime_fast(14), constants.delta()
    v = inputs.ozaki_matrix(1, 256, 0.5, seed=3)[0]
    widths = []
    for s in (0, 10, 20, 40):
        a = v * 2.0 ** s
        S = scaling.norm_sq_ru(a)
        amax = float(np.max(np.abs(a)))
        e = scaling.alg1_log2_mu(S, amax, pf, d)
        widths.append(e + fp.floor_log2(Fraction(amax)) + 1)
    assert widths[0] > widths[1] > widths[2] > widths[3]


def test_alg2_all_ones_closed_form():
    """All-ones row of length k times alpha = 2**s, N = 20: S = k alpha**2
    exactly, log2f(1) = 0, so t = 2**-23 and w = P'_prop - 0.5 (log2 k + 2s);
    P'_prop(20) = 77.1856..., hence log2 mu = floor(77.1856 - log2(k)/2) - s:
    72 - s for k = 1024 and 70 - s for k = 16384."""
    pp = constants.p_prime_prop(20)
    for k, base in ((1024, 72), (16384, 70)):
        for s in range(-10, 11):
            S = scaling.norm_sq_ru(np.full(k, 2.0 ** s))
            assert S == k * 4.0 ** s
            assert scaling.alg2_log2_mu(S, pp) == base - s


def test_alg1_all_ones_constant_width_below_threshold():
    """Section 3.1: for all-ones rows with alpha <= k**-1/2 the fast-mode
    exponent gives every integer entry 2**floor(P'_fast - 1), independent of
    alpha."""
    pf, d = constants.p_prime_fast(20), constants.delta()
    top = math.floor(float(pf) - 1)
    for k in (1024, 16384):
        for s in range(-10, 11):
            if 2.0 ** s > k ** -0.5:
                continue
            S = scaling.norm_sq_ru(np.full(k, 2.0 ** s))
            e = scaling.alg1_log2_mu(S, 2.0 ** s, pf, d)
            assert e + s == top


def test_zero_row_gets_exponent_zero():
    assert scaling.alg2_log2_mu(0.0, constants.p_prime_prop(14)) == 0
    assert scaling.norm_sq_ru(np.zeros(100)) == 0.0
