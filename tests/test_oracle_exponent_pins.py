"""Closed-form pins for the oracle's Algorithm 1 (original fast mode) and
accurate-mode exponents (CPU only).

Every expected value below is derived by hand in the docstring of its test
from the formulas of Section 2.3 and the binary32 constants of the scaling
(Appendix values: delta = 0x3F000003 = 1/2 + 3 * 2^-24; for N = 20,
P'_fast = 0x42985F11 = 76.18567657..., P'_accu = P'_prop = 0x429A5F11 =
77.18567657...).  None of them is produced by the oracle.
"""
import math
import struct

import numpy as np
import pytest

from oracle import constants, ozaki2, scaling
from paper_2606_29129_amd import inputs

N20 = 20


def _f32(hexbits: str) -> float:
    return struct.unpack(">f", bytes.fromhex(hexbits))[0]


def test_scaling_constants_used_by_the_derivations():
    """The derivations below use these binary32 constants; the oracle's own
    values must be them (P'_fast is P'_prop - 1: both lie in [64, 128),
    where the binary32 spacing 2^-17 makes the shift by one exact)."""
    assert float(constants.delta()) == _f32("3f000003") == 0.5 + 3 * 2.0 ** -24
    assert float(constants.p_prime_prop(N20)) == _f32("429a5f11")
    assert float(constants.p_prime_accu(N20)) == _f32("429a5f11")
    assert float(constants.p_prime_fast(N20)) == _f32("42985f11")
    assert _f32("42985f11") == _f32("429a5f11") - 1


# Algorithm 1, all-ones rows: A = 2^s J (1 x k), N = 20.
#
# S = k 4^s exactly, so the log of S is the integer L = log2 k + 2s (the
# log2 of the mantissa 1 is 0 and the rounded-up sum is exact).
#  * L <= 0: delta L <= 0 is rounded up to a value <= 0, clamped to 1, and
#    floor(P'_fast - 1) = floor(75.1857) = 75.
#  * L >= 2 (L is even): delta L = L/2 + 3 L 2^-24; rounded up to binary32 it
#    lies in (L/2, L/2 + 2^-17], far below the fraction 0.1857 of P'_fast, so
#    floor(P'_fast - t) = 76 - L/2.
# The largest magnitude is 2^s, so log2 mu = W - s with W = 75 (L <= 0) or
# 76 - L/2 (L >= 2): every entry of A' is 2^W, and A'B' = k 4^W, i.e.
# log2(A'B') = log2 k + 2 W.
#  k = 1024  (log2 k = 10): W = 75 for s <= -4 (at s = -4, L = 2: 76 - 1),
#            W = 71 - s for s >= -4: 74, 73, ..., 61 at s = 10;
#            log2(A'B') = 160 for s <= -4, then 158, 156, 154 at s = -3..-1.
#  k = 16384 (log2 k = 14): W = 75 for s <= -6, W = 69 - s for s >= -6:
#            74 at s = -5 down to 59 at s = 10;
#            log2(A'B') = 164 for s <= -6, then 162, 160, 158, 156, 154 at
#            s = -5..-1.
ALG1_WIDTH = {
    1024: [75] * 7 + list(range(74, 60, -1)),      # s = -10..-4, then -3..10
    16384: [75] * 5 + list(range(74, 58, -1)),     # s = -10..-6, then -5..10
}
ALG1_LOG2_PRODUCT = {
    1024: {-10: 160, -4: 160, -3: 158, -2: 156, -1: 154, 0: 152, 10: 132},
    16384: {-10: 164, -6: 164, -5: 162, -4: 160, -3: 158, -2: 156, -1: 154, 10: 132},
}


@pytest.mark.parametrize("k", [1024, 16384])
def test_alg1_all_ones_exponents(k):
    """Algorithm 1 per s (hand derivation above): the exponent of the scaled
    row, through the whole path (A' entries are exactly 2^W)."""
    pf, d = constants.p_prime_fast(N20), constants.delta()
    widths = ALG1_WIDTH[k]
    assert len(widths) == 21
    for s, W in zip(range(-10, 11), widths):
        S = scaling.norm_sq_ru(np.full(k, 2.0 ** s))
        assert scaling.alg1_log2_mu(S, 2.0 ** s, pf, d) == W - s, s
    for s in (-10, -4, -3, 0, 10):
        A, B = inputs.ones_problem(1, 1, k, s)
        r = ozaki2.gemm(A, B, N20, ozaki2.ORIGINAL)
        W = widths[s + 10]
        assert r["e_rows"] == [W - s] and r["e_cols"] == [W - s]
        assert all(int(x) == 1 << W for x in r["Aint"].ravel())


@pytest.mark.parametrize("k", [1024, 16384])
def test_alg1_all_ones_product_width(k):
    """log2(A'B') of the all-ones product (hand derivation above): 2^160 /
    2^164 below the threshold, falling by 2 per step of s; CRT recovery
    needs A'B' < P/2 with log2(P/2) = 154.37, so it fails exactly for
    s <= -2 (Section 3.1)."""
    _, P, _, _ = constants.step1(N20)
    for s, lg in ALG1_LOG2_PRODUCT[k].items():
        A, B = inputs.ones_problem(1, 1, k, s)
        r = ozaki2.gemm(A, B, N20, ozaki2.ORIGINAL)
        ex = int(ozaki2.exact_product(r["Aint"], r["Bint"])[0, 0])
        assert ex == 1 << lg, s
        assert (ex < P // 2) == (s >= -1)


@pytest.mark.parametrize("k,base", [(1024, 72), (16384, 70)])
def test_accurate_all_ones_closed_form(k, base):
    """Accurate mode, A = B = 2^s J, N = 20, s = -10..10.

    max|a| = 2^s, so mu' = 2^(5 - s) and every bar entry is ceil(2^5) = 32;
    cbar = 32 * 32 * k = 2^(10 + log2 k): 2^20 (k = 1024), 2^24 (k = 16384).
    tilde-log2 of a power of two is its exponent (log2 of the mantissa 1 is
    0): 20 or 24.  delta * 20 = 10 + 60 * 2^-24 rounds up to 10 + 4 * 2^-20;
    delta * 24 = 12 + 72 * 2^-24 rounds up to 12 + 5 * 2^-20.  With
    P'_accu = 77.18567...: floor(77.18567 - 10.000004) = 67 and
    floor(77.18567 - 12.000005) = 65.  So log2 mu = (5 - s) + 67 = 72 - s
    (k = 1024) and (5 - s) + 65 = 70 - s (k = 16384); A' = 2^72 or 2^70
    everywhere, A'B' = 2^154 < P/2, and C = k 4^s exactly."""
    pa, d = constants.p_prime_accu(N20), constants.delta()
    for s in range(-10, 11):
        A = np.full((1, k), 2.0 ** s)
        B = np.full((k, 1), 2.0 ** s)
        emu, enu, Abar, Bbar, Cbar = scaling.accurate_log2(A, B, pa, d)
        assert (Abar == 32).all() and (Bbar == 32).all()
        assert int(Cbar[0, 0]) == 1024 * k
        assert emu == [base - s] and enu == [base - s]
    for s in (-10, 0, 10):
        A, B = inputs.ones_problem(1, 1, k, s)
        r = ozaki2.gemm(A, B, N20, ozaki2.ACCURATE)
        assert all(int(x) == 1 << base for x in r["Aint"].ravel())
        assert float(r["C"][0, 0]) == k * 4.0 ** s


def _accurate_case():
    """A (1 x 86) and B (86 x 2) with hand-chosen bar matrices.

    Row of A: 85 entries 63/32 and one 34/32; max|a| = 63/32 in [1, 2), so
    mu' = 2^5 and the bar row is 85 x 63 and 34 (exact: 32 a is an integer).
    Column 0 of B: 85 x 63/32 and one 51/32 (bar 85 x 63 and 51); column 1 of
    B: all ones (max 1, nu' = 2^5, bar all 32).
    cbar_00 = 85 * 63^2 + 34 * 51 = 337365 + 1734 = 339099;
    cbar_01 = 32 * (85 * 63 + 34) = 32 * 5389 = 172448."""
    a = np.array([63 / 32] * 85 + [34 / 32])
    b0 = np.array([63 / 32] * 85 + [51 / 32])
    b1 = np.ones(86)
    return a.reshape(1, 86), np.stack([b0, b1], axis=1)


def test_accurate_hand_case_bar_products():
    A, B = _accurate_case()
    _, _, Abar, Bbar, Cbar = scaling.accurate_log2(
        A, B, constants.p_prime_accu(N20), constants.delta())
    assert Abar.tolist() == [[63] * 85 + [34]]
    assert Bbar[:, 0].tolist() == [63] * 85 + [51]
    assert Bbar[:, 1].tolist() == [32] * 86
    assert Cbar.tolist() == [[339099, 172448]]


def test_accurate_hand_case_exponents_and_rounding_direction():
    """Exponents of the hand case (N = 20), where the rounding directions of
    accurate mode decide the result.

    cbar = 339099 = 2^18 * 1.2935...: log2 = 18.3713470043...; the binary32
    log2 of the mantissa, rounded to nearest, is 0x3EBE2132 = 0.37134701...;
    plus 18 is 18.37134701013..., rounded up 0x4192F885 = 18.371347427...
    (rounded down it would be 0x4192F884).  delta times that is exactly
    9.1856769987...; rounded up 0x4112F889 = 9.185677528..., rounded down
    0x4112F888 = 9.185676574707031, which is exactly P'_accu - 68.
    floor(P'_accu - 9.185677528) = floor(67.99999905) = 67.  Rounding the
    product down (or tilde-log2 down) would give 68: a larger scale than the
    paper's bound allows.  log2 mu_0 = 5 + 67 = 72 (the row maximum of cbar
    is 339099); log2 nu_0 = 5 + 67 = 72 (column 0).

    cbar = 172448 = 2^17 * 1.3157...: tilde-log2 = 0x418B2A9B = 17.3958034...,
    delta times it rounded up 0x410B2A9F = 8.6979055..., and
    floor(77.1856766 - 8.6979055) = floor(68.48777) = 68: log2 nu_1 = 73.

    Then A' = trunc(2^72 a) = 63 * 2^67 (85 times) and 34 * 2^67, B' column 0
    likewise with 51 * 2^67, column 1 = 2^73: C''_00 = 339099 * 2^134 and
    C''_01 = 5389 * 2^140, both below P/2 = 2^154.37, and C is the exact
    product: 339099 / 1024 and 5389 / 32."""
    pa, d = constants.p_prime_accu(N20), constants.delta()
    A, B = _accurate_case()
    emu, enu, _, _, _ = scaling.accurate_log2(A, B, pa, d)
    assert emu == [72]
    assert enu == [72, 73]
    assert float(scaling.tilde_log2_ru(339099)) == _f32("4192f885")
    assert float(scaling.tilde_log2_ru(172448)) == _f32("418b2a9b")
    r = ozaki2.gemm(A, B, N20, ozaki2.ACCURATE)
    assert r["e_rows"] == [72] and r["e_cols"] == [72, 73]
    assert int(r["Cpp"][0, 0]) == 339099 << 134
    assert int(r["Cpp"][0, 1]) == 5389 << 140
    assert float(r["C"][0, 0]) == 339099 / 1024
    assert float(r["C"][0, 1]) == 5389 / 32


def test_accurate_rounding_boundary_is_exact_in_binary32():
    """The boundary the hand case sits on: P'_accu - 68 is the binary32
    0x4112F888 exactly, and delta * tilde-log2(339099) lies strictly between
    it and the next binary32 value 0x4112F889 (so the rounding direction
    decides the floor)."""
    lo, hi = _f32("4112f888"), _f32("4112f889")
    assert _f32("429a5f11") - 68 == lo
    t = _f32("4192f885")
    prod_num = (0.5 + 3 * 2.0 ** -24)
    # exact product of two binary32 values fits binary64 (24 + 24 bits)
    exact = prod_num * t
    assert lo < exact < hi
    assert math.floor(_f32("429a5f11") - hi) == 67
    assert math.floor(_f32("429a5f11") - lo) == 68


def _edge_rows(rng, rows, cols):
    out = np.empty((rows, cols))
    for i in range(rows):
        kind = i % 4
        if kind == 0:
            out[i] = rng.standard_normal(cols) * np.exp(2 * rng.standard_normal(cols))
        elif kind == 1:
            out[i] = rng.standard_normal(cols) * 2.0 ** -1060     # scaled entries below normal
            out[i, 0] = 2.0 ** -1000
        elif kind == 2:
            out[i] = rng.choice([0.0, 1.0, -3.0, 2.0 ** 500, 5e-324], cols)
        else:
            out[i] = 0.0
    return out


def test_accurate_bars_array_form_equals_scalar_form():
    """The array form of accurate mode's first step (used for checks at full
    size) gives the same exponents and bar matrices as ``accurate_log2``'s
    entry-by-entry rational arithmetic, including zero rows, entries that
    scale below the normal range and subnormal inputs."""
    rng = np.random.default_rng(3)
    A = _edge_rows(rng, 12, 9)
    B = _edge_rows(rng, 8, 9).T.copy()          # columns carry the edge cases
    emu, enu, Abar, Bbar, _ = scaling.accurate_log2(
        A, B, constants.p_prime_accu(14), constants.delta())
    e1, nz, bar = scaling.accurate_bars(A)
    assert (bar == Abar).all()
    assert (bar.max() <= 64) and (bar.min() >= 0)
    e1b, nzb, barb = scaling.accurate_bars(B.T)
    assert (barb.T == Bbar).all()
    # exponents: recombine through the shared final step
    Cbar = Abar @ Bbar
    pa, d = constants.p_prime_accu(14), constants.delta()
    got = [scaling.accurate_final_exponent(int(e1[i]) if nz[i] else None, int(Cbar[i].max()), pa, d)
           for i in range(A.shape[0])]
    assert got == emu
    got = [scaling.accurate_final_exponent(int(e1b[j]) if nzb[j] else None, int(Cbar[:, j].max()),
                                           pa, d) for j in range(B.shape[1])]
    assert got == enu
