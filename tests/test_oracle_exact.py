"""Pins for the exact mode of the oracle (CPU only): an optional variant of
Algorithm 2, not in the paper, that takes the exact maximal exponent of the
Cauchy-Schwarz condition of Section 4 and falls back to entries scaled by
2**-600 where the squared norm overflows binary64.

Pinned against Algorithm 2 (an independent float-log computation that must
land on the same exponent or one below), exact scale invariance at every
power of two (Algorithm 2 loses it at 2**+-300), the all-ones closed form,
the CRT bound with its maximality, and for huge rows the identity with the
same problem scaled down by 2**600 (a different branch of the code) plus the
a-priori error bound against the exact product."""
import math
import random
from fractions import Fraction

import numpy as np
import pytest

from oracle import complex as zref, constants, fp, ozaki2, reference, scaling
from paper_2606_29129_amd import inputs


def _random_S(rng, lo=-120, hi=120):
    return float(rng.uniform(1, 2)) * 2.0 ** rng.randint(lo, hi)


@pytest.mark.parametrize("N", [2, 5, 9, 14, 17, 20])
def test_algorithm2_is_emax_or_one_below(N):
    """Algorithm 2 (binary32 log and slack) returns the exact maximum or one
    less wherever its w is exact (|P'_prop - s/2| < 64): equal on random S,
    one less for S just below a boundary of the condition, S = RD((P - 1)
    2**-(2e+1)) (where e_max = e exactly and the slack costs the bit)."""
    _, P, _, _ = constants.step1(N)
    pp = constants.p_prime_prop(N)
    rng = random.Random(N)
    for _ in range(200):
        S = _random_S(rng)
        assert scaling.alg2_log2_mu(S, pp) == scaling.emax_log2_mu(S, P), S
    below = 0
    for _ in range(50):
        e = rng.randint(-60, 60)
        S = float(fp.round_rational(Fraction(P - 1) / fp._pow2(2 * e + 1), fp.BINARY64, "RD"))
        assert scaling.emax_log2_mu(S, P) == e
        a2 = scaling.alg2_log2_mu(S, pp)
        assert a2 in (e - 1, e)
        below += a2 == e - 1
    assert below > 0


@pytest.mark.parametrize("N", [3, 14, 20])
def test_emax_is_maximal_for_the_condition(N):
    """2**(2e+1) S <= P - 1 holds at e_max and fails at e_max + 1, checked
    with Python integers on S's integer significand."""
    _, P, _, _ = constants.step1(N)
    rng = random.Random(7 * N)
    for _ in range(200):
        S = _random_S(rng, -1000, 1000)
        e = scaling.emax_log2_mu(S, P)
        n, d = S.as_integer_ratio()        # S = n / d, d a power of two
        assert (n << (2 * e + 1) if 2 * e + 1 >= 0 else n) * (1 if 2 * e + 1 >= 0 else 1) \
            <= (P - 1) * d * (1 if 2 * e + 1 >= 0 else 2 ** -(2 * e + 1))
        assert (n << (2 * e + 3) if 2 * e + 3 >= 0 else n) * (1 if 2 * e + 3 >= 0 else 1) \
            > (P - 1) * d * (1 if 2 * e + 3 >= 0 else 2 ** -(2 * e + 3))


def test_emax_is_exactly_scale_invariant_where_algorithm2_is_not():
    """e_max(4**s S) = e_max(S) - s for every s (the theorem of Section 4,
    exactly); Algorithm 2 breaks it at 2**+-300 on the witness of its w
    rounding."""
    N = 14
    _, P, _, _ = constants.step1(N)
    pp = constants.p_prime_prop(N)
    rng = random.Random(3)
    for _ in range(100):
        S = _random_S(rng, -200, 200)
        e0 = scaling.emax_log2_mu(S, P)
        for s in (-300, -150, -1, 1, 77, 300):
            assert scaling.emax_log2_mu(S * 4.0 ** s, P) == e0 - s
    W = float.fromhex("0x1.1e3f12b23acd6p-3")
    assert scaling.alg2_log2_mu(W * 4.0 ** 300, pp) != scaling.alg2_log2_mu(W, pp) - 300
    assert scaling.emax_log2_mu(W * 4.0 ** 300, P) == scaling.emax_log2_mu(W, P) - 300


@pytest.mark.parametrize("k", [1024, 16384])
def test_all_ones_closed_form(k):
    """A = B = 2**s J: S = k 4**s exactly, so e_max = floor((L - 1 - log2 k)
    / 2) - s with L = floor(log2(P - 1)); the product k 4**s is recovered
    exactly for every s, including 2**+-300; and A = 2**600 J (squares
    overflow, the fallback branch) times B = 2**-600 J (squares underflow)
    gives C = k exactly."""
    N = 20
    _, P, _, _ = constants.step1(N)
    L = (P - 1).bit_length() - 1
    lk = k.bit_length() - 1
    for s in (-300, -10, -2, 0, 5, 300):
        A, B = inputs.ones_problem(1, 1, k, s)
        r = ozaki2.gemm(A, B, N, ozaki2.EXACT)
        expect = (L - 1 - lk) // 2 - s
        assert r["e_rows"] == [expect] and r["e_cols"] == [expect], s
        assert r["C"][0, 0] == k * 4.0 ** s
    A = np.full((1, k), 2.0 ** 600)
    B = np.full((k, 1), 2.0 ** -600)
    r = ozaki2.gemm(A, B, N, ozaki2.EXACT)
    assert r["e_rows"] == [(L - 1 - lk) // 2 - 600]
    assert r["C"][0, 0] == float(k)


@pytest.mark.parametrize("N", [8, 14, 20])
def test_crt_bound_holds_and_is_nearly_tight(N):
    """2 ||a'|| ||b'|| <= P - 1 (as 4 ||a'||^2 ||b'||^2 <= (P - 1)^2 in
    integers) on random inputs, and the exact mode's integers are never
    narrower than Algorithm 2's (one bit wider where e_max = e_alg2 + 1)."""
    _, P, _, _ = constants.step1(N)
    A, B = inputs.problem(6, 5, 70, 2.0, seed=N)
    rx = ozaki2.gemm(A, B, N, ozaki2.EXACT)
    rr = ozaki2.gemm(A, B, N, ozaki2.REVISED)
    na = [sum(int(x) ** 2 for x in rx["Aint"][i]) for i in range(6)]
    nb = [sum(int(x) ** 2 for x in rx["Bint"][:, j]) for j in range(5)]
    assert 4 * max(na) * max(nb) <= (P - 1) ** 2
    d = [a - b for a, b in zip(rx["e_rows"] + rx["e_cols"], rr["e_rows"] + rr["e_cols"])]
    assert set(d) <= {0, 1}
    ex = ozaki2.exact_product(rx["Aint"], rx["Bint"])
    assert (rx["Cpp"] == ex).all()


def test_huge_rows_equal_the_problem_scaled_down():
    """Rows and columns beyond 1e154 (squared norms overflow) go through the
    fallback; the result equals 2**600 (resp. 2**300 per side) times the exact
    mode's result on the inputs scaled down by 2**600 -- which runs the
    ordinary branch -- bit for bit, and meets the a-priori error bound."""
    N = 16
    A, B = inputs.problem(5, 4, 40, 1.0, seed=11)
    A[1] *= 2.0 ** 700
    A[3, ::2] *= 2.0 ** 900           # mixed magnitudes in one row
    B[:, 2] *= 2.0 ** 600
    r = ozaki2.gemm(A, B, N, ozaki2.EXACT)
    As, Bs = A.copy(), B.copy()
    As[1] *= 2.0 ** -600
    As[3] *= 2.0 ** -600
    Bs[:, 2] *= 2.0 ** -600
    rs = ozaki2.gemm(As, Bs, N, ozaki2.EXACT)
    assert r["e_rows"][1] == rs["e_rows"][1] - 600 and r["e_rows"][3] == rs["e_rows"][3] - 600
    assert r["e_cols"][2] == rs["e_cols"][2] - 600
    for i in range(5):
        for j in range(4):
            sh = 600 * ((i in (1, 3)) + (j == 2))
            want = fp.round_dyadic(int(rs["Cpp"][i, j]),
                                   -(rs["e_rows"][i] + rs["e_cols"][j]) + sh)
            assert r["C"][i, j] == want or (math.isinf(r["C"][i, j]) and math.isinf(want))
    k = A.shape[1]
    for i in range(5):
        for j in range(4):
            e, f = r["e_rows"][i], r["e_cols"][j]
            c = r["C"][i, j]
            if not math.isfinite(c):
                continue
            exact = reference.exact_dot(A[i, :], B[:, j])
            bound = (abs(Fraction(c)) * Fraction(1, 2**53)
                     + fp._pow2(-f) * sum(Fraction(abs(float(x))) for x in A[i, :])
                     + fp._pow2(-e) * sum(Fraction(abs(float(x))) for x in B[:, j])
                     + k * fp._pow2(-(e + f)))
            assert abs(Fraction(c) - exact) <= bound
    # the revised mode cannot scale these rows
    with pytest.raises(OverflowError):
        ozaki2.gemm(A, B, N, ozaki2.REVISED)


def test_rescaled_norm_rounds_tiny_entries_up():
    """In the fallback, entries that underflow after the 2**-600 scaling count
    as the smallest subnormal (rounded up), keeping S an upper bound."""
    v = np.array([2.0 ** 700, 2.0 ** -1000, -(2.0 ** -1074)])
    S = scaling.norm_sq_ru_rescaled(v)
    exact = sum(Fraction(float(x)) ** 2 for x in v) / Fraction(4) ** 600
    assert Fraction(S) >= exact
    assert S == fp.ru_add(fp.ru_add(4.0 ** 100, fp.ru_square(2.0 ** -1074)),
                          fp.ru_square(2.0 ** -1074))


def test_non_finite_entries_stay_non_finite():
    _, P, _, _ = constants.step1(14)
    for bad in (np.inf, -np.inf, np.nan):
        with pytest.raises(OverflowError):
            scaling.exact_mode_log2_mu(np.array([1.0, bad, 2.0]), P)


def test_complex_exact_mode_reduces_to_real():
    """For k <= 32 the complex exact mode on real inputs equals the real one,
    also through the overflow fallback."""
    A, B = inputs.problem(3, 4, 20, 1.0, seed=2)
    A[0] *= 2.0 ** 650
    D = ozaki2.gemm(A, B, 12, ozaki2.EXACT)["C"]
    C = zref.gemm(A + 0j, B + 0j, 12, ozaki2.EXACT)["C"]
    assert np.array_equal(C.real, D) and not C.imag.any()
