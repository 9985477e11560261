"""Whole-path pins for the oracle (CPU only): the paper's all-ones analysis,
brute force on tiny inputs, exact integer inputs, scale invariance and an
a-priori error bound."""
import math
import random
from fractions import Fraction

import numpy as np
import pytest

from oracle import constants, fp, ozaki2, reference
from paper_2606_29129_amd import inputs

N20 = 20


@pytest.mark.parametrize("k", [1024, 16384])
def test_all_ones_revised_is_exact_for_every_alpha(k):
    """Section 4 / Section 3.1 example: with the proposed scaling the
    all-ones product A = B = alpha J is recovered exactly (C = k alpha**2)
    for every alpha = 2**s, s = -10..10, N = 20, and A'B' stays below P/2."""
    _, P, _, _ = constants.step1(N20)
    for s in range(-10, 11):
        A, B = inputs.ones_problem(1, 1, k, s)
        r = ozaki2.gemm(A, B, N20, ozaki2.REVISED)
        ex = ozaki2.exact_product(r["Aint"], r["Bint"])
        assert all(int(x) < P // 2 for x in ex.ravel())
        assert (r["Cpp"] == ex).all()
        assert (r["C"] == k * 4.0 ** s).all()


@pytest.mark.parametrize("k", [1024, 16384])
def test_all_ones_original_fast_fails_exactly_below_quarter(k):
    """Section 3.1: with the original fast mode (Algorithm 1) and N = 20 the
    all-ones product A'B' exceeds P/2 -- CRT recovery fails -- exactly in the
    region alpha <= 2**-2, for k = 1024 and k = 16384."""
    _, P, _, _ = constants.step1(N20)
    for s in range(-10, 11):
        A, B = inputs.ones_problem(1, 1, k, s)
        r = ozaki2.gemm(A, B, N20, ozaki2.ORIGINAL)
        ex = ozaki2.exact_product(r["Aint"], r["Bint"])
        fails = int(ex[0, 0]) >= P // 2
        assert fails == (s <= -2), s
        assert bool((r["Cpp"] != ex).any()) == fails
        assert bool((r["C"] == k * 4.0 ** s).all()) == (not fails)


def _edge_matrix(rng, rows, cols):
    vals = []
    for _ in range(rows * cols):
        kind = rng.random()
        if kind < 0.15:
            v = 0.0
        elif kind < 0.3:
            v = rng.choice([-1, 1]) * 2.0 ** rng.randint(-40, 40)
        elif kind < 0.4:
            v = rng.uniform(-1, 1) * 2.0 ** rng.randint(-1000, 500)
        elif kind < 0.45:
            v = rng.randint(1, 2**52) * 2.0 ** -1074          # subnormal
        else:
            v = rng.uniform(-1, 1) * math.exp(3 * rng.gauss(0, 1))
        vals.append(v)
    return np.array(vals, dtype=np.float64).reshape(rows, cols)


@pytest.mark.parametrize("N", [2, 3, 7, 14, 16, 17, 20])
@pytest.mark.parametrize("mode", [ozaki2.REVISED, ozaki2.ACCURATE])
def test_brute_force_tiny(N, mode):
    """Tiny random shapes with zeros, powers of two, huge/tiny and subnormal
    entries: Step 3 recovers A'B' exactly (Theorem 1 + eq. os2-condition),
    the condition 2 sum|a'||b'| < P holds (Section 4: CRT never fails), and
    Step 4 is the correctly rounded A'B' 2**(-e-f), checked with CPython's
    correctly rounded integer division."""
    _, P, _, _ = constants.step1(N)
    rng = random.Random(1000 * N + mode)
    for trial in range(12):
        m, n, k = rng.randint(1, 5), rng.randint(1, 5), rng.randint(1, 6)
        A = _edge_matrix(rng, m, k)
        B = _edge_matrix(rng, k, n)
        r = ozaki2.gemm(A, B, N, mode)
        ex = ozaki2.exact_product(r["Aint"], r["Bint"])
        assert (r["Cpp"] == ex).all()
        assert ozaki2.crt_condition_lhs(r["Aint"], r["Bint"]) < P
        for i in range(m):
            for j in range(n):
                E = r["e_rows"][i] + r["e_cols"][j]
                x = int(ex[i, j])
                try:
                    ref = x / (1 << E) if E >= 0 else float(x << -E)
                except OverflowError:
                    ref = math.inf if x > 0 else -math.inf
                assert r["C"][i, j] == ref


def test_residues_and_products_brute_force():
    """Residues are congruent to the integers and lie in the INT8 range; the
    per-modulus products equal the plain integer dot products."""
    A, B = inputs.problem(5, 4, 9, 2.0, seed=11)
    r = ozaki2.gemm(A, B, 20)
    p = constants.moduli(20)
    for t, pt in enumerate(p):
        RA, RB, G = r["RA"][t], r["RB"][t], r["G"][t]
        assert RA.min() >= -128 and RA.max() <= 127
        for i in range(5):
            for h in range(9):
                assert (int(r["Aint"][i, h]) - int(RA[i, h])) % pt == 0
                if pt != 256:
                    assert abs(int(RA[i, h])) <= (pt - 1) // 2
        for i in range(5):
            for j in range(4):
                assert int(G[i, j]) == sum(int(RA[i, h]) * int(RB[h, j]) for h in range(9))


@pytest.mark.parametrize("N", [8, 14, 20])
def test_integer_inputs_give_the_exact_product(N):
    """Integer entries in [-8, 8]: mu, nu >= 1, so the truncation loses
    nothing and C equals the exact integer product AB."""
    rng = np.random.default_rng(N)
    A = rng.integers(-8, 9, (7, 33)).astype(np.float64)
    B = rng.integers(-8, 9, (33, 6)).astype(np.float64)
    C = ozaki2.dgemm(A, B, N)
    exact = A.astype(np.int64) @ B.astype(np.int64)
    assert (C == exact.astype(np.float64)).all()


def test_scale_invariance_powers_of_two():
    """Section 4: A -> 2**s A leaves A' unchanged and scales C by exactly
    2**s (s = +-300) for every row whose exponent Algorithm 2 shifts exactly
    (all rows of this seeded input; the binary32 rounding of w can lower an
    exponent by one at such scales, see test_oracle_scaling); the original
    fast mode changes A'."""
    A, B = inputs.problem(6, 5, 40, 1.0, seed=3)
    r0 = ozaki2.gemm(A, B, 14)
    for s in (300, -300):
        r1 = ozaki2.gemm(A * 2.0 ** s, B, 14)
        assert (r1["Aint"] == r0["Aint"]).all()
        assert [e + s for e in r1["e_rows"]] == r0["e_rows"]
        assert (r1["C"] == r0["C"] * 2.0 ** s).all()
    f0 = ozaki2.gemm(A, B, 14, ozaki2.ORIGINAL)
    f1 = ozaki2.gemm(A * 2.0 ** 30, B, 14, ozaki2.ORIGINAL)
    assert not (f1["Aint"] == f0["Aint"]).all()


def test_scale_invariance_general_constant_bit_width():
    """A -> c A with c = 3.7e+-100: the effective bit width of every integer
    row, log2 mu_i + floor(log2 max|a_i|) + 1, moves by at most one."""
    A, B = inputs.problem(8, 3, 64, 2.0, seed=4)

    def widths(M):
        r = ozaki2.gemm(M, B, 14)
        return [r["e_rows"][i] + fp.floor_log2(Fraction(float(np.max(np.abs(M[i]))))) + 1
                for i in range(M.shape[0])]

    w0 = widths(A)
    for c in (3.7e100, 3.7e-100):
        w1 = widths(A * c)
        assert all(abs(a - b) <= 1 for a, b in zip(w0, w1))


@pytest.mark.parametrize("N", [10, 14, 20])
def test_a_priori_error_bound(N):
    """With a' = mu a - theta, |theta| < 1 (truncation) the product obeys
    |C - AB| <= u|C| + 2**-f_j sum|a_ih| + 2**-e_i sum|b_hj| + k 2**-(e_i+f_j)
    entrywise, checked against the exact rational product."""
    A, B = inputs.problem(6, 5, 50, 3.0, seed=N)
    r = ozaki2.gemm(A, B, N)
    k = A.shape[1]
    for i in range(6):
        for j in range(5):
            e, f = r["e_rows"][i], r["e_cols"][j]
            exact = reference.exact_dot(A[i, :], B[:, j])
            c = Fraction(float(r["C"][i, j]))
            bound = (abs(c) * Fraction(1, 2**53)
                     + fp._pow2(-f) * sum(Fraction(abs(float(x))) for x in A[i, :])
                     + fp._pow2(-e) * sum(Fraction(abs(float(x))) for x in B[:, j])
                     + k * fp._pow2(-(e + f)))
            assert abs(c - exact) <= bound


def test_accuracy_improves_with_N():
    """More moduli give larger integers and a smaller error (Section 5.1)."""
    A, B = inputs.problem(8, 8, 48, 1.0, seed=12)
    errs = [reference.errors(ozaki2.dgemm(A, B, N), A, B)["max_comp"] for N in (8, 12, 16, 20)]
    assert errs[0] > errs[1] > errs[2] >= errs[3]
    assert errs[3] < 2.0 ** -50


def test_sampled_entry_matches_full_path():
    A, B = inputs.problem(5, 6, 70, 1.5, seed=8)
    r = ozaki2.gemm(A, B, 16)
    for i, j in ((0, 0), (4, 5), (2, 3)):
        c, G, cpp = ozaki2.entry(A[i, :], B[:, j], r["e_rows"][i], r["e_cols"][j], 16)
        assert c == r["C"][i, j] and cpp == r["Cpp"][i, j]
        assert G == [int(g[i, j]) for g in r["G"]]


def test_sgemm_rounds_once_to_binary32():
    A, B = inputs.problem(4, 4, 20, 1.0, seed=2)
    A32, B32 = A.astype(np.float32), B.astype(np.float32)
    r = ozaki2.gemm(A32.astype(np.float64), B32.astype(np.float64), 9, out_fmt=fp.BINARY32)
    C = ozaki2.sgemm(A, B, 9)
    assert C.dtype == np.float32
    for i in range(4):
        for j in range(4):
            E = r["e_rows"][i] + r["e_cols"][j]
            ref = fp.round_rational(Fraction(int(r["Cpp"][i, j])) * fp._pow2(-E), fp.BINARY32, "RN")
            assert float(C[i, j]) == float(ref)


def test_vectorised_residues_equal_the_definition():
    """The array form of the residues equals rmod(x, p) (odd p, Section 2.1)
    and the low-byte reading (p = 256) entry by entry, for integers up to
    2**80 of both signs."""
    rng = random.Random(21)
    xs = [rng.randint(-2**80, 2**80) for _ in range(400)] + list(range(-600, 600))
    X = np.array(xs, dtype=object)
    for p in constants.MODULI:
        r = ozaki2.residues(X, p)
        for x, v in zip(xs, r):
            if p == 256:
                assert v == x - 256 * ((x + 128) // 256)
            else:
                assert v == x - p * ozaki2.round_half_even_div(x, p)
