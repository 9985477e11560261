"""Pins of the FP8 (E4M3) engine oracle: the E4M3 codes against torch's own
float8_e4m3fn conversion (a library routine written independently of the
oracle), the digit split by brute force over every residue, the binary32
block bound in closed form and by float32 accumulation, and the engine
product against the plain integer product."""
import numpy as np
import pytest

from oracle import constants, fp8, ozaki2 as ref
from paper_2606_29129_amd import inputs

torch = pytest.importorskip("torch")


def _torch_codes(values):
    t = torch.tensor([float(v) for v in values], dtype=torch.float32)
    return [int(c) for c in t.to(torch.float8_e4m3fn).view(torch.uint8)]


def test_codes_of_digits_match_torch_e4m3fn():
    vals = list(range(-16, 17)) + [16 * h for h in range(-8, 9)] + [448, -448, 96, 112, 240]
    assert [fp8.e4m3_encode(v) for v in vals] == _torch_codes(vals)


def test_decode_matches_torch_on_every_code():
    codes = [c for c in range(256) if c not in (0x7F, 0xFF)]
    t = torch.tensor(codes, dtype=torch.uint8).view(torch.float8_e4m3fn).to(torch.float64)
    assert [float(fp8.e4m3_decode(c)) for c in codes] == t.tolist()
    for c in codes:       # every finite code round-trips where the value is an integer
        v = fp8.e4m3_decode(c)
        if v.denominator == 1 and v != 0:
            assert fp8.e4m3_encode(int(v)) == c


def test_inexact_or_out_of_range_integers_are_refused():
    for v in (17, 33, 449, 512, -130, 1000):
        with pytest.raises(ValueError):
            fp8.e4m3_encode(v)


def test_digits_of_every_residue():
    worst = 0
    for r in range(-128, 128):
        h, l = fp8.digits(r)
        assert r == 16 * h + l and -8 <= l <= 7 and -8 <= h <= 8
        worst = max(worst, 16 * abs(h) + abs(l))
        # both engine operands are exact E4M3 values
        assert fp8.e4m3_decode(fp8.e4m3_encode(16 * h)) == 16 * h
        assert fp8.e4m3_decode(fp8.e4m3_encode(l)) == l
    assert worst == 136 and fp8.digits(120) == (8, -8) and fp8.digits(-120) == (-7, -8)
    assert fp8.digits(-128) == (-8, 0) and fp8.digits(127) == (8, -1)
    assert fp8.BLOCK_BOUND == 512 * 136 ** 2 < 2 ** 24


def test_block_sums_are_exact_in_binary32():
    """Float32 accumulation, in the given and in shuffled orders, of the four
    digit terms over a block of 512 indices: residues at the digit maximum
    (r = 120, whose digits 8 and -8 reach the bound 136) and their negations and random residues."""
    rng = np.random.default_rng(3)
    cases = [np.full(512, 120), np.full(512, -120), rng.integers(-128, 128, 512)]
    for ra in cases:
        rb = np.sign(ra) * 120 if ra is not cases[2] else rng.integers(-128, 128, 512)
        terms = []
        for x, y in zip(ra, rb):
            hx, lx = fp8.digits(int(x))
            hy, ly = fp8.digits(int(y))
            terms += [16 * hx * 16 * hy, 16 * hx * ly, lx * 16 * hy, lx * ly]
        terms = np.array(terms, dtype=np.int64)
        exact = int((ra * rb).sum())
        assert int(terms.sum()) == exact
        for order in (np.arange(terms.size), rng.permutation(terms.size)):
            acc = np.float32(0.0)
            for v in terms[order]:
                acc = np.float32(acc + np.float32(v))
            assert int(acc) == exact


def test_engine_product_equals_integer_product():
    rng = np.random.default_rng(5)
    for m, k, n in [(3, 1, 2), (17, 1300, 9), (5, 512, 4), (4, 1025, 3)]:
        RA = rng.integers(-128, 128, (m, k))
        RB = rng.integers(-128, 128, (k, n))
        assert np.array_equal(fp8.product(RA, RB), RA @ RB)
    # extremes: every residue at -128 or at 127
    for v in (-128, 127):
        RA = np.full((2, 700), v)
        assert np.array_equal(fp8.product(RA, RA.T), RA @ RA.T)


def test_engine_products_of_a_problem_equal_step3():
    A, B = inputs.problem(20, 15, 600, 1.5, seed=7)
    N = 9
    r = ref.gemm(A, B, N)
    p = constants.moduli(N)
    for t in range(N):
        assert np.array_equal(fp8.product(r["RA"][t], r["RB"][t]), r["G"][t]), p[t]
