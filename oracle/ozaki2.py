"""Ozaki scheme II, Steps 2-4 of Section 2.2 (test infrastructure only).

    Step 2   a'_ih = trunc(mu_i a_ih),  b'_hj = trunc(nu_j b_hj)
    Step 3   C'  = sum_t P_t q_t * rmod(A', p_t) rmod(B', p_t)
             C'' = rmod(C', P)
    Step 4   C   = diag(mu)^-1 C'' diag(nu)^-1

The scale factors are powers of two and are carried as integer exponents
(mu_i = 2**e_i), so Step 2 and Step 4 are exact scalings followed by one
truncation or one rounding.  All integer work uses Python integers (any
width); the N residue products use numpy int64 matrix products, which are
exact here (|entries| <= 128 and k <= 2**17 keep every partial sum below
2**32).  Step 4 rounds the exact rational C''_ij * 2**(-e_i - f_j) once, to
nearest even, in the output format.

Reading for the modulus 256 (Section 2.2 defines rmod with ties to even, which
gives +128 for x = 128 mod 256, a value INT8 cannot hold): the residue for
p = 256 is the two's-complement low byte of x, i.e. the representative in
[-128, 127].  It is congruent to rmod(x, 256) modulo 256, so C'' is unchanged.
For odd p there are no ties and the residue is rmod(x, p) in
[-(p-1)/2, (p-1)/2].
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

from . import constants, fp, scaling

REVISED, ORIGINAL, ACCURATE, EXACT = 0, 1, 2, 3


def round_half_even_div(x: int, P: int) -> int:
    """round(x / P) with ties to even, for integers (P > 0)."""
    q, r = divmod(x, P)          # x = q P + r, 0 <= r < P
    if 2 * r > P or (2 * r == P and q % 2 == 1):
        q += 1
    return q


def rmod(x: int, P: int) -> int:
    """rmod(x, P) = x - P round(x / P) (Section 2.1)."""
    return x - P * round_half_even_div(x, P)


def residue(x: int, p: int) -> int:
    """The INT8 residue of integer x for modulus p used in Step 3."""
    if p == 256:
        return ((x + 128) % 256) - 128
    return rmod(x, p)


def scaled_integer(a: float, e: int) -> int:
    """trunc(a * 2**e) for a binary64 value a (Step 2).

    a = n * 2**ea exactly, so a * 2**e = n * 2**(ea + e); truncation toward
    zero drops the fractional bits of |n| * 2**(ea + e)."""
    n, ea = fp.int_exp(a)
    sh = ea + e
    mag = abs(n) << sh if sh >= 0 else abs(n) >> -sh
    return -mag if n < 0 else mag


def step2(A, e_rows):
    """A' = trunc(diag(2**e) A) as a numpy object array of Python ints."""
    A = np.asarray(A, dtype=np.float64)
    out = np.empty(A.shape, dtype=object)
    for i in range(A.shape[0]):
        for h in range(A.shape[1]):
            out[i, h] = scaled_integer(float(A[i, h]), e_rows[i])
    return out


def residues(Aint, p: int) -> np.ndarray:
    """Elementwise INT8 residues of an integer matrix (object array).

    Vectorised form of ``residue``: for odd p, x - p round(x/p) equals
    ((x + h) mod p) - h with h = (p-1)/2, because x/p is never a half-integer
    and floor((x + h)/p) = floor(x/p + 1/2) for every integer x; for p = 256
    it is the low byte ((x + 128) mod 256) - 128."""
    X = np.asarray(Aint, dtype=object)
    h = 128 if p == 256 else (p - 1) // 2
    return (((X + h) % p) - h).astype(np.int64)


def step3(Aint, Bint, N: int):
    """Step 3: residue products G_t = rmod(A',p_t) rmod(B',p_t) and C''.

    Returns (RA list, RB list, G list of int64 arrays, C' and C'' as object
    arrays).
    """
    p, P, Pi, qi = constants.step1(N)
    RA = [residues(Aint, pt) for pt in p]
    RB = [residues(Bint, pt) for pt in p]
    G = [ra @ rb for ra, rb in zip(RA, RB)]
    m, n = G[0].shape if G else (0, 0)
    Cp = np.zeros((m, n), dtype=object)
    for t in range(N):
        Cp = Cp + (Pi[t] * qi[t]) * G[t].astype(object)
    Cpp = np.empty((m, n), dtype=object)
    for i in range(m):
        for j in range(n):
            Cpp[i, j] = rmod(int(Cp[i, j]), P)
    return RA, RB, G, Cp, Cpp


def step4(Cpp, e_rows, e_cols, fmt=fp.BINARY64):
    """Step 4: C_ij = RN(C''_ij * 2**(-e_i - f_j)) in the output format."""
    m, n = Cpp.shape
    dt = np.float64 if fmt == fp.BINARY64 else np.float32
    C = np.empty((m, n), dtype=dt)
    for i in range(m):
        for j in range(n):
            C[i, j] = fp.round_dyadic(int(Cpp[i, j]), -(e_rows[i] + e_cols[j]), fmt, "RN")
    return C


def scale_exponents(A, B, N: int, mode: int = REVISED):
    """Row exponents log2(mu) and column exponents log2(nu) for a mode,
    with the squared norms they came from (None for accurate mode)."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    if mode == ACCURATE:
        emu, enu, _, _, _ = scaling.accurate_log2(
            A, B, constants.p_prime_accu(N), constants.delta())
        return emu, enu, None, None
    if mode == EXACT:
        SA = SB = None
    else:
        SA = [scaling.norm_sq_ru(A[i, :]) for i in range(A.shape[0])]
        SB = [scaling.norm_sq_ru(B[:, j]) for j in range(B.shape[1])]
    if mode == REVISED:
        pp = constants.p_prime_prop(N)
        emu = [scaling.alg2_log2_mu(S, pp) for S in SA]
        enu = [scaling.alg2_log2_mu(S, pp) for S in SB]
    elif mode == EXACT:
        # squared norms recomputed per vector (the overflow fallback may
        # replace them): the norms returned are the ones the exponents used
        _, P, _, _ = constants.step1(N)
        ra = [scaling.exact_mode_log2_mu(A[i, :], P) for i in range(A.shape[0])]
        rb = [scaling.exact_mode_log2_mu(B[:, j], P) for j in range(B.shape[1])]
        emu, SA = [e for e, _ in ra], [S for _, S in ra]
        enu, SB = [e for e, _ in rb], [S for _, S in rb]
    elif mode == ORIGINAL:
        pf, d = constants.p_prime_fast(N), constants.delta()
        amaxA = [float(np.max(np.abs(A[i, :]))) for i in range(A.shape[0])]
        amaxB = [float(np.max(np.abs(B[:, j]))) for j in range(B.shape[1])]
        emu = [scaling.alg1_log2_mu(S, a, pf, d) for S, a in zip(SA, amaxA)]
        enu = [scaling.alg1_log2_mu(S, b, pf, d) for S, b in zip(SB, amaxB)]
    else:
        raise ValueError(f"unknown mode {mode}")
    return emu, enu, SA, SB


def gemm(A, B, N: int, mode: int = REVISED, out_fmt=fp.BINARY64):
    """The whole emulated product C ~ A B with every intermediate.

    A is m x k and B is k x n (row-major numpy arrays of binary64 or binary32
    values).  Returns a dict with keys SA, SB (squared norms), e_rows, e_cols
    (log2 mu, log2 nu), Aint, Bint (A', B'), RA, RB (residue matrices per
    modulus), G (INT32 products per modulus), Cp, Cpp (C', C'') and C.
    """
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    emu, enu, SA, SB = scale_exponents(A, B, N, mode)
    Aint = step2(A, emu)
    Bint = step2(B.T, enu).T
    RA, RB, G, Cp, Cpp = step3(Aint, Bint, N)
    C = step4(Cpp, emu, enu, out_fmt)
    return dict(SA=SA, SB=SB, e_rows=emu, e_cols=enu, Aint=Aint, Bint=Bint,
                RA=RA, RB=RB, G=G, Cp=Cp, Cpp=Cpp, C=C)


def dgemm(A, B, N: int, mode: int = REVISED):
    """C ~ A B for binary64 inputs (Section 2.2)."""
    return gemm(A, B, N, mode, fp.BINARY64)["C"]


def sgemm(A, B, N: int, mode: int = REVISED):
    """C ~ A B for binary32 inputs and output (Section 5 evaluates SGEMM with
    the same scheme)."""
    A32 = np.asarray(A, dtype=np.float32)
    B32 = np.asarray(B, dtype=np.float32)
    return gemm(A32.astype(np.float64), B32.astype(np.float64), N, mode,
                fp.BINARY32)["C"]


def exact_product(Aint, Bint):
    """A'B' with Python integers (no CRT): what Step 3 must recover."""
    m, k = Aint.shape
    n = Bint.shape[1]
    out = np.empty((m, n), dtype=object)
    for i in range(m):
        for j in range(n):
            out[i, j] = sum(int(Aint[i, h]) * int(Bint[h, j]) for h in range(k))
    return out


def crt_condition_lhs(Aint, Bint):
    """max_ij 2 * sum_h |a'_ih| |b'_hj| (left side of eq. os2-condition)."""
    absA = np.vectorize(lambda x: abs(int(x)), otypes=[object])(Aint)
    absB = np.vectorize(lambda x: abs(int(x)), otypes=[object])(Bint)
    best = 0
    m, k = Aint.shape
    n = Bint.shape[1]
    for i in range(m):
        for j in range(n):
            best = max(best, 2 * sum(absA[i, h] * absB[h, j] for h in range(k)))
    return best


# ---------------------------------------------------------------------------
# Sampled entries: the same steps for one output C_ij at any size
# ---------------------------------------------------------------------------

def entry(a_row, b_col, e_i: int, f_j: int, N: int, out_fmt=fp.BINARY64):
    """C_ij from row i of A and column j of B and their exponents.

    Runs Steps 2-4 for one output entry; used to check large problems on
    sampled entries.  Returns (C_ij, G_t list, C''_ij).
    """
    p, P, Pi, qi = constants.step1(N)
    ai = [scaled_integer(float(x), e_i) for x in np.asarray(a_row, np.float64)]
    bj = [scaled_integer(float(x), f_j) for x in np.asarray(b_col, np.float64)]
    G = []
    Cp = 0
    for t, pt in enumerate(p):
        g = sum(residue(x, pt) * residue(y, pt) for x, y in zip(ai, bj))
        G.append(g)
        Cp += Pi[t] * qi[t] * g
    Cpp = rmod(Cp, P)
    C = fp.round_dyadic(Cpp, -(e_i + f_j), out_fmt, "RN")
    return C, G, Cpp
