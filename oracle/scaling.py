"""Scale exponents log2(mu_i), log2(nu_j) (test infrastructure only).

* ``norm_sq_ru``       the squared 2-norm as an upper bound, every square and
                       addition rounded toward +inf (Algorithms 1 and 2,
                       Section 4)
* ``alg2_log2_mu``     Algorithm 2, the proposed scaling (Section 4)
* ``alg1_log2_mu``     Algorithm 1, the original fast mode (Section 2.3)
* ``accurate_log2``    accurate mode (Section 2.3)
* ``emax_log2_mu``, ``exact_mode_log2_mu``  the exact mode, an optional
                       variant (not in the paper): the exact maximal exponent
                       of the Cauchy-Schwarz condition, with an overflow
                       fallback for huge rows

Every rounding is done exactly on rationals (``oracle.fp``).

Readings taken where the paper leaves a choice open:

* Summation order of the rounded-up sum of squares (not fixed by the paper;
  every order gives an upper bound).  The oracle uses one fixed order,
  ``KC``-element chunks: each chunk's squares are added left to right, then
  the chunk sums are added left to right, every square and every addition
  rounded toward +inf in binary64.  Binary64 (not binary32) is used because
  binary32 squares overflow or underflow for inputs scaled by 2**+-300.
* The binary64 quantity a_norm / 2**s in [1, 2) is converted to binary32 for
  the logarithm by rounding up, which can only make the bound more
  conservative.
* The fast log2 is the correctly rounded binary32 log2 (``fp.log2_rn32``).
* A row (or column) whose squared norm is 0 gets exponent 0: log2(0) is
  undefined, and every entry of the integer row is 0 whatever the scale.
* floor(w - t) in Algorithm 2 is taken on the exact difference of the two
  binary32 values.
* Algorithm 1 scales the log by delta in binary32 rounded up; this is taken
  as two binary32 operations, each rounded up: the sum of the mantissa's log
  and the exponent, then its product with delta.
* Accurate mode: the paper writes mu_i = mu'^{-1}_i * 2^(...), which does not
  satisfy the bound its own proof derives; the proof needs
  mu_i = mu'_i * 2^(...), which is what is implemented.  The binary32
  product delta * tilde-log2(.) is rounded up.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

from . import fp

KC = 64  # chunk length of the fixed summation order


def norm_sq_ru(v, kc: int = KC) -> float:
    """sum(v_h**2) with every square and addition rounded toward +inf.

    Order: chunks of ``kc`` consecutive entries; inside a chunk left to right;
    then the chunk sums left to right.  Returns a binary64 value (inf if the
    sum overflows, NaN if an entry is NaN).
    """
    v = [float(x) for x in np.asarray(v, dtype=np.float64).ravel()]
    partials = []
    for c0 in range(0, len(v), kc):
        part = 0.0
        for a in v[c0:c0 + kc]:
            part = fp.ru_add(part, fp.ru_square(a))
        partials.append(part)
    total = 0.0
    for part in partials:
        total = fp.ru_add(total, part)
    return total


def _split_pow2(S: float):
    """s = floor(log2 S) and the exact ratio S / 2**s in [1, 2)."""
    x = Fraction(S)
    s = fp.floor_log2(x)
    return s, x / fp._pow2(s)


def alg2_log2_mu(S: float, p_prop: Fraction) -> int:
    """Algorithm 2 (Section 4): log2(mu_i) from the rounded-up squared norm.

    The squared norm S is split into its binary exponent s and a mantissa in
    [1, 2).  An upper estimate of the mantissa's half-log (half its binary32
    log2, plus 2 u32 to cover that log's error) is rounded up to binary32;
    P'_prop - s/2 is rounded down to binary32; the exponent is the floor of
    their exact difference, so 2 mu_i**2 S stays at most P - 1.
    """
    if not math.isfinite(S):
        raise OverflowError("non-finite squared norm")
    if S == 0.0:
        return 0
    s, x = _split_pow2(S)
    L = fp.log2_rn32(fp.ru32(x))
    t = fp.ru32(L / 2 + 2 * fp.U32)
    w = fp.rd32(Fraction(p_prop) - Fraction(s, 2))
    return math.floor(w - t)


def alg1_log2_mu(S: float, amax: float, p_fast: Fraction, delta: Fraction) -> int:
    """Algorithm 1 (Section 2.3): log2(mu_i) in the original fast mode.

    An upper estimate of half log2 S (the binary32 log2 of S, rounded up,
    times delta, rounded up again) is clamped from below at 1 and taken from
    P'_fast; the floor of that, less the exponent of the largest entry
    magnitude a_max, is the exponent.
    """
    if not math.isfinite(S):
        raise OverflowError("non-finite squared norm")
    if S == 0.0:
        return 0
    s, x = _split_pow2(S)
    L = fp.log2_rn32(fp.ru32(x))
    t = fp.ru32(Fraction(delta) * fp.ru32(L + s))
    return math.floor(Fraction(p_fast) - max(Fraction(1), t)) - fp.floor_log2(Fraction(amax))


# --- exact mode (not in the paper: an optional variant of Algorithm 2) -------

RESCALE = 600   # exponent shift of the overflow fallback of the exact mode


def emax_log2_mu(S: float, P: int) -> int:
    """Exact maximal exponent: the largest integer e with
    2**(2e+1) * S <= P - 1, by exact rational comparison (S >= 0 finite).

    This is the condition Section 4 derives from Cauchy-Schwarz (the product
    of the two scaled norms at most (P-1)/2) with S an upper bound of the
    squared norm; Algorithm 2 reaches it up to its binary32 slack (it returns
    this value or one less on ordinary data).  A zero vector gets 0.
    """
    if not math.isfinite(S):
        raise OverflowError("non-finite squared norm")
    if S == 0.0:
        return 0
    x = Fraction(S)
    # 2**(2e+1) x <= P - 1 < 2**(LP+1) with x >= 2**Lx gives e <= (LP - Lx) / 2
    e = (fp.floor_log2(Fraction(P - 1)) - fp.floor_log2(x)) // 2
    while fp._pow2(2 * e + 1) * x > P - 1:
        e -= 1
    return e


def norm_sq_ru_rescaled(v, shift: int = -RESCALE) -> float:
    """``norm_sq_ru`` of the entries scaled by 2**shift, each scaled
    magnitude rounded up to binary64 (so tiny entries that underflow still
    count, and the result times 4**-shift bounds the squared norm)."""
    scaled = []
    for a in np.asarray(v, dtype=np.float64).ravel():
        a = abs(float(a))
        if not math.isfinite(a):
            scaled.append(a)
        else:
            scaled.append(float(fp.round_rational(Fraction(a) * fp._pow2(shift),
                                                  fp.BINARY64, "RU")))
    return norm_sq_ru(scaled)


def exact_mode_log2_mu(v, P: int):
    """Exact mode: (log2 mu, the squared norm used).

    The squared norm is ``norm_sq_ru(v)``; where it overflows binary64 (an
    entry or the sum beyond about 1.3e154) the entries are scaled by 2**-600
    first (``norm_sq_ru_rescaled``) and the exponent is shifted back by 600.
    NaN, or an infinite entry, stays non-finite (OverflowError).
    """
    S = norm_sq_ru(v)
    if math.isnan(S):
        raise OverflowError("NaN in the vector")
    if math.isinf(S):
        S2 = norm_sq_ru_rescaled(v)
        if not math.isfinite(S2):
            raise OverflowError("infinite entry")
        return emax_log2_mu(S2, P) - RESCALE, S2
    return emax_log2_mu(S, P), S


def tilde_log2_ru(x: int) -> Fraction:
    """tilde-log2 of eq. (flog2), Section 2.3, for an integer x > 0: the
    binary32 log2 of x's mantissa in [1, 2) plus x's binary exponent, the sum
    rounded up to binary32."""
    e = fp.floor_log2(Fraction(x))
    L = fp.log2_rn32(fp.ru32(Fraction(x) / fp._pow2(e)))
    return fp.ru32(L + e)


def accurate_log2(A, B, p_accu: Fraction, delta: Fraction):
    """Accurate mode (Section 2.3): returns (log2 mu, log2 nu, Abar, Bbar, Cbar).

    mu'_i = 2**(5 - floor(log2 max_h |a_ih|)), Abar = ceil(mu' |A|) <= 64,
    Cbar = Abar Bbar (an exact integer product), and
    log2 mu_i = log2 mu'_i + floor(P'_accu - delta * tilde-log2(max_h cbar_ih)),
    likewise for nu_j with column maxima of Cbar.
    """
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    m, k = A.shape
    n = B.shape[1]

    def first_scale(rows):
        out = []
        for r in rows:
            amax = float(np.max(np.abs(r))) if r.size else 0.0
            out.append(None if amax == 0.0 else 5 - fp.floor_log2(Fraction(amax)))
        return out

    ea = first_scale(A)
    eb = first_scale(B.T)

    def ceil_scaled(x: float, e):
        if e is None:
            return 0
        v = Fraction(abs(x)) * fp._pow2(e)
        return -((-v.numerator) // v.denominator)

    Abar = np.array([[ceil_scaled(A[i, h], ea[i]) for h in range(k)] for i in range(m)],
                    dtype=np.int64).reshape(m, k)
    Bbar = np.array([[ceil_scaled(B[h, j], eb[j]) for j in range(n)] for h in range(k)],
                    dtype=np.int64).reshape(k, n)
    assert Abar.size == 0 or Abar.max() <= 127
    Cbar = Abar @ Bbar

    emu = [accurate_final_exponent(ea[i], int(Cbar[i, :].max()) if n else 0, p_accu, delta)
           for i in range(m)]
    enu = [accurate_final_exponent(eb[j], int(Cbar[:, j].max()) if m else 0, p_accu, delta)
           for j in range(n)]
    return emu, enu, Abar, Bbar, Cbar


def accurate_final_exponent(e1, cmax: int, p_accu: Fraction, delta: Fraction) -> int:
    """Accurate mode's exponent of one row (column) from its first exponent
    e1 = log2 mu'_i (None for a zero vector) and the largest entry cmax of
    its row (column) of Cbar: e1 + floor(P'_accu - delta * tilde-log2(cmax)),
    the product rounded up to binary32.  0 for a zero vector or cmax = 0."""
    if e1 is None or cmax == 0:
        return 0
    corr = fp.ru32(Fraction(delta) * tilde_log2_ru(int(cmax)))
    return e1 + math.floor(Fraction(p_accu) - corr)


def accurate_bars(X):
    """Accurate mode's first step for every row of the binary64 matrix X
    (finite entries), in array form for large checks: returns (e1, nonzero,
    bar) with e1[i] = 5 - floor(log2 max_h |x_ih|) (0 where the row is zero,
    flagged False in ``nonzero``) and bar[i, h] = ceil(2**e1[i] |x_ih|) as
    int64 (<= 64).

    Same values as ``accurate_log2``'s first scale and bar matrices: the
    exponent of max|x| comes from frexp (exact); 2**e1 |x| is exact in
    binary64 except where it falls below the normal range, and there its
    exact value lies in (0, 1), whose ceiling is 1 -- so a positive entry
    that scales to a (rounded) subnormal or to zero gets 1."""
    X = np.abs(np.asarray(X, dtype=np.float64))
    if X.ndim != 2:
        raise ValueError("X must be a matrix")
    rows = X.shape[0]
    amax = X.max(axis=1) if X.shape[1] else np.zeros(rows)
    nonzero = amax > 0
    _, ex = np.frexp(np.where(nonzero, amax, 1.0))    # amax = f 2**ex, f in [0.5, 1)
    e1 = np.where(nonzero, 5 - (ex.astype(np.int64) - 1), 0)
    bar = np.ceil(np.ldexp(X, e1[:, None].astype(np.int32)))
    bar = np.where((X > 0) & (bar < 1), 1.0, bar)
    bar[~nonzero] = 0.0
    return e1, nonzero, bar.astype(np.int64)
