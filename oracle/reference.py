"""Exact reference products and accuracy metrics (test infrastructure only).

The paper measures the maximum relative error against a double-double
reference (Sections 3.2 and 5.1).  The oracle uses the exact rational product
instead, which a double-double product approximates: every binary64 value is
an integer times a power of two, so a dot product is summed exactly in Python
integers and rounded once.

Metrics (the paper does not say what it does where the reference entry is 0):

* ``max_rel_err``: max over reference entries != 0 of |C - R| / |R|, plus the
  number of entries where R == 0 but C != 0;
* ``max_comp_err``: max over entries of |C - R| / (|A||B|)_ij, the
  componentwise measure (entries with (|A||B|)_ij == 0 must match exactly).
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def _int_exp(x: float):
    """x = n * 2**e with integer n (exact)."""
    num, den = float(x).as_integer_ratio()
    return num, -(den.bit_length() - 1)


def exact_dot(a, b) -> Fraction:
    """sum_h a_h b_h exactly, for binary64 (or binary32) vectors."""
    terms = []
    emin = None
    for x, y in zip(np.asarray(a, np.float64), np.asarray(b, np.float64)):
        if x == 0.0 or y == 0.0:
            continue
        nx, ex = _int_exp(x)
        ny, ey = _int_exp(y)
        e = ex + ey
        terms.append((nx * ny, e))
        emin = e if emin is None else min(emin, e)
    if not terms:
        return Fraction(0)
    total = sum(n << (e - emin) for n, e in terms)
    return Fraction(total, 1) * (Fraction(2) ** emin if emin >= 0 else Fraction(1, 2 ** (-emin)))


def exact_abs_dot(a, b) -> Fraction:
    return exact_dot(np.abs(np.asarray(a, np.float64)), np.abs(np.asarray(b, np.float64)))


def errors(C, A, B, rows=None, cols=None):
    """Error metrics of C against the exact product on a set of entries.

    ``rows``/``cols`` select sampled entries (all by default); C is indexed
    by the same sampled positions (C[r, c] for r in rows, c in cols).
    Returns dict(max_rel, n_zero_ref_nonzero, max_comp).
    """
    A = np.asarray(A, np.float64)
    B = np.asarray(B, np.float64)
    rows = range(A.shape[0]) if rows is None else rows
    cols = range(B.shape[1]) if cols is None else cols
    max_rel = Fraction(0)
    max_comp = Fraction(0)
    zero_bad = 0
    for ii, i in enumerate(rows):
        for jj, j in enumerate(cols):
            R = exact_dot(A[i, :], B[:, j])
            c = float(C[ii, jj]) if C.shape == (len(rows), len(cols)) else float(C[i, j])
            if not np.isfinite(c):
                return dict(max_rel=float("inf"), n_zero_ref_nonzero=zero_bad,
                            max_comp=float("inf"))
            d = abs(Fraction(c) - R)
            if R != 0:
                max_rel = max(max_rel, d / abs(R))
            elif c != 0:
                zero_bad += 1
            absd = exact_abs_dot(A[i, :], B[:, j])
            if absd != 0:
                max_comp = max(max_comp, d / absd)
            elif d != 0:
                max_comp = Fraction(10**30)
    return dict(max_rel=float(max_rel), n_zero_ref_nonzero=zero_bad,
                max_comp=float(max_comp))
