"""Complex products C ~ A B with Ozaki scheme II (test infrastructure only).

The paper extends its scaling to complex products only in words: Section 1
notes that the same scaling formula serves the complex (ZGEMM, CGEMM) fast
mode, and Section 6 lists the complex case as future work.  It prints no
complex algorithm, so this module applies Section 2.2 and Algorithm 2 (or
Algorithm 1) to complex matrices under the following readings:

* Scaling.  A complex row a = x + i y (length k) is scaled as the real vector
  of its 2k components in storage order, (x_1, y_1, x_2, y_2, ...).  The
  squared 2-norm of that vector is sum_h |a_h|^2, the squared 2-norm of the
  complex row; its rounded-up value uses the fixed order of
  ``scaling.norm_sq_ru`` over the 2k components (chunks of 64 components,
  i.e. 32 complex entries).  Algorithm 1's maximum is the largest component
  magnitude.  Columns of B likewise.
  Why this keeps the CRT exact: each of |Re(a b)| and |Im(a b)| is at most
  |a||b|, so |Re c'_ij| and |Im c'_ij| are at most sum_h |a'_ih||b'_hj|
  <= ||a'_i|| ||b'_j|| (Cauchy-Schwarz), the quantity Algorithm 2 keeps below
  P/2.
* Step 2 truncates both components with the row's (column's) scale:
  a' = trunc(2^e x) + i trunc(2^e y); then |a'_h| <= 2^e |a_h|.
* Step 3 recovers the real and imaginary parts of the complex integer
  product A'B' separately by the CRT: with A' = X + iY and B' = U + iV,
  Re = XU - YV and Im = XV + YU, each formed per modulus from the residues of
  the four integer matrices.
* Step 4 rounds each part once, to nearest even, in the output format.

Accurate mode is not defined here (its bound product would need complex
magnitudes, which the paper does not discuss).  The exact mode (an optional
variant, ``scaling.exact_mode_log2_mu``) applies to the 2k components as
well.
"""
from __future__ import annotations

import numpy as np

from . import constants, fp, scaling
from .ozaki2 import (EXACT, ORIGINAL, REVISED, residue, residues, rmod, scaled_integer, step2,
                     step4)


def components(v) -> np.ndarray:
    """The 2k real components of a complex vector in storage order
    (re_1, im_1, re_2, im_2, ...)."""
    v = np.asarray(v, dtype=np.complex128).ravel()
    out = np.empty(2 * v.size, dtype=np.float64)
    out[0::2] = v.real
    out[1::2] = v.imag
    return out


def scale_exponents(A, B, N: int, mode: int = REVISED):
    """log2(mu_i), log2(nu_j) and the rounded-up squared norms of the rows of
    A and the columns of B (complex matrices)."""
    A = np.asarray(A, dtype=np.complex128)
    B = np.asarray(B, dtype=np.complex128)
    rows = [components(A[i, :]) for i in range(A.shape[0])]
    cols = [components(B[:, j]) for j in range(B.shape[1])]
    if mode == EXACT:
        _, P, _, _ = constants.step1(N)
        ra = [scaling.exact_mode_log2_mu(r, P) for r in rows]
        rb = [scaling.exact_mode_log2_mu(c, P) for c in cols]
        return [e for e, _ in ra], [e for e, _ in rb], [S for _, S in ra], [S for _, S in rb]
    SA = [scaling.norm_sq_ru(r) for r in rows]
    SB = [scaling.norm_sq_ru(c) for c in cols]
    if mode == REVISED:
        pp = constants.p_prime_prop(N)
        emu = [scaling.alg2_log2_mu(S, pp) for S in SA]
        enu = [scaling.alg2_log2_mu(S, pp) for S in SB]
    elif mode == ORIGINAL:
        pf, d = constants.p_prime_fast(N), constants.delta()
        amax = lambda v: float(np.max(np.abs(v))) if v.size else 0.0
        emu = [scaling.alg1_log2_mu(S, amax(r), pf, d) for S, r in zip(SA, rows)]
        enu = [scaling.alg1_log2_mu(S, amax(c), pf, d) for S, c in zip(SB, cols)]
    else:
        raise ValueError(f"mode {mode} is not defined for complex products")
    return emu, enu, SA, SB


def _crt(G, N):
    """C'' = rmod(sum_t P_t q_t G_t, P) for a list of integer matrices G_t."""
    _, P, Pi, qi = constants.step1(N)
    m, n = G[0].shape
    Cp = np.zeros((m, n), dtype=object)
    for t in range(N):
        Cp = Cp + (Pi[t] * qi[t]) * G[t].astype(object)
    Cpp = np.empty((m, n), dtype=object)
    for i in range(m):
        for j in range(n):
            Cpp[i, j] = rmod(int(Cp[i, j]), P)
    return Cpp


def gemm(A, B, N: int, mode: int = REVISED, out_fmt=fp.BINARY64):
    """The whole emulated complex product with its intermediates.

    A (m x k) and B (k x n) are complex numpy arrays (row-major).  Returns a
    dict: SA, SB, e_rows, e_cols, X, Y (A' = X + iY), U, V (B' = U + iV),
    Gre, Gim (per-modulus integer products of the residues), Cpp_re, Cpp_im
    (C'' parts) and C (complex128 for binary64 output, complex64 for
    binary32).
    """
    A = np.asarray(A, dtype=np.complex128)
    B = np.asarray(B, dtype=np.complex128)
    emu, enu, SA, SB = scale_exponents(A, B, N, mode)
    X, Y = step2(A.real, emu), step2(A.imag, emu)
    U, V = step2(B.real.T, enu).T, step2(B.imag.T, enu).T
    p, _, _, _ = constants.step1(N)
    Gre, Gim = [], []
    for pt in p:
        rx, ry, ru, rv = (residues(M, pt) for M in (X, Y, U, V))
        Gre.append(rx @ ru - ry @ rv)
        Gim.append(rx @ rv + ry @ ru)
    Cre, Cim = _crt(Gre, N), _crt(Gim, N)
    re = step4(Cre, emu, enu, out_fmt)
    im = step4(Cim, emu, enu, out_fmt)
    ct = np.complex128 if out_fmt == fp.BINARY64 else np.complex64
    C = np.empty(re.shape, dtype=ct)
    C.real = re
    C.imag = im
    return dict(SA=SA, SB=SB, e_rows=emu, e_cols=enu, X=X, Y=Y, U=U, V=V,
                Gre=Gre, Gim=Gim, Cpp_re=Cre, Cpp_im=Cim, C=C)


def zgemm(A, B, N: int, mode: int = REVISED):
    """C ~ A B for complex binary64 inputs and output."""
    return gemm(A, B, N, mode, fp.BINARY64)["C"]


def cgemm(A, B, N: int, mode: int = REVISED):
    """C ~ A B for complex binary32 inputs and output (one rounding per part
    to binary32)."""
    A = np.asarray(A, dtype=np.complex64).astype(np.complex128)
    B = np.asarray(B, dtype=np.complex64).astype(np.complex128)
    return gemm(A, B, N, mode, fp.BINARY32)["C"]


def entry(a_row, b_col, e_i: int, f_j: int, N: int, out_fmt=fp.BINARY64):
    """C_ij from row i of A, column j of B and their exponents (Steps 2-4 for
    one output entry, to check large problems on sampled entries).
    Returns (C_ij as a Python complex, C''_re, C''_im)."""
    a = np.asarray(a_row, dtype=np.complex128)
    b = np.asarray(b_col, dtype=np.complex128)
    x = [scaled_integer(float(v), e_i) for v in a.real]
    y = [scaled_integer(float(v), e_i) for v in a.imag]
    u = [scaled_integer(float(v), f_j) for v in b.real]
    v = [scaled_integer(float(w), f_j) for w in b.imag]
    p, P, Pi, qi = constants.step1(N)
    cre = cim = 0
    for t, pt in enumerate(p):
        rx = [residue(z, pt) for z in x]
        ry = [residue(z, pt) for z in y]
        ru = [residue(z, pt) for z in u]
        rv = [residue(z, pt) for z in v]
        gre = sum(q * r - s * w for q, r, s, w in zip(rx, ru, ry, rv))
        gim = sum(q * w + s * r for q, r, s, w in zip(rx, ru, ry, rv))
        cre += Pi[t] * qi[t] * gre
        cim += Pi[t] * qi[t] * gim
    cre, cim = rmod(cre, P), rmod(cim, P)
    re = fp.round_dyadic(cre, -(e_i + f_j), out_fmt, "RN")
    im = fp.round_dyadic(cim, -(e_i + f_j), out_fmt, "RN")
    return complex(re, im), cre, cim
