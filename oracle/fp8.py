"""Ozaki scheme II on an FP8 (E4M3) matrix engine: the residue products of
Step 3 (test infrastructure only).

Section 1 states that the scaling of Section 2.2 carries over to the fast
mode of Ozaki scheme II on FP8 matrix engines, and Section 6 leaves that
extension to future work; the paper gives no FP8 design.  The reading used
here changes nothing but the engine that forms the residue products:

* scaling (Algorithm 2 or 1), the integers A' and B' (Step 2), their
  residues rmod(A', p_t) and rmod(B', p_t) (the INT8 residues of the INT8
  path, modulus 256 as the two's-complement low byte) and the CRT and
  unscaling (Steps 3-4) are exactly those of the INT8 path, so C is the same
  to the last bit;
* an E4M3 value holds every integer of magnitude at most 16 exactly, but a
  residue reaches 128 in magnitude, so each residue r in [-128, 127] is
  split into two digits r = 16 h + l with l = ((r + 8) mod 16) - 8 in
  [-8, 7] and h = (r - l) / 16 in [-8, 8]; the engine operands are the
  E4M3 values 16 h (a power-of-two multiple of a digit, exact) and l;
* r_A r_B = (16 h_A)(16 h_B) + (16 h_A) l_B + l_A (16 h_B) + l_A l_B: four
  engine products per index of the sum, all accumulated into one binary32
  sum.  Per index the four terms add up in magnitude to at most
  (16 |h_A| + |l_A|)(16 |h_B| + |l_B|) <= 136^2 (136 is reached at
  r = 120), so over a block of KB = 512 indices every partial sum, in any
  order, is an integer of magnitude at most 512 * 136^2 < 2^24 and binary32
  holds it exactly; after each block the (exact) binary32 sum is added to
  an integer accumulator.  The product of a modulus is therefore exactly
  G_t = rmod(A', p_t) rmod(B', p_t), the INT8 path's product.

E4M3 here is the OCP 8-bit format with 4 exponent bits (bias 7) and 3
fraction bits: sign in bit 7, exponent field in bits 6-3, fraction in bits
2-0; a normal value is (-1)^s 2^(E-7) (1 + f/8) for E in 1..15 (E = 15 with
f = 7 is NaN), a subnormal one (-1)^s 2^-6 (f/8).
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

KB = 512                      # indices per binary32 block
BLOCK_BOUND = KB * 136 * 136  # largest |partial sum| of a block


def digits(r: int):
    """(h, l) with r = 16 h + l, l in [-8, 7], for a residue r in [-128, 127]."""
    if not -128 <= r <= 127:
        raise ValueError(f"residue {r} outside [-128, 127]")
    l = ((r + 8) % 16) - 8
    h = (r - l) // 16
    return h, l


def e4m3_decode(code: int) -> Fraction:
    """The value of an E4M3 code (a byte), from the format definition."""
    s, E, f = (code >> 7) & 1, (code >> 3) & 15, code & 7
    if E == 15 and f == 7:
        raise ValueError("NaN code")
    v = Fraction(f, 8) * Fraction(2) ** -6 if E == 0 else (1 + Fraction(f, 8)) * Fraction(2) ** (E - 7)
    return -v if s else v


def e4m3_encode(v: int) -> int:
    """The E4M3 code of an integer that the format holds exactly (|v| <= 448
    and at most 4 significant bits); raises otherwise."""
    if v == 0:
        return 0
    a = abs(v)
    E = a.bit_length() - 1            # 2^E <= a < 2^(E + 1)
    if E > 8 or a & ((1 << max(E - 3, 0)) - 1):
        raise ValueError(f"{v} is not exact in E4M3")
    f = ((a << 3) >> E) - 8 if E <= 3 else (a >> (E - 3)) - 8
    code = ((E + 7) << 3) | f
    if code >= 0x7F:
        raise ValueError(f"{v} is out of the E4M3 range")
    return code | (0x80 if v < 0 else 0)


def digit_codes(R):
    """E4M3 codes of the two digit operands of an int residue matrix:
    (codes of 16 h, codes of l), uint8 arrays of R's shape."""
    R = np.asarray(R, dtype=np.int64)
    H = np.empty(R.shape, dtype=np.uint8)
    L = np.empty(R.shape, dtype=np.uint8)
    for idx, r in np.ndenumerate(R):
        h, l = digits(int(r))
        H[idx] = e4m3_encode(16 * h)
        L[idx] = e4m3_encode(l)
    return H, L


def product(RA, RB):
    """G = RA RB for residue matrices RA (m x k) and RB (k x n), formed as
    the FP8 engine forms it: the four digit products per index, each block
    of KB indices summed (exactly, the block bound checked), the blocks
    added as integers.  Equals RA @ RB."""
    RA = np.asarray(RA, dtype=np.int64)
    RB = np.asarray(RB, dtype=np.int64)
    HA, LA = digit_codes(RA)
    HB, LB = digit_codes(RB)
    dec = np.vectorize(lambda c: int(e4m3_decode(int(c))), otypes=[np.int64])
    hA, lA, hB, lB = dec(HA), dec(LA), dec(HB), dec(LB)   # 16 h and l as integers
    m, k = RA.shape
    n = RB.shape[1]
    G = np.zeros((m, n), dtype=np.int64)
    for k0 in range(0, k, KB):
        s = slice(k0, min(k, k0 + KB))
        blk = hA[:, s] @ hB[s] + hA[:, s] @ lB[s] + lA[:, s] @ hB[s] + lA[:, s] @ lB[s]
        mag = (np.abs(hA[:, s]) + np.abs(lA[:, s])) @ (np.abs(hB[s]) + np.abs(lB[s]))
        if mag.size and int(mag.max()) > BLOCK_BOUND:
            raise AssertionError("a block's binary32 sum could be inexact")
        G += blk
    return G
