// oz2_tables.hpp -- Step 1 constants (Section 2.2) for each N, computed on
// the host with a small fixed-width big integer, and the device table that
// the kernels read from constant memory.
#pragma once

#include <math.h>
#include <stdint.h>
#include <string.h>

namespace oz2 {

constexpr int kMaxN = 20;
constexpr int kMaxSlices = 4;    // 39-bit slices of P and of the CRT weights
constexpr int kSliceBits = 39;
constexpr int kLimbBits = 40;    // limbs of a' used by the residue kernel

// The moduli printed in Section 3.1; N moduli means the first N.
constexpr int kModuli[kMaxN] = {256, 255, 253, 251, 247, 241, 239, 233, 229, 227,
                                223, 217, 211, 199, 197, 193, 191, 181, 179, 173};

// Everything a kernel needs for one N.  Integers are stored as exact doubles.
struct ModTable {
  int N;
  int slices;                      // number of 39-bit slices covering P
  int limbs;                       // 40-bit limbs covering |a'| (2 or 3)
  int pad_;
  double p[kMaxN];                 // p_t
  double inv_p[kMaxN];             // RN(1/p_t), only for quotient estimates
  double powL[kMaxN][4];           // 2^(40 j) mod p_t, j = 0..3
  double w[kMaxN][kMaxSlices];     // W_t = P_t q_t (< P) in 39-bit slices
  double P[kMaxSlices];            // P in 39-bit slices
  double H[kMaxSlices];            // P/2 in 39-bit slices
  double invP;                     // RN(1/P), only for quotient estimates
  double quarterP;                 // a binary64 value a little below P/4
  double pm1_rd;                   // RD64(P - 1): x <= P - 1 iff x <= pm1_rd (binary64 x)
  float p_prop;                    // P'_prop = RD32(log2(P-1)/2 - 0.5)
  float p_fast;                    // P'_fast = RD32(log2(P-1)/2 - 1.5)
  float delta;                     // RU32(0.5 / (1 - 4 u32))
  float pad2_;
  double log2P;                    // informative
};

// Unsigned big integer with 32-bit limbs, little-endian; enough for P < 2^156.
struct Big {
  static constexpr int L = 6;
  uint32_t d[L];
  Big() { memset(d, 0, sizeof d); }
  explicit Big(uint64_t v) {
    memset(d, 0, sizeof d);
    d[0] = (uint32_t)v;
    d[1] = (uint32_t)(v >> 32);
  }
  Big mul_small(uint32_t s) const {
    Big r;
    uint64_t carry = 0;
    for (int i = 0; i < L; ++i) {
      uint64_t v = (uint64_t)d[i] * s + carry;
      r.d[i] = (uint32_t)v;
      carry = v >> 32;
    }
    return r;
  }
  Big div_small(uint32_t s, uint32_t* rem) const {
    Big r;
    uint64_t cur = 0;
    for (int i = L - 1; i >= 0; --i) {
      cur = (cur << 32) | d[i];
      r.d[i] = (uint32_t)(cur / s);
      cur %= s;
    }
    if (rem) *rem = (uint32_t)cur;
    return r;
  }
  Big sub_small(uint32_t s) const {
    Big r = *this;
    uint64_t borrow = s;
    for (int i = 0; i < L && borrow; ++i) {
      uint64_t v = (uint64_t)r.d[i];
      if (v >= borrow) { r.d[i] = (uint32_t)(v - borrow); borrow = 0; }
      else { r.d[i] = (uint32_t)(v + (1ull << 32) - borrow); borrow = 1; }
    }
    return r;
  }
  int bitlen() const {
    for (int i = L - 1; i >= 0; --i)
      if (d[i]) return 32 * i + (32 - __builtin_clz(d[i]));
    return 0;
  }
  // bits [lo, lo+n) as an integer (n <= 63)
  uint64_t bits(int lo, int n) const {
    uint64_t v = 0;
    for (int b = 0; b < n; ++b) {
      int pos = lo + b;
      if (pos < 32 * L && ((d[pos / 32] >> (pos % 32)) & 1u)) v |= 1ull << b;
    }
    return v;
  }
  // log2 of the value via its top 64 bits (relative error ~2^-64).
  long double log2l_approx() const {
    int bl = bitlen();
    int sh = bl > 63 ? bl - 63 : 0;
    return log2l((long double)bits(sh, 63)) + (long double)sh;
  }
};

inline uint32_t inv_mod(uint32_t a, uint32_t p) {
  // extended Euclid on small integers
  int64_t t = 0, nt = 1, r = p, nr = a % p;
  while (nr) {
    int64_t q = r / nr, tmp;
    tmp = t - q * nt; t = nt; nt = tmp;
    tmp = r - q * nr; r = nr; nr = tmp;
  }
  if (r != 1) return 0;
  if (t < 0) t += p;
  return (uint32_t)t;
}

inline uint32_t pow2_mod(int e, uint32_t p) {
  uint64_t r = 1 % p;
  for (int i = 0; i < e; ++i) r = (r * 2) % p;
  return (uint32_t)r;
}

// RD32 / RU32 of a long double with a check that the rounding is decided by
// the long double value (distance to the binary32 grid well above its error).
inline bool round_f32_checked(long double x, bool up, float* out) {
  float f = (float)x;
  if (up) { if ((long double)f < x) f = nextafterf(f, INFINITY); }
  else    { if ((long double)f > x) f = nextafterf(f, -INFINITY); }
  long double lo = up ? (long double)nextafterf(f, -INFINITY) : (long double)f;
  long double hi = up ? (long double)f : (long double)nextafterf(f, INFINITY);
  long double margin = fabsl(x) * 0x1p-55L + 0x1p-60L;
  if (x - lo < margin && x != lo) return false;
  if (hi - x < margin && x != hi) return false;
  *out = f;
  return true;
}

// Fill the table for N moduli.  Returns false if N is out of range or a
// constant could not be rounded safely.
inline bool build_table(int N, bool accurate_limbs, ModTable* T) {
  if (N < 2 || N > kMaxN) return false;
  memset(T, 0, sizeof *T);
  T->N = N;
  Big P(1);
  for (int t = 0; t < N; ++t) P = P.mul_small((uint32_t)kModuli[t]);
  const int pbits = P.bitlen();
  T->slices = (pbits + kSliceBits - 1) / kSliceBits;
  if (T->slices > kMaxSlices) return false;
  // Fast modes: |a'| <= sqrt((P-1)/2) < 2^((pbits-1)/2), so pbits/2 bits
  // suffice; accurate mode allows up to 64x more (bar entries <= 64).
  int abits = pbits / 2 + (accurate_limbs ? 7 : 0);
  int limbs = (abits + kLimbBits - 1) / kLimbBits;
  T->limbs = limbs < 2 ? 2 : limbs;
  if (T->limbs > 4) return false;
  for (int t = 0; t < N; ++t) {
    uint32_t p = (uint32_t)kModuli[t];
    uint32_t rem;
    Big Pt = P.div_small(p, &rem);
    uint32_t Pt_mod = 0;
    Pt.div_small(p, &Pt_mod);
    uint32_t q = inv_mod(Pt_mod, p);
    if (q == 0) return false;
    Big W = Pt.mul_small(q);  // P_t q_t < P, already reduced
    T->p[t] = (double)p;
    T->inv_p[t] = 1.0 / (double)p;
    for (int j = 0; j < 4; ++j) T->powL[t][j] = (double)pow2_mod(kLimbBits * j, p);
    for (int s = 0; s < kMaxSlices; ++s) T->w[t][s] = (double)W.bits(kSliceBits * s, kSliceBits);
  }
  uint32_t r2;
  Big H = P.div_small(2, &r2);
  for (int s = 0; s < kMaxSlices; ++s) {
    T->P[s] = (double)P.bits(kSliceBits * s, kSliceBits);
    T->H[s] = (double)H.bits(kSliceBits * s, kSliceBits);
  }
  long double log2P = P.log2l_approx();
  T->log2P = (double)log2P;
  T->invP = (double)exp2l(-log2P);
  T->quarterP = (double)(exp2l(log2P - 2.0L) * (1.0L - 0x1p-30L));
  {
    // P - 1 rounded down to binary64: its top 53 bits, truncated.
    const Big Pm1 = P.sub_small(1);
    const int bl = Pm1.bitlen();
    const int sh = bl > 53 ? bl - 53 : 0;
    T->pm1_rd = ldexp((double)Pm1.bits(sh, 53), sh);
  }
  long double log2Pm1 = P.sub_small(1).log2l_approx();
  if (!round_f32_checked(log2Pm1 / 2 - 0.5L, false, &T->p_prop)) return false;
  if (!round_f32_checked(log2Pm1 / 2 - 1.5L, false, &T->p_fast)) return false;
  if (!round_f32_checked(0.5L / (1.0L - 0x1p-22L), true, &T->delta)) return false;
  return true;
}

}  // namespace oz2
