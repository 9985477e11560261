// oz2_math.hpp -- scalar arithmetic of the scaling step (host and device).
//
// Everything here is exact or directed-rounded by construction, built from
// round-to-nearest binary64 operations plus error-free transforms, so that
// the GPU reproduces the rounded-up squared norms and the scale exponents of
// Algorithms 1 and 2 bit for bit.  Compile with -ffp-contract=off: every
// fused multiply-add is written explicitly.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define OZ2_HD __host__ __device__ __forceinline__

namespace oz2 {

// A binary64 constant held in a scalar register pair.  gfx9's three-operand
// (VOP3) encoding takes no literal, so an FMA with a constant factor whose
// addend stays live was encoded in the two-operand form with a literal,
// after a copy of the addend: one extra move per use.  From a scalar
// register the FMA is a single VOP3 instruction.
OZ2_HD double sconst(double c) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r;
  asm("s_mov_b64 %0, %1" : "=s"(r) : "s"(c));
  return r;
#else
  return c;
#endif
}

// A value the compiler may not look through (it stays in its vector
// registers unchanged).  A multiplier of +-1 is otherwise rewritten as a
// select between x and -x: two 32-bit selects and a sign flip per binary64
// operand instead of one multiply.
OZ2_HD double opaque_v(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  asm("" : "+v"(x));
#endif
  return x;
}

// The low bytes of four 32-bit values in one dword (v0's in byte 0): two
// byte permutes gather the pairs, a third joins them (three instructions;
// masking and shifting each byte takes six).
OZ2_HD uint32_t pack_low_bytes(uint32_t v0, uint32_t v1, uint32_t v2, uint32_t v3) {
#if defined(__HIP_DEVICE_COMPILE__)
  const uint32_t lo = __builtin_amdgcn_perm(v1, v0, 0x0c0c0400u);  // v0.b0, v1.b0, 0, 0
  const uint32_t hi = __builtin_amdgcn_perm(v3, v2, 0x0c0c0400u);
  return __builtin_amdgcn_perm(hi, lo, 0x05040100u);             // lo.b0, lo.b1, hi.b0, hi.b1
#else
  return (v0 & 0xFFu) | ((v1 & 0xFFu) << 8) | ((v2 & 0xFFu) << 16) | ((v3 & 0xFFu) << 24);
#endif
}

OZ2_HD double bits_to_f64(uint64_t u) { return __builtin_bit_cast(double, u); }
OZ2_HD uint64_t f64_to_bits(double d) { return __builtin_bit_cast(uint64_t, d); }
OZ2_HD float bits_to_f32(uint32_t u) { return __builtin_bit_cast(float, u); }
OZ2_HD uint32_t f32_to_bits(float f) { return __builtin_bit_cast(uint32_t, f); }

// The symmetric residue r = c - q p, q = round(c / p), of an integer c with
// |c| < 2^31 for an odd modulus p < 256 (ip = 1/p rounded to nearest), as a
// 32-bit two's complement word: two fmas and an integer add.
// fma(c, ip, 1.5 2^52) = 1.5 2^52 + q: the product is exact inside the fma
// and the sum's unit is 1; c / p lies at least 1/(2p) from a half-integer
// while |c ip - c / p| < 2^-22 / p, so q is the integer nearest to c / p.
// fma(1.5 2^52 + q, -p, 1.5 2^52 (p + 1)) has the exact value
// 1.5 2^52 - q p (|q p| < 2^31 + p, inside the binade of 1.5 2^52, whose
// unit is 1), whose low word is -q p in two's complement, so c plus that
// word is r, |r| <= (p - 1) / 2.
OZ2_HD uint32_t residue_sym_i32(int32_t c, double p, double ip) {
  constexpr double kMagic = 0x1.8p52;
  const double magic_p1 = kMagic * (p + 1.0);             // exact: 1.5 (p + 1) < 2^9
  const double tq = fma((double)c, ip, kMagic);           // 1.5 2^52 + q
  const double nq = fma(tq, -p, magic_p1);                // 1.5 2^52 - q p, exact
  return (uint32_t)c + (uint32_t)f64_to_bits(nq);
}

// Next binary64 above a finite non-negative x (0 -> smallest subnormal).
OZ2_HD double next_up_nonneg(double x) { return bits_to_f64(f64_to_bits(x) + 1); }

// Next binary32 above / below a finite f.
OZ2_HD float next_up_f32(float f) {
  if (f == 0.0f) return bits_to_f32(1u);
  uint32_t b = f32_to_bits(f);
  return bits_to_f32(f > 0.0f ? b + 1u : b - 1u);
}
OZ2_HD float next_down_f32(float f) { return -next_up_f32(-f); }

// single_up(d) / single_down(d): binary64 -> binary32 rounded toward +inf /
// -inf (Section 2.1 notation).  The cast rounds to nearest; one step fixes it.
OZ2_HD float ru_f32(double d) {
  float f = (float)d;
  if ((double)f < d) f = next_up_f32(f);
  return f;
}
OZ2_HD float rd_f32(double d) {
  float f = (float)d;
  if ((double)f > d) f = next_down_f32(f);
  return f;
}

// RU(x*x) for x = 0 or x >= 2^-480: the FMA residual fma(x, x, -p) is then
// exact.  An infinite or NaN square passes through (its residual is not
// positive).
OZ2_HD double ru_square_normal(double x) {
  const double p = x * x;
  return fma(x, x, -p) > 0.0 ? next_up_nonneg(p) : p;
}

// RU(a*a) in binary64.  Below |a| = 2^-480 the residual would not be exact,
// so the square is formed on a*2^600 and scaled back, rounding up once more
// (rounding up onto a coarser grid after rounding up onto a finer one that
// contains it is one rounding up).
OZ2_HD double ru_square(double a) {
  const double x = a < 0 ? -a : a;
  if (x < 0x1p-480 && x != 0.0) {
    double b = ldexp(x, 600);              // exact, b < 2^120
    double pb = b * b;                     // >= 2^-948: residual exact
    double eb = fma(b, b, -pb);
    if (eb > 0.0) pb = next_up_nonneg(pb);
    double r = ldexp(pb, -1200);           // one correctly rounded scaling
    if (ldexp(r, 1200) < pb) r = next_up_nonneg(r);  // scaling back is exact
    return r;
  }
  return ru_square_normal(x);
}

// RU(x + y) for x, y >= 0: the rounded sum, raised by one ulp when the exact
// error (TwoSum) is positive.  An infinite or NaN sum passes through (its
// error is NaN).
OZ2_HD double ru_add(double x, double y) {
  const double s = x + y;
  const double bb = s - x;
  const double err = (x - (s - bb)) + (y - bb);
  return err > 0.0 ? next_up_nonneg(s) : s;
}

// s + a_0^2 + ... + a_{NA-1}^2 with every square and every addition rounded
// up, in that order.  The group is screened once for tiny entries
// (0 < |a| < 2^-480, which take ru_square's scaled path); a group without
// any runs as straight-line code.
template <int NA>
OZ2_HD double ru_add_squares(double s, const double (&a)[NA]) {
  bool tiny = false;
#pragma unroll
  for (int i = 0; i < NA; ++i) {
    const double x = a[i] < 0 ? -a[i] : a[i];
    tiny = tiny || (x < 0x1p-480 && x != 0.0);
  }
  if (tiny) {
#pragma unroll
    for (int i = 0; i < NA; ++i) s = ru_add(s, ru_square(a[i]));
  } else {
#pragma unroll
    for (int i = 0; i < NA; ++i) s = ru_add(s, ru_square_normal(a[i] < 0 ? -a[i] : a[i]));
  }
  return s;
}

// floor(log2 x) of a finite x > 0 and the exact ratio x / 2^s in [1, 2).
OZ2_HD int split_pow2(double x, double* frac) {
  int e;
  double f = frexp(x, &e);  // x = f 2^e, f in [0.5, 1)
  *frac = 2.0 * f;
  return e - 1;
}

// The binary32 log2 that stands in for the paper's fast log2: the binary64
// log2 of a binary32 input rounded to nearest binary32.  For the inputs used
// here (binary32 values in [1, 2]) this is the correctly rounded log2; the
// test suite checks that for every such input.
OZ2_HD float log2_rn32(float x) { return (float)log2((double)x); }

// Algorithm 2 (Section 4): log2(mu_i) from the rounded-up squared norm S.
// S is split into its binary exponent and a mantissa in [1, 2); half the
// binary32 log2 of the mantissa, plus a slack of 2^-23 that covers the log's
// error, is rounded up (an upper estimate of the fractional half-log); the
// integer part, P'_prop minus half the exponent, is rounded down.  Their
// exact difference, floored, is the exponent: never above the largest e with
// 2^(2e+1) S <= P - 1.  The mantissa goes to binary32 rounding up; S = 0
// gives 0.
OZ2_HD int alg2_exponent(double S, float p_prop) {
  if (S == 0.0) return 0;
  double x;
  int s = split_pow2(S, &x);
  float L = log2_rn32(ru_f32(x));
  float t = ru_f32(0.5 * (double)L + 0x1p-23);        // exact sum, one rounding
  float w = rd_f32((double)p_prop - 0.5 * (double)s);  // exact difference
  return (int)floor((double)w - (double)t);            // exact difference
}

// Exact mode (an optional variant of Algorithm 2): the largest e with
// 2^(2e+1) S <= P - 1 for a finite S > 0.  S 2^(2e+1) is a binary64 value
// near P (no overflow or underflow), and a binary64 x satisfies x <= P - 1
// exactly when x <= RD64(P - 1) = pm1_rd, so the comparison is exact.  With
// S in [2^ES, 2^(ES+1)) and pm1_rd in [2^EQ, 2^(EQ+1)) the answer lies in
// [floor((EQ - ES) / 2) - 1, floor((EQ - ES) / 2)].  S = 0 gives 0.
OZ2_HD int emax_exponent(double S, double pm1_rd) {
  if (S == 0.0) return 0;
  double f;
  const int ES = split_pow2(S, &f), EQ = split_pow2(pm1_rd, &f);
  int e = (EQ - ES) >> 1;   // floor division (arithmetic shift)
  if (ldexp(S, 2 * e + 1) > pm1_rd) --e;
  return e;
}

// Algorithm 1 (Section 2.3): the original fast-mode exponent.  An upper
// estimate of half log2 S (the binary32 log2 of S rounded up, times delta,
// rounded up again; at least 1) is taken from P'_fast, floored, and the
// exponent of the largest entry magnitude is subtracted.
OZ2_HD int alg1_exponent(double S, double amax, float p_fast, float delta) {
  if (S == 0.0) return 0;
  double x;
  int s = split_pow2(S, &x);
  float L = log2_rn32(ru_f32(x));
  float u = ru_f32((double)L + (double)s);
  float t = ru_f32((double)delta * (double)u);          // exact product
  double mx = (double)t > 1.0 ? (double)t : 1.0;
  int e1 = (int)floor((double)p_fast - mx);
  double dummy;
  return e1 - split_pow2(amax, &dummy);
}

// tilde-log2 of eq. (flog2) for an integer c > 0 (accurate mode): the
// binary32 log2 of c's mantissa plus c's binary exponent, the sum rounded up.
OZ2_HD float tilde_log2_ru(int64_t c) {
  double x;
  int e = split_pow2((double)c, &x);
  float L = log2_rn32(ru_f32(x));
  return ru_f32((double)L + (double)e);
}

// Accurate mode (Section 2.3): the first exponent log2 mu'_i plus the floor
// of P'_accu less an upper estimate of half log2 of the row's largest bound
// product (delta times tilde-log2 of it, rounded up).
OZ2_HD int accurate_exponent(int e_first, int64_t cmax, float p_accu, float delta) {
  if (cmax <= 0) return 0;
  float corr = ru_f32((double)delta * (double)tilde_log2_ru(cmax));
  return e_first + (int)floor((double)p_accu - (double)corr);
}

}  // namespace oz2
