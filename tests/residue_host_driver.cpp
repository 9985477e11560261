// Host build of the GEMM epilogue's residue arithmetic (test
// infrastructure): for every odd modulus p in [3, 255] and a fixed set of
// INT32 values c -- the ends of the range a product entry can take, values
// next to the points where the nearest multiple of p changes (c = q p +- (p -
// 1) / 2 and one beyond), and a pseudo-random sweep (Marsaglia's xorshift64)
// over the whole range and over small magnitudes -- compares
// residue_sym_i32 with the symmetric residue from integer division.  Then
// K2's residue of a truncated scaled entry a' given as 40-bit limbs
// (residue_odd, two limbs as in the fast modes and three as in accurate
// mode) against the residue of a' itself, a 128-bit integer, for random a'
// of every length up to the modes' bounds and for a' next to the points
// where the nearest multiple of p changes.  Prints "cases mismatches" and,
// for the first few mismatches, "p c got want" (or "p a' got want").
#include <cstdint>
#include <cstdio>

#include "oz2_k2_split.hpp"

using namespace oz2;

static int64_t want_residue(int64_t c, int64_t p) {
  int64_t r = c % p;  // sign of c, |r| < p
  const int64_t h = (p - 1) / 2;
  if (r > h) r -= p;
  if (r < -h) r += p;
  return r;
}

int main() {
  uint64_t state = 0x9E3779B97F4A7C15ull;
  auto next = [&state]() {
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return state;
  };
  long long cases = 0, bad = 0;
  auto check = [&](int64_t c, int p) {
    if (c > INT32_MAX || c < -(int64_t)INT32_MAX) return;
    const double pd = (double)p, ip = 1.0 / pd;
    const int32_t got = (int32_t)residue_sym_i32((int32_t)c, pd, ip);
    const int64_t want = want_residue(c, p);
    ++cases;
    if (got != want && ++bad <= 5) printf("%d %lld %d %lld\n", p, (long long)c, got, (long long)want);
  };
  for (int p = 3; p <= 255; p += 2) {
    const int64_t h = (p - 1) / 2;
    for (int64_t c : {(int64_t)0, (int64_t)1, (int64_t)-1, (int64_t)INT32_MAX, -(int64_t)INT32_MAX,
                      (int64_t)INT32_MAX - 1, -(int64_t)INT32_MAX + 1})
      check(c, p);
    // both sides of every switch of q near the ends and in the middle
    for (int64_t q0 : {(int64_t)0, (int64_t)INT32_MAX / p - 2, -((int64_t)INT32_MAX / p) + 2,
                       (int64_t)1 << 20, -((int64_t)1 << 20)})
      for (int64_t q = q0 - 2; q <= q0 + 2; ++q)
        for (int64_t d : {-h - 1, -h, h, h + 1}) check(q * p + d, p);
    for (int i = 0; i < 100000; ++i) {
      const uint64_t r = next();
      check((int64_t)(int32_t)(uint32_t)r, p);                        // whole range
      check((int64_t)((int32_t)(uint32_t)(r >> 32) >> (r & 31)), p);  // every magnitude
      const int64_t q = (int64_t)(int32_t)(uint32_t)(r >> 16) / p;    // next to a switch
      check(q * p + ((r & 1) ? h : -h), p);
    }
  }
  // residue_odd: a' with |a'| < 2^79 (two limbs) or 2^86 (three limbs)
  auto limb_check = [&](__int128 a, int p, int limbs) {
    // signed 40-bit limbs with the sign of a', as make_limbs forms them
    const bool neg = a < 0;
    unsigned __int128 m = neg ? (unsigned __int128)(-a) : (unsigned __int128)a;
    double x[3];
    for (int j = 0; j < 3; ++j) {
      const double v = (double)(uint64_t)(m & (((unsigned __int128)1 << kLimbBits) - 1));
      x[j] = neg ? -v : v;
      m >>= kLimbBits;
    }
    double pw[3];
    for (int j = 0; j < 3; ++j) {
      unsigned __int128 w = ((unsigned __int128)1 << (kLimbBits * j)) % (unsigned)p;
      pw[j] = (double)(uint64_t)w;
    }
    int got;
    if (limbs == 2) {
      Limbs<2> L{{x[0], x[1]}};
      got = residue_odd<2>(L, pw, (double)p, 1.0 / (double)p);
    } else {
      Limbs<3> L{{x[0], x[1], x[2]}};
      got = residue_odd<3>(L, pw, (double)p, 1.0 / (double)p);
    }
    __int128 r = a % p;
    const int h = (p - 1) / 2;
    if (r > h) r -= p;
    if (r < -h) r += p;
    ++cases;
    if (got != (int)r && ++bad <= 10)
      printf("%d %.17g %d %d\n", p, (double)a, got, (int)r);
  };
  for (int p = 3; p <= 255; p += 2) {
    for (int i = 0; i < 20000; ++i) {
      for (int limbs = 2; limbs <= 3; ++limbs) {
        const int maxbits = limbs == 2 ? 79 : 86;
        const int nb = 1 + (int)(next() % maxbits);
        unsigned __int128 v = ((unsigned __int128)next() << 64) | next();
        v &= (((unsigned __int128)1 << nb) - 1);
        __int128 a = (__int128)v;
        if (next() & 1) a = -a;
        limb_check(a, p, limbs);
        // next to a switch of the nearest multiple: a = q p +- (p - 1) / 2
        __int128 q = a / p;
        const __int128 lim = ((__int128)1 << maxbits) - 1 - p;
        if (q * p + p < lim && q * p - p > -lim)
          limb_check(q * p + ((next() & 1) ? (p - 1) / 2 : -(p - 1) / 2), p, limbs);
      }
    }
  }
  printf("%lld %lld\n", cases, bad);
  return bad != 0;
}
