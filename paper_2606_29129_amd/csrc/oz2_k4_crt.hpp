// oz2_k4_crt.hpp -- K4: CRT reconstruction (Step 3) and unscaling (Step 4).
//
// For each output entry, with U_t = rmod(C_t, p_t) from K3 (a signed byte;
// any representative of C_t modulo p_t of magnitude < 2^9 would do):
//   X   = sum_t W_t U_t,   W_t = P_t q_t  (< P)           (eq. os2-C')
//   C'' = X - P round(X / P)  in (-P/2, P/2)                (eq. os2-C'')
//   C   = RN(C'' 2^-(e_i + f_j))                            (Step 4)
// Because |A'B'| < P/2 (eq. os2-condition), C'' = A'B' exactly.
//
// Exact arithmetic in binary64: W_t is held as 39-bit slices w_ts, so each
// slice sum |Acc_s| = |sum_t w_ts U_t| < 20 * 2^39 * 2^9 < 2^53 is exact.
// The quotient Q = round(X / P) (|Q| < 2^14) is estimated from a rounded X; every
// R_s = Acc_s - Q P_s is exact, and an exact signed comparison with P/2
// corrects a quotient that is off by one (skipped when a rounded value of R
// already shows |R| < P/4).  That rounded value also gives the sign; the
// magnitude's slices are normalised (carries propagated exactly) and rounded
// once, to nearest even, at the bit position that the output format
// (binary64 or binary32, subnormals included) dictates: for normal results by
// one binary64 addition of two exact operands, otherwise by cutting the
// slices at that bit.
#pragma once

#include "oz2_k1_norm.hpp"
#include "oz2_k3_gemm.hpp"
#include "oz2_tables.hpp"

namespace oz2 {

template <int S>
OZ2_HD void normalize(double (&R)[S]) {
#pragma unroll
  for (int s = 0; s < S - 1; ++s) {
    double c = floor(R[s] * 0x1p-39);
    R[s] = fma(-c, 0x1p39, R[s]);
    R[s + 1] += c;
  }
}

// Sign of sum_s D_s 2^(39 s) after normalisation (lower slices in [0, 2^39)).
template <int S>
OZ2_HD int sign_of(double (&D)[S]) {
  normalize(D);
  if (D[S - 1] != 0.0) return D[S - 1] > 0.0 ? 1 : -1;
#pragma unroll
  for (int s = S - 2; s >= 0; --s)
    if (D[s] != 0.0) return 1;
  return 0;
}

// Rounded value of sum_s R_s 2^(39 s), by Horner steps (one rounding each).
// For integer slices |R_s| < 2^53 - 2^39 the result is exact while
// |sum| < 2^53: every partial sum is then an integer below 2^53.
// Otherwise each step rounds a partial sum of magnitude at least 2^52
// times its slice weight, so the relative error stays below S 2^-53 (1 + 2^-37)
// < 2^-50: the result has the sign of the sum, is zero only for a zero sum,
// and is within a factor 1 +- 2^-50 of it.
template <int S>
OZ2_HD double slices_value(const double (&R)[S]) {
  double v = R[S - 1];
#pragma unroll
  for (int s = S - 2; s >= 0; --s) v = fma(v, sconst(0x1p39), R[s]);
  return v;
}

// Correct rounding, to nearest even at the output format's quantum, of
// V 2^-E for V = sum_s R_s 2^(39 s) > 0 with normalised slices (every R_s
// in [0, 2^39)): the exponent of the leading bit, L = floor(log2 V), fixes
// the quantum 2^q, q = max(L - (PREC - 1), E + EMIN_Q), and the slices are
// cut at bit q.  Used for the outputs the direct form below does not cover
// (subnormal results and zero).
template <int S, int PREC, int EMIN_Q>
OZ2_HD double round_slices_general(const double (&R)[S], int32_t E) {
  int j = S - 1;
  while (j > 0 && R[j] == 0.0) --j;
  if (R[j] == 0.0) return 0.0;
  double frac;
  const int L = 39 * j + split_pow2(R[j], &frac);   // floor(log2 V)
  const int q = (L - (PREC - 1)) > (E + EMIN_Q) ? (L - (PREC - 1)) : (E + EMIN_Q);
  if (q <= 0) {
    double v = 0.0;
#pragma unroll
    for (int s = S - 1; s >= 0; --s) v += ldexp(R[s], 39 * s);  // exact: V < 2^PREC
    return ldexp(v, -E);
  }
  if (q - 1 > L) return 0.0;                         // below half the quantum
  const int sstar = (q - 1) / 39;                    // slice holding bit q-1
  double Tq = 0.0, ftop = 0.0;
  bool rest = false;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    double vs = ldexp(R[s], 39 * s - q);             // exact
    double I = floor(vs);
    double f = vs - I;
    Tq += I;
    if (s == sstar) ftop = f;
    else if (s < sstar && f != 0.0) rest = true;
  }
  const double cmp = ftop - 0.5;
  const bool odd = floor(Tq * 0.5) * 2.0 != Tq;     // Tq < 2^53: an exact integer
  const bool up = cmp > 0.0 || (cmp == 0.0 && (rest || odd));
  return ldexp(Tq + (up ? 1.0 : 0.0), q - E);
}

// The same rounding in a few binary64 operations when the top slice R_{S-1}
// is nonzero and the result is normal.  In units u = 2^(39 (S-2)),
// V / u = t 2^39 + u1 + u2 2^-39 + z (t = R_{S-1}, u1 = R_{S-2},
// u2 = R_{S-3}, z = the rest, 0 <= z < 2^-39), and the 53-bit rounding of
// V / u is one binary64 addition X + Y of two exact operands:
//  * t < 2^14: X = t 2^39 + u1 < 2^53 (exact), Y = u2 2^-39 plus 2^-40 when
//    z > 0.  V / u >= 2^39, so every rounding boundary (half an ulp) is a
//    multiple of 2^-14; V / u and X + Y lie on the same side of each such
//    multiple of 2^-39 (both strictly between two of them when z > 0).
//  * t >= 2^14: X = t 2^39, Y = u1 plus 1/2 when u2 or z is nonzero.
//    V / u >= 2^53, so the boundaries are integers, and the same argument
//    holds with integer spacing.
// For binary32 the sum is rounded to odd at 53 bits (Y - (s - X) is the exact
// error of s = X + Y, |X| >= |Y|): rounding that to 24 bits is the correct
// rounding of V, since 53 >= 24 + 2.  Returns false (leaving out unset)
// when the scaled result falls below the smallest normal number.
template <int S, int PREC, int EMIN_Q>
OZ2_HD bool round_slices_top(const double (&R)[S], int32_t E, double* out) {
  double res;
  int k;
  if constexpr (S == 1) {
    res = R[0];                                      // exact
    k = -E;
  } else {
    const double t = R[S - 1], u1 = R[S - 2];
    double u2 = 0.0;
    if constexpr (S >= 3) u2 = R[S - 3];
    bool z = false;
#pragma unroll
    for (int s = 0; s + 3 < S; ++s) z = z || R[s] != 0.0;
    const bool small = t < 0x1p14;
    const double X = small ? fma(t, sconst(0x1p39), u1) : t * 0x1p39;
    const double Y = small ? fma(u2, sconst(0x1p-39), z ? 0x1p-40 : 0.0)
                           : u1 + ((z || u2 != 0.0) ? 0.5 : 0.0);
    res = X + Y;
    if constexpr (PREC < 53) {
      const double err = Y - (res - X);
      if (err != 0.0) {
        uint64_t b = f64_to_bits(res);
        if (err < 0.0) b -= 1;
        res = bits_to_f64(b | 1);
      }
    }
    k = 39 * (S - 2) - E;
  }
  int ex;
  (void)frexp(res, &ex);                             // res in [2^(ex-1), 2^ex)
  if (ex - 1 + k < EMIN_Q + PREC - 1) return false;
  *out = ldexp(res, k);
  return true;
}

// PREC = 53 (binary64) or 24 (binary32); EMIN_Q = exponent of the smallest
// subnormal (-1074 or -149).
template <int S, int PREC, int EMIN_Q>
OZ2_HD double crt_unscale(const double (&acc)[S], const ModTable& T, int32_t E) {
  // Quotient estimate and the exact residual R = X - Q P (|R_s| < 2^52:
  // |Acc_s| < 2^51 and |Q P_s| < 2^51).
  const double Q = rint(slices_value(acc) * T.invP);
  double R[S];
#pragma unroll
  for (int s = 0; s < S; ++s) R[s] = fma(-Q, T.P[s], acc[s]);
  // Bring R into (-P/2, P/2): R = C'' + jP with |j| <= 1 and |C''| < P/2.
  // Fast test first: the rounded value r of R is within a factor 1 +- 2^-50
  // of R, so |r| <= quarterP (< P/4 (1 - 2^-30)) proves |R| < P/2, i.e.
  // R = C''.  Otherwise the exact comparisons with P/2 decide.
  double r = slices_value(R);
  if (!(fabs(r) <= T.quarterP)) {
    double D[S];
#pragma unroll
    for (int s = 0; s < S; ++s) D[s] = R[s] - T.H[s];
    if (sign_of(D) > 0) {
#pragma unroll
      for (int s = 0; s < S; ++s) R[s] -= T.P[s];
    } else {
#pragma unroll
      for (int s = 0; s < S; ++s) D[s] = R[s] + T.H[s];
      if (sign_of(D) < 0) {
#pragma unroll
        for (int s = 0; s < S; ++s) R[s] += T.P[s];
      }
    }
    r = slices_value(R);
  }
  // r has the sign of C'': the magnitude's slices, normalised into
  // [0, 2^39) (all of them: the magnitude is non-negative).
  const bool neg = r < 0.0;
  const double sg = opaque_v(neg ? -1.0 : 1.0);
#pragma unroll
  for (int s = 0; s < S; ++s) R[s] *= sg;
  normalize(R);
  // Leading zero slices shifted out (V 2^-E = V' 2^-(E + 39 sh)).
  int sh = 0;
  while (sh < S - 1 && R[S - 1] == 0.0) {
#pragma unroll
    for (int s = S - 1; s > 0; --s) R[s] = R[s - 1];
    R[0] = 0.0;
    ++sh;
  }
  const int32_t Es = E + 39 * sh;
  double res;
  if (!(R[S - 1] != 0.0 && round_slices_top<S, PREC, EMIN_Q>(R, Es, &res)))
    res = round_slices_general<S, PREC, EMIN_Q>(R, Es);
  return neg ? -res : res;
}

// WPB (2 or 4) waves per 32 x 32 block: wave h of the block takes the
// R = 16 / WPB accumulator-order entries R h .. R h + R - 1 of each lane,
// i.e. rows (32 / WPB) h .. (32 / WPB)(h + 1) - 1 of the block (all 32
// columns), R of the 16 bytes each plane holds per lane.  (More waves than
// one per block: at small sizes the grid is otherwise one wave or less per
// SIMD whose plane loads and reconstruction run back to back; two per block
// in general, four for small outputs.)  The results go through a per-wave
// LDS tile so that each store instruction writes column segments of
// 32 / WPB entries.
constexpr int kK4WavesPerBlock = 2;
constexpr int kK4WavesPerBlockSmall = 4;

template <int S, typename TO, int WPB = kK4WavesPerBlock>
__device__ __forceinline__ void k4_crt_body(
    const uint8_t* __restrict__ U, const int32_t* __restrict__ eA,
    const int32_t* __restrict__ eB, const ModTable* __restrict__ tab, int N,
    int64_t m, int64_t n, int64_t Mp, int64_t Np, TO* __restrict__ C, int64_t ldc, int64_t bx) {
  static_assert(WPB == 2 || WPB == 4, "waves per block");
  constexpr int RPW = 32 / WPB;             // rows of the block per wave
  __shared__ TO tile[4][RPW][33];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t Mb = Mp / 32, Nb = Np / 32;
  const int64_t wid = bx * 4 + wave;
  const int64_t blk = wid / WPB;
  const int h = (int)(wid % WPB);
  const int64_t mb_used = (m + 31) / 32;
  const int64_t nb_used = (n + 31) / 32;
  if (blk >= mb_used * nb_used) return;  // whole wave: the tile is per wave
  const int64_t bi = blk % mb_used, bj = blk / mb_used;
  constexpr int R = 16 / WPB, RW = R / 4, PF = 4;
  const uint8_t* src = U + (bj * Mb + bi) * 1024 + lane * 16 + R * h;
  const int64_t plane = Nb * Mb * 1024;
  const int lc = acc_col(lane);
  const int64_t col = bj * 32 + lc;
  const int32_t f = col < n ? eB[col] : 0;
  const ModTable& T = *tab;
  // The plane bytes are loaded in groups of PF planes, the next group's
  // loads issued before the current group is accumulated, so a wave waits
  // for memory once per group instead of once per plane.  The next group's
  // plane indices are clamped to N - 1 (a repeated, in-bounds load) rather
  // than skipped: with a fixed number of loads in flight the waits before
  // the current group's accumulation leave the next group's loads pending.
  // The row exponents of this lane's outputs, loaded up front.
  int32_t er[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t row = bi * 32 + acc_row(R * h + r, lane);
    er[r] = row < m ? eA[row] : 0;
  }
  double acc[R][S];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int s = 0; s < S; ++s) acc[r][s] = 0.0;
  auto load_plane = [&](int t, uint32_t (&ws)[RW]) {
    if constexpr (RW == 2) {
      const uint2 w = *reinterpret_cast<const uint2*>(src + (int64_t)t * plane);
      ws[0] = w.x;
      ws[1] = w.y;
    } else {
      ws[0] = *reinterpret_cast<const uint32_t*>(src + (int64_t)t * plane);
    }
  };
  auto accumulate = [&](int t, const uint32_t (&ws)[RW]) {
    double wt[S];
#pragma unroll
    for (int s = 0; s < S; ++s) wt[s] = tab->w[t][s];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double u = (double)(int)(int8_t)(ws[r >> 2] >> (8 * (r & 3)));
#pragma unroll
      for (int s = 0; s < S; ++s) acc[r][s] = fma(wt[s], u, acc[r][s]);
    }
  };
  uint32_t cur[PF][RW] = {}, nxt[PF][RW] = {};
#pragma unroll
  for (int i = 0; i < PF; ++i) load_plane(i < N ? i : N - 1, cur[i]);
  for (int t0 = 0; t0 < N; t0 += PF) {
#pragma unroll
    for (int i = 0; i < PF; ++i)
      load_plane(t0 + PF + i < N ? t0 + PF + i : N - 1, nxt[i]);
#pragma unroll
    for (int i = 0; i < PF; ++i)
      if (t0 + i < N) accumulate(t0 + i, cur[i]);
#pragma unroll
    for (int i = 0; i < PF; ++i)
#pragma unroll
      for (int q = 0; q < RW; ++q) cur[i][q] = nxt[i][q];
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int lr = acc_row(R * h + r, lane);     // RPW h .. RPW h + RPW - 1
    const int64_t row = bi * 32 + lr;
    double v = 0.0;
    if (row < m && col < n) {
      const int32_t e = er[r];
      if (e == kExpNonFinite || f == kExpNonFinite) {
        v = __builtin_nan("");
      } else {
        double a[S];
#pragma unroll
        for (int s = 0; s < S; ++s) a[s] = acc[r][s];
        if constexpr (sizeof(TO) == 8) v = crt_unscale<S, 53, -1074>(a, T, e + f);
        else v = crt_unscale<S, 24, -149>(a, T, e + f);
      }
    }
    tile[wave][lr - RPW * h][lc] = (TO)v;
  }
  // LDS operations of one wave complete in order; the fence keeps the
  // compiler from moving the reads above the writes.
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const int orow = lane % RPW;
  const int64_t row = bi * 32 + RPW * h + orow;
#pragma unroll
  for (int i = 0; i < RPW / 2; ++i) {
    const int oc = (64 / RPW) * i + lane / RPW;
    const int64_t c = bj * 32 + oc;
    if (row < m && c < n) C[row + c * ldc] = tile[wave][orow][oc];
  }
}

template <int S, typename TO, int WPB = kK4WavesPerBlock>
__global__ __launch_bounds__(256) void k4_crt(
    const uint8_t* __restrict__ U, const int32_t* __restrict__ eA,
    const int32_t* __restrict__ eB, const ModTable* __restrict__ tab, int N,
    int64_t m, int64_t n, int64_t Mp, int64_t Np, TO* __restrict__ C, int64_t ldc) {
  k4_crt_body<S, TO, WPB>(U, eA, eB, tab, N, m, n, Mp, Np, C, ldc, blockIdx.x);
}

// C = 0 (k = 0).
template <typename TO>
__global__ void k_zero(TO* __restrict__ C, int64_t m, int64_t n, int64_t ldc) {
  int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= m * n) return;
  int64_t j = g / m, i = g - j * m;
  C[i + j * ldc] = (TO)0;
}

}  // namespace oz2
