// oz2_autotune.hpp -- the number of moduli N for an accuracy target.
//
// The error of the emulated product is set by how many bits of each entry
// the scaled integers keep (more moduli: larger P, wider integers) and by the
// spread of the entry magnitudes.  For the distribution of the paper's
// experiments, (rand - 0.5) exp(phi randn) (Section 3.2), log|a| has variance
// 1 + phi^2, so phi is estimated from the variance of log|a| within the
// vectors the scaling treats -- the rows of A, the columns of B -- pooled
// over a sample of about 2^20 entries of each operand (zeros and non-finite
// entries skipped): the spread of magnitudes inside a vector is what its
// scale exponent cannot absorb, so, like the revised scaling itself, the
// estimate does not change when rows or columns are scaled by different
// powers of two.  N is the smallest number of moduli whose error estimate is
// at most target / kTuneMargin.  The estimate is an upper
// envelope of the calibrated maxima (oz2_autotune_table.hpp), so that the
// pick never falls when k, phi or the accuracy demand grows even where the
// single-seed measurements are not monotone: at each grid point the largest
// tabulated error over every grid point at or below it, for this N or any
// larger one, and between grid points that envelope's log interpolated
// bilinearly in (log2 k, phi).  Beyond the largest calibrated k it grows by
// sqrt(k / k_max) (the scaling keeps about half a bit less per
// doubling of k: the norm grows with sqrt(k)); beyond the largest calibrated
// phi there is no basis for an estimate and the pick is the largest N.
#pragma once

#include <math.h>
#include <stdint.h>

#include "oz2_autotune_table.hpp"

namespace oz2 {

constexpr double kTuneMargin = 4.0;
constexpr int64_t kPhiSample = int64_t(1) << 20;   // entries per operand
constexpr int kStatBlocks = 16;                     // blocks per operand

// Envelope at grid point (ik, ip) for the j-th tabulated N: the largest
// tabulated error at or below the grid point, for this N or a larger one.
inline double tune_envelope(int ik, int ip, int j) {
  double e = 0.0;
  for (int a = 0; a <= ik; ++a)
    for (int b = 0; b <= ip; ++b)
      for (int jj = j; jj < kTuneNN; ++jj) e = e > kTuneErr[a][b][jj] ? e : kTuneErr[a][b][jj];
  return e;
}

// Error estimate for (k, phi) with the j-th tabulated N (see above): the
// envelope's log interpolated bilinearly in (log2 k, phi) between the grid
// points around (k, phi) (the end points below the grid); a negative value
// means phi lies beyond the calibrated range.
inline double tune_error_estimate(int64_t k, double phi, int j) {
  if (phi > kTunePhi[kTuneNPhi - 1] + 1e-12) return -1.0;
  const double kc = (double)(k < kTuneK[0] ? kTuneK[0] : k);
  int k1 = kTuneNK - 1;
  for (int i = 0; i < kTuneNK; ++i)
    if ((double)kTuneK[i] >= kc) { k1 = i; break; }
  const int k0 = k1 > 0 ? k1 - 1 : 0;
  double wk = 0.0;
  if (k1 > k0)
    wk = kc < (double)kTuneK[k1]
             ? log2(kc / (double)kTuneK[k0]) / log2((double)kTuneK[k1] / (double)kTuneK[k0])
             : 1.0;
  const double pc = phi < kTunePhi[0] ? kTunePhi[0] : phi;
  int p1 = kTuneNPhi - 1;
  for (int i = 0; i < kTuneNPhi; ++i)
    if (kTunePhi[i] >= pc - 1e-12) { p1 = i; break; }
  const int p0 = p1 > 0 ? p1 - 1 : 0;
  double wp = 0.0;
  if (p1 > p0) wp = (pc - kTunePhi[p0]) / (kTunePhi[p1] - kTunePhi[p0]);
  if (wp > 1.0) wp = 1.0;
  double e;
  if ((wk == 0.0 || wk == 1.0) && (wp == 0.0 || wp == 1.0)) {
    e = tune_envelope(wk == 0.0 ? k0 : k1, wp == 0.0 ? p0 : p1, j);   // on a grid point
  } else {
    const double l00 = log2(tune_envelope(k0, p0, j)), l01 = log2(tune_envelope(k0, p1, j));
    const double l10 = log2(tune_envelope(k1, p0, j)), l11 = log2(tune_envelope(k1, p1, j));
    e = exp2((1.0 - wk) * ((1.0 - wp) * l00 + wp * l01) + wk * ((1.0 - wp) * l10 + wp * l11));
  }
  if (k > kTuneK[kTuneNK - 1]) e *= sqrt((double)k / (double)kTuneK[kTuneNK - 1]);
  return e;
}

// Smallest N whose error estimate meets the target (the largest N when none
// does, or when phi lies beyond the calibrated range).
inline int tune_pick_N(int64_t k, double phi, double target) {
  for (int j = 0; j < kTuneNN; ++j) {
    const double e = tune_error_estimate(k, phi, j);
    if (e < 0.0) break;
    if (e * kTuneMargin <= target) return kTuneN0 + j;
  }
  return kTuneN0 + kTuneNN - 1;
}

// The sample of one operand whose log-magnitude spread is wanted: nvec
// vectors -- the rows of A or the columns of B, the vectors the scaling
// treats one by one -- of len entries each; entry e of vector v at
// X[v vstride + e estride].
struct StatSrc {
  const double* X;
  int64_t nvec, len, vstride, estride;
};

typedef __attribute__((address_space(1))) const double GlobalDouble;

// Count, sum and sum of squares of log|x| - x0 over the entries e0, e0 +
// step, ... below e1 of vector v (zeros and non-finite entries skipped), x0
// being log|x| of the vector's first entry when that is finite and nonzero,
// else 0 (the shift keeps the variance free of cancellation when the
// vector's magnitudes sit far from 1).  Four entries per round, their loads
// issued together.
__device__ __forceinline__ void vec_logsums(GlobalDouble* X, const StatSrc& s, int64_t v,
                                            int64_t e0, int64_t e1, int64_t step, double* n,
                                            double* s1, double* s2) {
  GlobalDouble* x = X + v * s.vstride;
  const double f = fabs(x[0]);
  const double x0 = (f > 0.0 && f <= 1.7976931348623157e308) ? log(f) : 0.0;
  double c = 0.0, a = 0.0, q = 0.0;
  auto add = [&](double y) {
    y = fabs(y);
    if (y > 0.0 && y <= 1.7976931348623157e308) {
      const double d = log(y) - x0;
      c += 1.0;
      a += d;
      q += d * d;
    }
  };
  int64_t e = e0;
  for (; e + 3 * step < e1; e += 4 * step) {
    double y[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) y[i] = x[(e + i * step) * s.estride];
#pragma unroll
    for (int i = 0; i < 4; ++i) add(y[i]);
  }
  for (; e < e1; e += step) add(x[e * s.estride]);
  *n = c;
  *s1 = a;
  *s2 = q;
}

// Per-block partial sums of the pooled within-vector statistics of one
// operand: W = sum over vectors of sum (log|x| - mean of the vector)^2 and
// D = sum over vectors of (count - 1), vectors with fewer than two entries
// left out.  Block b covers operand b / kStatBlocks; the host adds the
// partials of an operand in block order (deterministic).  Strided vectors
// (rows of a column-major matrix): kStatRows consecutive vectors per pass of
// a block, the block's threads split into kStatSegs groups that take
// consecutive ranges of the entries (a load of a wave reads kStatRows
// neighbouring vectors in each of its groups' columns), the groups' sums of
// a vector added in group order.  Contiguous vectors (columns): one wave per
// vector, its lanes reading neighbouring entries, the lanes' sums combined
// across the wave.
constexpr int kStatSegs = 16, kStatRows = 256 / kStatSegs;
__global__ __launch_bounds__(256) void k_logstats(const StatSrc* __restrict__ src,
                                                  double* __restrict__ part) {
  __shared__ double red[2][256];
  __shared__ double ws[3][kStatSegs][kStatRows];
  const int op = blockIdx.x / kStatBlocks, sub = blockIdx.x % kStatBlocks;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const StatSrc s = src[op];
  // The operand pointer comes from a descriptor, so the compiler cannot tell
  // it is global memory; read through a global pointer (generic loads would
  // be flat accesses, each waited for before the next use).
  GlobalDouble* X = (GlobalDouble*)s.X;
  double W = 0.0, D = 0.0;
  if (s.estride != 1) {
    const int r = tid % kStatRows, sg = tid / kStatRows;
    const int64_t q = (s.len + kStatSegs - 1) / kStatSegs;
    const int64_t e0 = sg * q, e1 = e0 + q < s.len ? e0 + q : s.len;
    for (int64_t g = sub; g * kStatRows < s.nvec; g += kStatBlocks) {
      const int64_t v = g * kStatRows + r;
      double n = 0.0, s1 = 0.0, s2 = 0.0;
      if (v < s.nvec) vec_logsums(X, s, v, e0, e1, 1, &n, &s1, &s2);
      ws[0][sg][r] = n;
      ws[1][sg][r] = s1;
      ws[2][sg][r] = s2;
      __syncthreads();
      if (tid < kStatRows && v < s.nvec) {
        double t[3] = {0.0, 0.0, 0.0};
        for (int j = 0; j < kStatSegs; ++j)
#pragma unroll
          for (int k = 0; k < 3; ++k) t[k] += ws[k][j][tid];
        if (t[0] >= 2.0) {
          W += t[2] - t[1] * t[1] / t[0];
          D += t[0] - 1.0;
        }
      }
      __syncthreads();
    }
  } else {
    for (int64_t v = (int64_t)sub * 4 + wave; v < s.nvec; v += (int64_t)kStatBlocks * 4) {
      double n, s1, s2;
      vec_logsums(X, s, v, lane, s.len, 64, &n, &s1, &s2);
      for (int o = 32; o > 0; o >>= 1) {
        n += __shfl_xor(n, o);
        s1 += __shfl_xor(s1, o);
        s2 += __shfl_xor(s2, o);
      }
      if (lane == 0 && n >= 2.0) {
        W += s2 - s1 * s1 / n;
        D += n - 1.0;
      }
    }
  }
  red[0][tid] = W;
  red[1][tid] = D;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) {
      red[0][tid] += red[0][tid + w];
      red[1][tid] += red[1][tid + w];
    }
    __syncthreads();
  }
  if (tid < 2) part[((int64_t)op * kStatBlocks + sub) * 2 + tid] = red[tid][0];
}

// phi from the partials of one operand: sqrt(max(var - 1, 0)) with var =
// W / D the pooled within-vector sample variance of log|x|; 0 when no vector
// has two entries.
inline double phi_from_partials(const double* p) {
  double W = 0.0, D = 0.0;
  for (int b = 0; b < kStatBlocks; ++b) {
    W += p[2 * b];
    D += p[2 * b + 1];
  }
  if (!(D > 0.0)) return 0.0;
  const double var = W / D;
  return var > 1.0 ? sqrt(var - 1.0) : 0.0;
}

// The sample of a column-major rows x cols matrix (leading dimension ld)
// whose vectors are its rows (by_cols = 0: A) or its columns (by_cols = 1:
// B): every vector with its first max(2, kPhiSample / (number of vectors))
// entries (all of them when it is shorter), about kPhiSample entries in all.
inline StatSrc stat_src(const double* X, int64_t rows, int64_t cols, int64_t ld, int by_cols) {
  const int64_t nvec = by_cols ? cols : rows, full = by_cols ? rows : cols;
  int64_t len = kPhiSample / (nvec > 0 ? nvec : 1);
  len = len < 2 ? 2 : len;
  len = len < full ? len : full;
  return by_cols ? StatSrc{X, nvec, len, ld, 1} : StatSrc{X, nvec, len, 1, ld};
}

}  // namespace oz2
