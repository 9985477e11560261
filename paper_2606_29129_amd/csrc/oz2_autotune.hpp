// oz2_autotune.hpp -- the number of moduli N for an accuracy target.
//
// The error of the emulated product is set by how many bits of each entry
// the scaled integers keep (more moduli: larger P, wider integers) and by the
// spread of the entry magnitudes.  For the distribution of the paper's
// experiments, (rand - 0.5) exp(phi randn) (Section 3.2), log|a| has variance
// 1 + phi^2, so phi is estimated from the sample variance of log|a| over the
// first 2^20 entries of each operand (storage order; zeros and non-finite
// entries skipped), and N is the smallest number of moduli whose error
// estimate is at most target / kTuneMargin.  The estimate is an upper
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

// One operand whose log-magnitude statistics are wanted.
struct StatSrc {
  const double* X;
  int64_t rows, ld, count;   // column-major rows x (count / rows ...), count <= 2^20
};

// Per-block partial statistics (number, sum and sum of squares of log|x|)
// of the first `count` entries in storage order (entry g at row g % rows,
// column g / rows).  Block b covers operand b / kStatBlocks; the host adds
// the partials of an operand in block order (deterministic).
__global__ __launch_bounds__(256) void k_logstats(const StatSrc* __restrict__ src,
                                                  double* __restrict__ part) {
  __shared__ double red[3][256];
  const int op = blockIdx.x / kStatBlocks, sub = blockIdx.x % kStatBlocks;
  const StatSrc s = src[op];
  // The operand pointer comes from a descriptor, so the compiler cannot tell
  // it is global memory; read through a global pointer (generic loads would
  // be flat accesses, each waited for before the next use).
  typedef __attribute__((address_space(1))) const double GlobalDouble;
  GlobalDouble* X = (GlobalDouble*)s.X;
  double c = 0.0, sum = 0.0, sq = 0.0;
  for (int64_t g = (int64_t)sub * 256 + threadIdx.x; g < s.count;
       g += (int64_t)kStatBlocks * 256) {
    const int64_t i = g % s.rows, h = g / s.rows;
    const double x = fabs(X[i + h * s.ld]);
    if (x > 0.0 && x <= 1.7976931348623157e308) {
      const double l = log(x);
      c += 1.0;
      sum += l;
      sq += l * l;
    }
  }
  red[0][threadIdx.x] = c;
  red[1][threadIdx.x] = sum;
  red[2][threadIdx.x] = sq;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 3) part[((int64_t)op * kStatBlocks + sub) * 3 + threadIdx.x] = red[threadIdx.x][0];
}

// phi from the partials of one operand: sqrt(max(var(log|x|) - 1, 0)) with
// the unbiased sample variance; fewer than two entries give 0.
inline double phi_from_partials(const double* p) {
  double c = 0.0, sum = 0.0, sq = 0.0;
  for (int b = 0; b < kStatBlocks; ++b) {
    c += p[3 * b];
    sum += p[3 * b + 1];
    sq += p[3 * b + 2];
  }
  if (c < 2.0) return 0.0;
  const double var = (sq - sum * sum / c) / (c - 1.0);
  return var > 1.0 ? sqrt(var - 1.0) : 0.0;
}

}  // namespace oz2
