// oz2_autotune.hpp -- the number of moduli N for an accuracy target.
//
// The error of the emulated product is set by how many bits of each entry
// the scaled integers keep (more moduli: larger P, wider integers) and by the
// spread of the entry magnitudes.  For the distribution of the paper's
// experiments, (rand - 0.5) exp(phi randn) (Section 3.2), log|a| has variance
// 1 + phi^2, so phi is estimated from the sample variance of log|a| over the
// first 2^20 entries of each operand (storage order; zeros and non-finite
// entries skipped), and N is the smallest number of moduli whose calibrated
// maximum relative error (oz2_autotune_table.hpp) at the next grid point at or
// above (k, phi) is at most target / kTuneMargin.
#pragma once

#include <math.h>
#include <stdint.h>

#include "oz2_autotune_table.hpp"

namespace oz2 {

constexpr double kTuneMargin = 4.0;
constexpr int64_t kPhiSample = int64_t(1) << 20;   // entries per operand
constexpr int kStatBlocks = 16;                     // blocks per operand

// Smallest N meeting the target at (k, phi) per the calibrated table (the
// last, largest N when none does).
inline int tune_pick_N(int64_t k, double phi, double target) {
  int ik = kTuneNK - 1;
  for (int i = 0; i < kTuneNK; ++i)
    if (kTuneK[i] >= k) { ik = i; break; }
  int ip = kTuneNPhi - 1;
  for (int i = 0; i < kTuneNPhi; ++i)
    if (kTunePhi[i] >= phi - 1e-12) { ip = i; break; }
  for (int j = 0; j < kTuneNN; ++j)
    if (kTuneErr[ik][ip][j] * kTuneMargin <= target) return kTuneN0 + j;
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
