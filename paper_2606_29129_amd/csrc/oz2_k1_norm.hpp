// oz2_k1_norm.hpp -- K1: rounded-up squared norms of the rows of A and the
// columns of B, and the scale exponents log2(mu_i), log2(nu_j) of Step 2.
//
// Fixed summation order (the paper allows any order for the rounded-up sum;
// a fixed one makes results reproducible): chunks of kKC consecutive entries,
// each chunk summed left to right, then the chunk sums left to right; every
// square and every addition rounded toward +inf in binary64.
//
// Pass 1 writes one partial sum per (chunk, vector); pass 2 folds the
// partials in chunk order and evaluates Algorithm 1 or 2 per vector.
#pragma once

#include "oz2_math.hpp"
#include "oz2_tables.hpp"

namespace oz2 {

constexpr int kKC = 64;
constexpr int32_t kExpNonFinite = INT32_MIN;  // exponent sentinel: NaN output
constexpr int32_t kExpRescale = INT32_MIN + 2;  // exact mode: norm overflowed, recompute
constexpr int kRescaleShift = 600;               // exact mode: entries scaled by 2^-600

// Exact mode's overflow fallback: |a| 2^-600 rounded up in binary64 (the
// scaling is exact unless the result is subnormal; scaling that result back
// up is exact, so a shortfall shows and the magnitude is raised by one ulp).
OZ2_HD double ru_scale_down(double a) {
  const double x = fabs(a);
  double r = ldexp(x, -kRescaleShift);
  if (ldexp(r, kRescaleShift) < x) r = next_up_nonneg(r);
  return r;
}

// Entry as summed by a partial-sum pass: itself, or (RESC) scaled down.
template <bool RESC>
OZ2_HD double norm_entry(double a) {
  if constexpr (RESC) return ru_scale_down(a);
  else return a;
}

// Vectors stored with stride `ld` between consecutive entries (rows of a
// column-major matrix): entry h of vector v is X[v + h * ld].  One lane per
// vector (64 consecutive vectors per wave, so every load is a contiguous 512
// bytes), one wave per chunk; non-temporal loads (the operand is streamed
// once and does not fit the caches).
// RESC: the exact mode's second pass, only for vectors whose exponent is
// kExpRescale (esel), summing the scaled-down entries.
template <typename T, bool RESC = false, bool NT = true>
__device__ __forceinline__ void k1_partials_strided_body(
    const T* __restrict__ X, int64_t ld, int64_t nvec, int64_t k, int64_t nchunks,
    double* __restrict__ part, double* __restrict__ pmax, int64_t bx, int64_t by,
    const int32_t* __restrict__ esel = nullptr) {
  const int lane = threadIdx.x & 63;
  const int64_t v = bx * 64 + lane;
  const int64_t c = by * 4 + (threadIdx.x >> 6);
  if (v >= nvec || c >= nchunks) return;
  if (RESC && esel[v] != kExpRescale) return;
  const int64_t h0 = c * kKC;
  const int64_t len = k - h0 < kKC ? k - h0 : kKC;
  const T* p = X + v + h0 * ld;
  double s = 0.0, mx = 0.0;
  if (len == kKC) {
#pragma unroll
    for (int b = 0; b < kKC; b += 16) {
      double a[16];
#pragma unroll
      for (int i = 0; i < 16; ++i)
        a[i] = norm_entry<RESC>(NT ? (double)__builtin_nontemporal_load(p + (int64_t)(b + i) * ld)
                                   : (double)p[(int64_t)(b + i) * ld]);
      s = ru_add_squares(s, a);
#pragma unroll
      for (int i = 0; i < 16; ++i) mx = fmax(mx, fabs(a[i]));
    }
  } else {
    for (int64_t h = 0; h < len; ++h) {
      double a = norm_entry<RESC>((double)p[h * ld]);
      s = ru_add(s, ru_square(a));
      mx = fmax(mx, fabs(a));
    }
  }
  part[c * nvec + v] = s;
  if (pmax) pmax[c * nvec + v] = mx;
}

template <typename T, bool RESC = false>
__global__ __launch_bounds__(256) void k1_partials_strided(
    const T* __restrict__ X, int64_t ld, int64_t nvec, int64_t k, int64_t nchunks,
    double* __restrict__ part, double* __restrict__ pmax,
    const int32_t* __restrict__ esel = nullptr) {
  k1_partials_strided_body<T, RESC>(X, ld, nvec, k, nchunks, part, pmax, blockIdx.x, blockIdx.y,
                                    esel);
}

// Vectors stored contiguously (columns of a column-major matrix): entry h of
// vector v is X[h + v * ld].  One lane per (vector, chunk); lanes of a wave
// take consecutive chunks.
template <typename T, bool RESC = false>
__device__ __forceinline__ void k1_partials_contig_body(
    const T* __restrict__ X, int64_t ld, int64_t nvec, int64_t k, int64_t nchunks,
    double* __restrict__ part, double* __restrict__ pmax, int64_t bx,
    const int32_t* __restrict__ esel = nullptr) {
  const int64_t g = bx * 256 + threadIdx.x;
  if (g >= nvec * nchunks) return;
  const int64_t v = g / nchunks;
  const int64_t c = g - v * nchunks;
  if (RESC && esel[v] != kExpRescale) return;
  const int64_t h0 = c * kKC;
  const int64_t len = k - h0 < kKC ? k - h0 : kKC;
  const T* p = X + v * ld + h0;
  double s = 0.0, mx = 0.0;
  if (len == kKC) {
#pragma unroll
    for (int b = 0; b < kKC; b += 16) {
      double a[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) a[i] = norm_entry<RESC>((double)p[b + i]);
      s = ru_add_squares(s, a);
#pragma unroll
      for (int i = 0; i < 16; ++i) mx = fmax(mx, fabs(a[i]));
    }
  } else {
    for (int64_t h = 0; h < len; ++h) {
      double a = norm_entry<RESC>((double)p[h]);
      s = ru_add(s, ru_square(a));
      mx = fmax(mx, fabs(a));
    }
  }
  part[c * nvec + v] = s;
  if (pmax) pmax[c * nvec + v] = mx;
}

template <typename T, bool RESC = false>
__global__ __launch_bounds__(256) void k1_partials_contig(
    const T* __restrict__ X, int64_t ld, int64_t nvec, int64_t k, int64_t nchunks,
    double* __restrict__ part, double* __restrict__ pmax,
    const int32_t* __restrict__ esel = nullptr) {
  k1_partials_contig_body<T, RESC>(X, ld, nvec, k, nchunks, part, pmax, blockIdx.x, esel);
}

// Pass 2: fold partial sums in chunk order and evaluate the exponent.
// mode 0: Algorithm 2 (revised); mode 1: Algorithm 1 (original fast mode);
// mode 3: the exact maximal exponent (an overflowing norm is marked for the
// fallback pass instead of flagged).
// A squared norm that is NaN or +inf yields the sentinel exponent and sets
// bit OZ2_STATUS_NONFINITE in *status.
// Fold the chunk sums of vector v left to right with rounded-up additions
// (and their maxima): 16 loads are issued ahead of each 16 sequential adds
// so that the chain waits on arithmetic, not on memory latency.
__device__ __forceinline__ void fold_chunks(const double* __restrict__ part,
                                            const double* __restrict__ pmax, int64_t nchunks,
                                            int64_t nvec, int64_t v, double* S_out, double* mx_out) {
  double S = 0.0, mx = 0.0;
  int64_t c = 0;
  for (; c + 16 <= nchunks; c += 16) {
    double b[16], q[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) b[i] = part[(c + i) * nvec + v];
    if (pmax) {
#pragma unroll
      for (int i = 0; i < 16; ++i) q[i] = pmax[(c + i) * nvec + v];
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      S = ru_add(S, b[i]);
      if (pmax) mx = fmax(mx, q[i]);
    }
  }
  for (; c < nchunks; ++c) {
    S = ru_add(S, part[c * nvec + v]);
    if (pmax) mx = fmax(mx, pmax[c * nvec + v]);
  }
  *S_out = S;
  *mx_out = mx;
}

__device__ __forceinline__ void k1_fold_body(
    const double* __restrict__ part, const double* __restrict__ pmax, int64_t nchunks,
    int64_t nvec, int mode, const ModTable* __restrict__ tab, int32_t* __restrict__ e_out,
    double* __restrict__ S_out, int* __restrict__ status, int64_t bx) {
  const int64_t v = bx * 256 + threadIdx.x;
  if (v >= nvec) return;
  double S, mx;
  fold_chunks(part, pmax, nchunks, nvec, v, &S, &mx);
  if (S_out) S_out[v] = S;
  int32_t e;
  if (mode == 3 && S > 1.7976931348623157e308) {
    e = kExpRescale;                  // +inf: the exact mode's fallback pass
  } else if (!(S <= 1.7976931348623157e308)) {
    e = kExpNonFinite;
    atomicOr(status, 1);
  } else if (mode == 0) {
    e = alg2_exponent(S, tab->p_prop);
  } else if (mode == 3) {
    e = emax_exponent(S, tab->pm1_rd);
  } else {
    e = alg1_exponent(S, mx, tab->p_fast, tab->delta);
  }
  e_out[v] = e;
}

// Exact mode, fallback fold: for the vectors marked kExpRescale, fold the
// partial sums of the scaled-down entries and shift the exponent back.
__global__ __launch_bounds__(256) void k1_fold_rescale(
    const double* __restrict__ part, int64_t nchunks, int64_t nvec,
    const ModTable* __restrict__ tab, int32_t* __restrict__ e_out,
    double* __restrict__ S_out, int* __restrict__ status) {
  const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (v >= nvec || e_out[v] != kExpRescale) return;
  double S, mx;
  fold_chunks(part, nullptr, nchunks, nvec, v, &S, &mx);
  if (S_out) S_out[v] = S;
  int32_t e;
  if (!(S <= 1.7976931348623157e308)) {   // an infinite entry
    e = kExpNonFinite;
    atomicOr(status, 1);
  } else {
    e = emax_exponent(S, tab->pm1_rd) - kRescaleShift;
  }
  e_out[v] = e;
}

__global__ __launch_bounds__(256) void k1_fold(
    const double* __restrict__ part, const double* __restrict__ pmax, int64_t nchunks,
    int64_t nvec, int mode, const ModTable* __restrict__ tab, int32_t* __restrict__ e_out,
    double* __restrict__ S_out, int* __restrict__ status) {
  k1_fold_body(part, pmax, nchunks, nvec, mode, tab, e_out, S_out, status, blockIdx.x);
}

// Accurate mode, first scale (Section 2.3): e'_v = 5 - floor(log2 max|a|) from
// the folded chunk maxima.  A zero vector gets kExpZero (its bar row is 0);
// a non-finite one gets kExpNonFinite and sets the status bit.
constexpr int32_t kExpZero = INT32_MIN + 1;

__global__ __launch_bounds__(256) void k1_fold_first(
    const double* __restrict__ part, const double* __restrict__ pmax, int64_t nchunks,
    int64_t nvec, int32_t* __restrict__ e1_out, int* __restrict__ status) {
  const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (v >= nvec) return;
  double S, mx;
  fold_chunks(part, pmax, nchunks, nvec, v, &S, &mx);
  int32_t e;
  if (!(S <= 1.7976931348623157e308)) {
    e = kExpNonFinite;
    atomicOr(status, 1);
  } else if (mx == 0.0) {
    e = kExpZero;
  } else {
    double f;
    e = 5 - split_pow2(mx, &f);
  }
  e1_out[v] = e;
}

// Accurate mode, final exponent: log2 mu = e' + floor(P'_accu - RU32(delta *
// tilde-log2(max_h cbar))) (the accurate-mode formula of Section 2.3).
__global__ __launch_bounds__(256) void k1_accurate_exponent(
    const int32_t* __restrict__ e1, const int32_t* __restrict__ cmax, int64_t nvec,
    const ModTable* __restrict__ tab, int32_t* __restrict__ e_out) {
  const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (v >= nvec) return;
  const int32_t a = e1[v];
  int32_t e;
  if (a == kExpNonFinite) e = kExpNonFinite;
  else if (a == kExpZero) e = 0;
  else e = accurate_exponent(a, (int64_t)cmax[v], tab->p_prop, tab->delta);
  e_out[v] = e;
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

// Status word reset at the start of each call (a kernel, not a memset, so
// the call can be captured in a graph).
// Both operands in one launch (the two halves are independent, so at small
// sizes they overlap instead of running one after the other): blocks
// [0, nA) take the rows of A (nA = gAx x ceil(nchunks / 4) blocks of the
// strided kernel's grid), the others the columns of B.  Block 0 also clears
// the status word, which only later launches read or write.
// NT = false (small problems): ordinary loads, so that the operands stay in
// the caches for the conversion kernel.
template <typename T, bool NT = true>
__global__ __launch_bounds__(256) void k1_partials_ab(
    const T* __restrict__ A, int64_t lda, int64_t m, const T* __restrict__ B, int64_t ldb,
    int64_t n, int64_t k, int64_t nchunks, double* __restrict__ partA,
    double* __restrict__ maxA, double* __restrict__ partB, double* __restrict__ maxB,
    int64_t gAx, int64_t nA, int* __restrict__ status) {
  const int64_t b = blockIdx.x;
  if (b == 0 && threadIdx.x == 0) status[0] = 0;
  if (b < nA)
    k1_partials_strided_body<T, false, NT>(A, lda, m, k, nchunks, partA, maxA, b % gAx, b / gAx);
  else
    k1_partials_contig_body<T>(B, ldb, n, k, nchunks, partB, maxB, b - nA);
}

// Both folds in one launch: blocks [0, nA) for the rows of A, the rest for
// the columns of B.
__global__ __launch_bounds__(256) void k1_fold_ab(
    const double* __restrict__ partA, const double* __restrict__ maxA, int64_t m,
    int32_t* __restrict__ eA, double* __restrict__ SA, const double* __restrict__ partB,
    const double* __restrict__ maxB, int64_t n, int32_t* __restrict__ eB,
    double* __restrict__ SB, int64_t nchunks, int mode, const ModTable* __restrict__ tab,
    int* __restrict__ status, int64_t nA) {
  const int64_t b = blockIdx.x;
  if (b < nA) k1_fold_body(partA, maxA, nchunks, m, mode, tab, eA, SA, status, b);
  else k1_fold_body(partB, maxB, nchunks, n, mode, tab, eB, SB, status, b - nA);
}

__global__ void k_clear_status(int* status) {
  if (threadIdx.x == 0) status[0] = 0;
}

// Exhaustive-check hook for the binary32 log2 of the scaling.
__global__ void k_log2f(const float* __restrict__ x, float* __restrict__ y, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] = log2_rn32(x[i]);
}

}  // namespace oz2
