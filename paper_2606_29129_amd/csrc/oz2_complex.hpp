// oz2_complex.hpp -- complex products (ZGEMM, CGEMM) on the real pipeline.
//
// The scaling of Algorithm 2 (or 1) is applied to a complex row (column) as
// to the real vector of its 2k components in storage order (re, im, re, ...):
// its squared 2-norm is sum_h |a_h|^2, and since |Re(ab)|, |Im(ab)| <= |a||b|
// both parts of every entry of A'B' stay within sum_h |a'_h||b'_h| <=
// ||a'|| ||b'||, the bound the scaling keeps below P/2 (Section 4; Section 1
// notes that the same scaling serves the complex fast mode).  Both parts of
// an entry are truncated with the row's (column's) exponent.
//
// Per modulus the complex residue product takes three INT8 GEMMs (Gauss /
// Karatsuba): with A' = X + iY and B' = U + iV,
//   G0 = X U,  G1 = Y V,  G2 = (X + Y)(U + V),
//   Re A'B' = G0 - G1,  Im A'B' = G2 - G0 - G1   (mod p_t),
// where X + Y and U + V are formed from the residues (reduced back into the
// INT8 range).  K2 writes three residue planes per modulus (component c at
// plane c N + t), K3 runs unchanged over each component's N planes, and K4
// forms the residues of both parts from the three uint8 planes, then
// reconstructs and unscales each part as in the real case.
#pragma once

#include "oz2_k1_norm.hpp"
#include "oz2_k2_split.hpp"
#include "oz2_k3_gemm.hpp"
#include "oz2_k4_crt.hpp"

namespace oz2 {

template <typename T>
struct Cplx;
template <>
struct Cplx<double> { using type = double2; };
template <>
struct Cplx<float> { using type = float2; };

// --- K1: rows of a column-major complex matrix ------------------------------
// Entry h of vector v is the pair at X2[v + h ld] (ld in complex entries).
// Chunks of kKC components = kKC / 2 complex entries, each summed in storage
// order (re^2, then im^2, entry by entry); one lane per vector, one wave per
// chunk as in the real strided kernel.  The columns of complex B need no
// kernel of their own: their components are contiguous, so the real
// contiguous kernel runs over 2k components with leading dimension 2 ldb.
// RESC: the exact mode's fallback pass (vectors marked kExpRescale only,
// entries scaled down), as in the real kernels.
template <typename T, bool RESC = false>
__global__ __launch_bounds__(256) void k1_partials_strided_cplx(
    const T* __restrict__ X, int64_t ld, int64_t nvec, int64_t k, int64_t nchunks,
    double* __restrict__ part, double* __restrict__ pmax,
    const int32_t* __restrict__ esel = nullptr) {
  using T2 = typename Cplx<T>::type;
  constexpr int KH = kKC / 2;
  const int lane = threadIdx.x & 63;
  const int64_t v = (int64_t)blockIdx.x * 64 + lane;
  const int64_t c = (int64_t)blockIdx.y * 4 + (threadIdx.x >> 6);
  if (v >= nvec || c >= nchunks) return;
  if (RESC && esel[v] != kExpRescale) return;
  const int64_t h0 = c * KH;
  const int64_t len = k - h0 < KH ? k - h0 : KH;
  const T2* p = reinterpret_cast<const T2*>(X) + v + h0 * ld;
  double s = 0.0, mx = 0.0;
  auto add = [&](T2 z) {
    const double a = norm_entry<RESC>((double)z.x), b = norm_entry<RESC>((double)z.y);
    s = ru_add(s, ru_square(a));
    s = ru_add(s, ru_square(b));
    mx = fmax(mx, fmax(fabs(a), fabs(b)));
  };
  if (len == KH) {
#pragma unroll
    for (int b = 0; b < KH; b += 8) {
      T2 z[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) z[i] = p[(int64_t)(b + i) * ld];
#pragma unroll
      for (int i = 0; i < 8; ++i) add(z[i]);
    }
  } else {
    for (int64_t h = 0; h < len; ++h) add(p[h * ld]);
  }
  part[c * nvec + v] = s;
  if (pmax) pmax[c * nvec + v] = mx;
}

// --- K2: residues of the three components ----------------------------------

// Residue of x (limbs L) for modulus t, in the INT8 range.
template <int LIMBS>
__device__ __forceinline__ int residue_t(const Limbs<LIMBS>& L, int t,
                                         const ModTable* __restrict__ tab) {
  if (t == 0) return residue_256<LIMBS>(L);
  return residue_odd<LIMBS>(L, tab->powL[t], tab->p[t], tab->inv_p[t]);
}

// x + y for two residues of modulus t, reduced back into the INT8 range:
// the low byte for 256, the symmetric range for odd p.
__device__ __forceinline__ int residue_sum(int x, int y, int t, int p) {
  int s = x + y;
  if (t == 0) return (int)(int8_t)(uint8_t)(s & 0xFF);
  const int h = (p - 1) >> 1;
  s = s > h ? s - p : s;
  return s < -h ? s + p : s;
}

// EPL complex entries (limbs of both parts) -> three packed words of EPL
// bytes (EPL = 8: uint2) for modulus t.
template <int LIMBS, int EPL>
__device__ __forceinline__ void pack_cplx(const Limbs<LIMBS> (&Lr)[EPL],
                                          const Limbs<LIMBS> (&Li)[EPL], int t,
                                          const ModTable* __restrict__ tab, uint2 (&w)[3]) {
  static_assert(EPL == 8, "two dwords per component");
  const int p = (int)tab->p[t];
  uint32_t v[3][EPL];
#pragma unroll
  for (int i = 0; i < EPL; ++i) {
    const int x = residue_t<LIMBS>(Lr[i], t, tab);
    const int y = residue_t<LIMBS>(Li[i], t, tab);
    v[0][i] = (uint32_t)x;
    v[1][i] = (uint32_t)y;
    v[2][i] = (uint32_t)residue_sum(x, y, t, p);
  }
#pragma unroll
  for (int c = 0; c < 3; ++c)
    w[c] = make_uint2(pack_low_bytes(v[c][0], v[c][1], v[c][2], v[c][3]),
                      pack_low_bytes(v[c][4], v[c][5], v[c][6], v[c][7]));
}

// Strided complex vectors (rows of column-major A).  A block covers 32
// vectors x 64 complex entries: lane = (vector tid % 32, group tid / 32 of 8
// entries), so each load instruction reads 32 consecutive complex entries of
// a column (512 or 256 contiguous bytes).  Per modulus the three components'
// bytes are staged in LDS and written out as 32 rows x 64 bytes per plane.
// 1-D grid: block b covers vector block b % gx and k block b / gx.
constexpr int kK2CVB = 32;   // vectors per block
constexpr int kK2CEPL = 8;   // complex entries per lane
constexpr int kK2CHB = (256 / kK2CVB) * kK2CEPL;   // complex entries per block (64)

template <typename T, int LIMBS>
__global__ __launch_bounds__(256) void k2_split_strided_cplx(
    const T* __restrict__ X, int64_t ld, int64_t nvec, int64_t k,
    const int32_t* __restrict__ e, const ModTable* __restrict__ tab, int N,
    int8_t* __restrict__ R, int64_t Vp, int64_t Kp, int64_t gx) {
  using T2 = typename Cplx<T>::type;
  constexpr int VB = kK2CVB, G = 256 / VB, EPL = kK2CEPL, HB = kK2CHB;
  __shared__ uint2 stage[2][3][VB][G + 1];
  const int64_t bx = (int64_t)blockIdx.x % gx, by = (int64_t)blockIdx.x / gx;
  const int vl = threadIdx.x % VB, g = threadIdx.x / VB;
  const int64_t v0 = bx * VB, v = v0 + vl;
  const int64_t h0 = by * HB + g * EPL;
  const int32_t ev = v < nvec ? e[v] : 0;
  Limbs<LIMBS> Lr[EPL], Li[EPL];
  {
    const T2* p = reinterpret_cast<const T2*>(X);
    T2 z[EPL];
#pragma unroll
    for (int i = 0; i < EPL; ++i) {
      if (v < nvec && h0 + i < k) z[i] = p[v + (h0 + i) * ld];
      else { z[i].x = 0; z[i].y = 0; }
    }
#pragma unroll
    for (int i = 0; i < EPL; ++i) {
      Lr[i] = make_limbs<LIMBS>((double)z[i].x, ev);
      Li[i] = make_limbs<LIMBS>((double)z[i].y, ev);
    }
  }
  const int64_t plane = Vp * Kp;
  const int orow = threadIdx.x / G, ochunk = threadIdx.x % G;   // 32 rows x 8 x 8 bytes
  int8_t* out = R + (v0 + orow) * Kp + by * HB + ochunk * 8;
  for (int t = 0; t < N; ++t) {
    const int sb = t & 1;
    uint2 w[3];
    pack_cplx<LIMBS, EPL>(Lr, Li, t, tab, w);
#pragma unroll
    for (int c = 0; c < 3; ++c) stage[sb][c][vl][g] = w[c];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c)
      nt_store(out + (int64_t)(c * N + t) * plane, stage[sb][c][orow][ochunk]);
  }
}

// Contiguous complex vectors (columns of column-major B): one lane per
// (vector, group of 8 consecutive complex entries); 8-byte stores per plane.
template <typename T, int LIMBS>
__global__ __launch_bounds__(256) void k2_split_contig_cplx(
    const T* __restrict__ X, int64_t ld, int64_t nvec, int64_t k,
    const int32_t* __restrict__ e, const ModTable* __restrict__ tab, int N,
    int8_t* __restrict__ R, int64_t Vp, int64_t Kp) {
  using T2 = typename Cplx<T>::type;
  constexpr int EPL = kK2CEPL;
  const int64_t groups = Kp / EPL;
  const int64_t gi = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (gi >= Vp * groups) return;
  const int64_t v = gi / groups;
  const int64_t h0 = (gi - v * groups) * EPL;
  const int32_t ev = v < nvec ? e[v] : 0;
  Limbs<LIMBS> Lr[EPL], Li[EPL];
  {
    const T2* p = reinterpret_cast<const T2*>(X) + v * ld + h0;
    T2 z[EPL];
#pragma unroll
    for (int i = 0; i < EPL; ++i) {
      if (v < nvec && h0 + i < k) z[i] = p[i];
      else { z[i].x = 0; z[i].y = 0; }
    }
#pragma unroll
    for (int i = 0; i < EPL; ++i) {
      Lr[i] = make_limbs<LIMBS>((double)z[i].x, ev);
      Li[i] = make_limbs<LIMBS>((double)z[i].y, ev);
    }
  }
  int8_t* out = R + v * Kp + h0;
  const int64_t plane = Vp * Kp;
  for (int t = 0; t < N; ++t) {
    uint2 w[3];
    pack_cplx<LIMBS, EPL>(Lr, Li, t, tab, w);
#pragma unroll
    for (int c = 0; c < 3; ++c)
      nt_store(out + (int64_t)(c * N + t) * plane, w[c]);
  }
}

// --- K4: both parts from the three planes ----------------------------------
// U holds 3N planes (component c, modulus t at plane c N + t), each
// rmod(C, p_t) as a signed byte in the GEMM's 32 x 32 block order.  For each
// entry and modulus re = U0 - U1 and im = U2 - U0 - U1, congruent to the two
// parts modulo p_t and below 2^9 in magnitude, so the slice sums stay below
// 2^53 (exact) as in the real case.  One wave per
// 32 x 32 block; the lane's 16 accumulator-order entries in PASSES passes
// (two accumulator sets, re and im).  Each entry is stored as one (re, im)
// pair.
template <int S, typename TO>
__global__ __launch_bounds__(256) void k4_crt_cplx(
    const uint8_t* __restrict__ U, const int32_t* __restrict__ eA,
    const int32_t* __restrict__ eB, const ModTable* __restrict__ tab, int N,
    int64_t m, int64_t n, int64_t Mp, int64_t Np, TO* __restrict__ C, int64_t ldc) {
  using T2 = typename Cplx<TO>::type;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t Mb = Mp / 32, Nb = Np / 32;
  const int64_t blk = (int64_t)blockIdx.x * 4 + wave;
  const int64_t mb_used = (m + 31) / 32;
  const int64_t nb_used = (n + 31) / 32;
  if (blk >= mb_used * nb_used) return;
  const int64_t bi = blk % mb_used, bj = blk / mb_used;
  const uint8_t* src = U + (bj * Mb + bi) * 1024 + lane * 16;
  const int64_t plane = Nb * Mb * 1024;
  const int64_t comp = (int64_t)N * plane;
  const int lc = acc_col(lane);
  const int64_t col = bj * 32 + lc;
  const int32_t f = col < n ? eB[col] : 0;
  const ModTable& T = *tab;
  T2* C2 = reinterpret_cast<T2*>(C);
  constexpr int PASSES = S >= 4 ? 4 : 2, R = 16 / PASSES;
#pragma unroll
  for (int h = 0; h < PASSES; ++h) {
    double ar[R][S], ai[R][S];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int s = 0; s < S; ++s) ar[r][s] = ai[r][s] = 0.0;
    for (int t = 0; t < N; ++t) {
      uint32_t w[3][R / 4];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const uint8_t* q = src + c * comp + (int64_t)t * plane + R * h;
        if constexpr (R == 8) {
          const uint2 x = *reinterpret_cast<const uint2*>(q);
          w[c][0] = x.x;
          w[c][1] = x.y;
        } else {
          w[c][0] = *reinterpret_cast<const uint32_t*>(q);
        }
      }
      double wt[S];
#pragma unroll
      for (int s = 0; s < S; ++s) wt[s] = T.w[t][s];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int sh = 8 * (r & 3);
        const int u0 = (int)(int8_t)(w[0][r >> 2] >> sh);
        const int u1 = (int)(int8_t)(w[1][r >> 2] >> sh);
        const int u2 = (int)(int8_t)(w[2][r >> 2] >> sh);
        const int re = u0 - u1;
        const int im = u2 - u0 - u1;
#pragma unroll
        for (int s = 0; s < S; ++s) {
          ar[r][s] = fma(wt[s], (double)re, ar[r][s]);
          ai[r][s] = fma(wt[s], (double)im, ai[r][s]);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t row = bi * 32 + acc_row(R * h + r, lane);
      if (row < m && col < n) {
        const int32_t e = eA[row];
        T2 out;
        if (e == kExpNonFinite || f == kExpNonFinite) {
          out.x = out.y = (TO)__builtin_nan("");
        } else {
          double a[S], b[S];
#pragma unroll
          for (int s = 0; s < S; ++s) {
            a[s] = ar[r][s];
            b[s] = ai[r][s];
          }
          if constexpr (sizeof(TO) == 8) {
            out.x = crt_unscale<S, 53, -1074>(a, T, e + f);
            out.y = crt_unscale<S, 53, -1074>(b, T, e + f);
          } else {
            out.x = (TO)crt_unscale<S, 24, -149>(a, T, e + f);
            out.y = (TO)crt_unscale<S, 24, -149>(b, T, e + f);
          }
        }
        C2[row + col * ldc] = out;
      }
    }
  }
}

}  // namespace oz2
