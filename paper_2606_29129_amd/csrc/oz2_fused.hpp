// oz2_fused.hpp -- K2 for A, K3 and K4 in one kernel when n <= 64.
//
// For a narrow B (n <= 64 columns) the unfused path is bound by memory: K2
// writes N residue bytes per entry of A, K3 reads them back once (a single
// tile column), and K4 reads the N product planes.  Here a wave owns 16 rows
// of C and all n <= 64 columns for every modulus at once (16 x 64 INT32
// accumulators per plane: 16 registers per lane, 16 planes at most), so it
//   * reads its rows of A (binary64) once, k step by k step, and forms the
//     integers and residues in registers (K2's arithmetic, Step 2 and the
//     residue part of Step 3);
//   * multiplies them with the residues of B (made by K2 beforehand, staged
//     through LDS, shared by the four waves of a workgroup) on
//     v_mfma_i32_16x16x64_i8;
//   * reduces every product modulo p_t and reconstructs and unscales the
//     results in registers (K4's arithmetic, Step 3's CRT and Step 4),
//     writing C directly.
// No residue plane of A and no product plane is stored.  The results are the
// unfused path's, bit for bit.
//
// 16x16x64 INT8 MFMA lane layout (checked on the device): lane l supplies
// row l % 16 of A and column l % 16 of B with the 16 k bytes of group l / 16;
// accumulator r of lane l is row 4 (l / 16) + r, column l % 16.
#pragma once

#include <utility>

#include "oz2_k1_norm.hpp"
#include "oz2_k2_split.hpp"
#include "oz2_k3_gemm.hpp"
#include "oz2_k4_crt.hpp"

namespace oz2 {

constexpr int kFuseCols = 64;   // n <= kFuseCols
constexpr int kFuseMaxN = 16;   // moduli: every plane's accumulators stay in registers
constexpr int kFuseK = 64;      // k per step (one MFMA)
constexpr int kFuseRows = 64;   // rows of C per workgroup (4 waves x 16)

// 16-byte chunk position of logical k chunk g in the LDS row of column c
// (rows of 64 bytes): spreads the 16-byte fragment reads of 8 consecutive
// columns over distinct banks.
__device__ __forceinline__ int fuse_swz(int c, int g) { return g ^ ((c >> 1) & 3); }

// Number of 39-bit CRT slices for the first NP moduli (P < 2^128 for NP <= 16),
// as the host tables compute it.
constexpr int fuse_slices(int NP) {
  unsigned __int128 P = 1;
  for (int t = 0; t < NP; ++t) P *= (unsigned)kModuli[t];
  int bits = 0;
  while (P) { ++bits; P >>= 1; }
  return (bits + kSliceBits - 1) / kSliceBits;
}

// 2^40 mod p (the weight of the high limb) and RN(1/p), as the host tables
// compute them, at compile time: the moduli of the fused kernel are template
// constants, so their constants need no table loads in the inner loop.
constexpr double fuse_pow40(int p) {
  unsigned long long r = 1;
  for (int i = 0; i < kLimbBits; ++i) r = (r * 2) % (unsigned long long)p;
  return (double)r;
}

template <typename F, int... I>
__device__ __forceinline__ void fuse_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
// f(integral_constant<int, t>) for t = 0 .. NP-1, in order.
template <int NP, typename F>
__device__ __forceinline__ void fuse_for(F&& f) {
  fuse_for_impl(f, std::make_integer_sequence<int, NP>{});
}

// Residue of a' (two limbs) for modulus index t, in the low byte of the
// result (what the packing reads): as residue_256_byte / residue_odd with
// the table values of modulus t.
template <int t>
__device__ __forceinline__ int fuse_residue(const Limbs<2>& L) {
  if constexpr (t == 0) {
    return (int)residue_256_byte<2>(L);
  } else {
    constexpr double p = (double)kModuli[t], ip = 1.0 / (double)kModuli[t];
    constexpr double c1 = fuse_pow40(kModuli[t]);
    const double y = fma(L.x[1], sconst(c1), L.x[0]);
    const double q = rint(y * ip);
    return (int)fma(-q, p, y);
  }
}

// Limbs of trunc(a 2^e) for this kernel, whose residues of A are never
// stored.  A row with a non-finite entry (exponent sentinel) gets a very
// negative exponent instead, so that its finite entries truncate to 0, and
// every value is clamped to [-2^78, 2^78] (infinities; NaNs too, since the
// minimum and maximum return the operand that is not a NaN): its residues
// are well-defined integers, and its outputs are NaN whatever its products
// are.  For every other row |a'| < 2^64 (P < 2^128 for N <= 16), so the clamp
// changes nothing and the limbs are make_limbs<2>'s.
__device__ __forceinline__ Limbs<2> fuse_limbs(double a, int32_t e) {
  const double v =
      __builtin_fmin(__builtin_fmax(trunc(ldexp(a, e)), sconst(-0x1p78)), sconst(0x1p78));
  Limbs<2> L;
  L.x[1] = trunc(v * 0x1p-40);
  L.x[0] = fma(-L.x[1], 0x1p40, v);
  return L;
}

// NP = N (a template parameter, so that every accumulator access and product
// is unconditional and the accumulators stay in the accumulation registers).
template <typename T, typename TO, int NP>
__global__ __launch_bounds__(256) void k234_fused(
    const T* __restrict__ A, int64_t lda, int64_t m, int64_t n, int64_t k,
    const int32_t* __restrict__ eA, const int32_t* __restrict__ eB,
    const int8_t* __restrict__ RB, int64_t Np, int64_t Kp,
    const ModTable* __restrict__ tab, TO* __restrict__ C, int64_t ldc) {
  static_assert(NP >= 2 && NP <= kFuseMaxN, "moduli");
  constexpr int S = fuse_slices(NP);
  constexpr int N = NP;
  constexpr int PB = kFuseCols * kFuseK;   // bytes of B residues per plane and step
  __shared__ __attribute__((aligned(16))) int8_t lds[2][NP * PB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t row0 = (int64_t)blockIdx.x * kFuseRows + wave * 16;
  const int64_t arow = row0 + (lane & 15);           // the row of A this lane converts
  const bool rowok = arow < m;
  // rows beyond m convert to zero through the non-finite sentinel (their
  // outputs are never written)
  const int32_t ea0 = rowok ? eA[arow] : kExpNonFinite;
  const int32_t ea = ea0 == kExpNonFinite ? -2000 : ea0;   // see fuse_limbs
  const T* Ap = A + (rowok ? arow : 0);               // clamped: every load in bounds
  const int kq = (lane >> 4) * 16;                    // this lane's k bytes in a step

  // B slab of a step: lane tid fills LDS slot tid of every plane, column
  // tid / 4, stored chunk tid % 4 (holding logical chunk fuse_swz(col, tid % 4),
  // the swizzle being an involution).
  const int bcol = tid >> 2;
  const int64_t boff = (int64_t)bcol * Kp + fuse_swz(bcol, tid & 3) * 16;
  auto load_b = [&](int buf, int64_t k0) {
#pragma unroll
    for (int t = 0; t < NP; ++t)
      load_lds16(RB + (int64_t)t * Np * Kp + boff + k0, lds[buf] + t * PB + wave * 64 * 16);
  };
  // A values of a step: 16 consecutive k of one row, lda apart.  Only the
  // last step can run past k: there out-of-range k reads the last column
  // (in bounds) and the value is zeroed when used.
  auto load_a = [&](int64_t k0, double (&raw)[16]) {
    const int64_t kb = k0 + kq;
    if (kb + 16 <= k) {
      const T* p = Ap + kb * lda;
#pragma unroll
      for (int j = 0; j < 16; ++j) raw[j] = (double)__builtin_nontemporal_load(p + j * lda);
    } else {
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int64_t kk = kb + j;
        const int64_t kc = kk < k ? kk : k - 1;
        raw[j] = (double)__builtin_nontemporal_load(Ap + kc * lda);
      }
    }
  };

  v4i acc[NP][4];
#pragma unroll
  for (int t = 0; t < NP; ++t)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) acc[t][cb] = v4i{0, 0, 0, 0};

  const int nsteps = (int)(Kp / kFuseK);
  double raw[16];
  load_b(0, 0);
  load_a(0, raw);
  for (int s = 0; s < nsteps; ++s) {
    const int buf = s & 1;
    const int64_t k0 = (int64_t)s * kFuseK;
    if (k0 + kq + 16 > k) {
#pragma unroll
      for (int j = 0; j < 16; ++j)
        if (k0 + kq + j >= k) raw[j] = 0.0;
    }
    Limbs<2> L[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) L[j] = fuse_limbs(raw[j], ea);
    const bool more = s + 1 < nsteps;
    if (more) {
      load_a(k0 + kFuseK, raw);
      wait_vmem_n<16>();   // all but the 16 A loads just issued: slab s is in LDS
    } else {
      wait_vmem_all();
    }
    __syncthreads();       // every wave's part of slab s; every wave done with slab s - 1
    if (more) load_b(buf ^ 1, k0 + kFuseK);
    // One plane at a time (fences keep the scheduler from hoisting every
    // plane's work, which would exhaust the registers): the plane's four
    // fragment reads first, so that its residue arithmetic covers their
    // latency, then the products.
    fuse_for<NP>([&](auto tc) {
      constexpr int t = decltype(tc)::value;
      v4i bf[4];
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        const int col = cb * 16 + (lane & 15);
        bf[cb] = *reinterpret_cast<const v4i*>(lds[buf] + t * PB + col * kFuseK +
                                               fuse_swz(col, lane >> 4) * 16);
      }
      __builtin_amdgcn_sched_barrier(0);
      uint32_t w[4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        w[q] = pack_low_bytes(fuse_residue<t>(L[4 * q]), fuse_residue<t>(L[4 * q + 1]),
                              fuse_residue<t>(L[4 * q + 2]), fuse_residue<t>(L[4 * q + 3]));
      const v4i af = {(int)w[0], (int)w[1], (int)w[2], (int)w[3]};
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
        acc[t][cb] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af, bf[cb], acc[t][cb], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
    });
  }

  // Epilogue: per output, U_t = C_t mod p_t in [0, p_t) (as the GEMM's own
  // epilogue computes it), the exact CRT sum, reconstruction and unscaling
  // (as K4 does).
  const ModTable& TB = *tab;
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
    const int64_t col = cb * 16 + (lane & 15);
    const int32_t f = col < n ? eB[col] : 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = row0 + 4 * (lane >> 4) + r;
      double X[S];
#pragma unroll
      for (int q = 0; q < S; ++q) X[q] = 0.0;
#pragma unroll
      for (int t = 0; t < NP; ++t) {
        const int c = acc[t][cb][r];
        double u;
        if (t == 0) {
          u = (double)((uint32_t)c & 0xFFu);
        } else {
          const double y = (double)c;
          const double rr = fma(-rint(y * TB.inv_p[t]), TB.p[t], y);  // exact
          u = rr < 0.0 ? rr + TB.p[t] : rr;
        }
#pragma unroll
        for (int q = 0; q < S; ++q) X[q] = fma(TB.w[t][q], u, X[q]);
      }
      if (row < m && col < n) {
        const int32_t e = eA[row];
        double v;
        if (e == kExpNonFinite || f == kExpNonFinite) v = __builtin_nan("");
        else if constexpr (sizeof(TO) == 8) v = crt_unscale<S, 53, -1074>(X, TB, e + f);
        else v = crt_unscale<S, 24, -149>(X, TB, e + f);
        C[row + col * ldc] = (TO)v;
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

}  // namespace oz2
