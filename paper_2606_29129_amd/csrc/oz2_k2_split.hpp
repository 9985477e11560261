// oz2_k2_split.hpp -- K2: Step 2 and the residue part of Step 3.
//
// For every entry a of a row (column) with exponent e: a' = trunc(a 2^e)
// (exact in binary64: a power-of-two scaling then a truncation), then the N
// INT8 residues of a' -- rmod(a', p) in [-(p-1)/2, (p-1)/2] for odd p, and
// the two's-complement low byte for p = 256 (congruent to rmod(a', 256); rmod
// itself can give +128, which INT8 cannot hold).
//
// Residues: a' is split into signed 40-bit limbs, a' = sum_j x_j 2^(40 j)
// (all limbs carry the sign of a', |x_j| < 2^40), so a' = y (mod p) with
// y = sum_j x_j (2^(40 j) mod p).  The fast modes have |a'| < 2^79 (two
// limbs, |x_1| < 2^39): |y| < 2^40 + 2^47; accurate mode has |a'| < 2^86
// (three limbs): |y| < 2^40 + 2^48 + 2^14.  So y is exact in binary64, and
// q = round(y / p) found from y RN(1/p) is exact as well: the estimate's
// error, |y / p| 2^-52 < 2^-3 / p, stays below the 1 / (2p) distance of y / p
// from a half-integer.  r = y - q p is the symmetric residue, with no
// correction step.  It is formed around 1.5 2^52, where the unit is 1:
// fma(y, RN(1/p), 1.5 2^52) = 1.5 2^52 + q (the product is exact inside the
// fma); fma(1.5 2^52 + q, -p, 1.5 2^52 (p + 1)) = 1.5 2^52 - q p and adding y
// gives 1.5 2^52 + r, both exact (every value is an integer in [2^52, 2^53));
// the low word of that encoding is r in two's complement.  Two fmas and an
// add, against a multiply, a rounding, an fma and a conversion.
//
// Output layout: plane t is a (Vp x Kp) int8 matrix, vector-major with the
// k index contiguous (what the GEMM reads); padding rows and columns are 0.
#pragma once

#include "oz2_k1_norm.hpp"
#include "oz2_tables.hpp"

namespace oz2 {

template <int LIMBS>
struct Limbs {
  double x[LIMBS];
};

template <int LIMBS>
OZ2_HD Limbs<LIMBS> make_limbs(double a, int32_t e) {
  Limbs<LIMBS> L;
  double v = (e == kExpNonFinite) ? 0.0 : trunc(ldexp(a, e));
  if (!(v == v)) v = 0.0;  // NaN entries of a flagged row give 0
#pragma unroll
  for (int j = LIMBS - 1; j >= 1; --j) {
    const double scale = ldexp(1.0, kLimbBits * j);
    double q = trunc(v * (1.0 / scale));
    v = fma(-q, scale, v);
    L.x[j] = q;
  }
  L.x[0] = v;
  return L;
}

template <int LIMBS>
OZ2_HD int residue_odd(const Limbs<LIMBS>& L, const double* pw, double p, double inv_p) {
  double y = L.x[0];
#pragma unroll
  for (int j = 1; j < LIMBS; ++j) y = fma(L.x[j], pw[j], y);
  constexpr double kMagic = 0x1.8p52;
  const double tq = fma(y, inv_p, kMagic);           // 1.5 2^52 + q
  const double s = fma(tq, -p, kMagic * (p + 1.0));  // 1.5 2^52 - q p (exact)
  return (int)(uint32_t)f64_to_bits(s + y);          // 1.5 2^52 + r: low word r
}

// a' = x_0 (mod 256) since 256 divides 2^40.  x_0 (|x_0| < 2^40) does not
// fit an int32; x_0 + 1.5 2^52 is exact and lies in [2^52, 2^53), where the
// integer significand is x_0 + 2^51 + 2^52, so the low 32 bits of its
// encoding are x_0 modulo 2^32 in two's complement: the residue is their low
// byte (the higher bits are not part of the result).
template <int LIMBS>
OZ2_HD uint32_t residue_256_byte(const Limbs<LIMBS>& L) {
  return (uint32_t)f64_to_bits(L.x[0] + 0x1.8p52);
}

// The same residue as a signed value in [-128, 127].
template <int LIMBS>
OZ2_HD int residue_256(const Limbs<LIMBS>& L) {
  return (int)(int8_t)(uint8_t)residue_256_byte<LIMBS>(L);
}

// Residues in plane t of EPT entries (limbs L), packed four to a dword in
// entry order.
template <int LIMBS, int EPT>
__device__ __forceinline__ void pack_residues(const Limbs<LIMBS> (&L)[EPT], int t,
                                              const ModTable* __restrict__ tab,
                                              uint32_t (&w)[EPT / 4]) {
  if (t == 0) {  // modulus 0 is 256
#pragma unroll
    for (int q = 0; q < EPT / 4; ++q)
      w[q] = pack_low_bytes(residue_256_byte<LIMBS>(L[4 * q]),
                            residue_256_byte<LIMBS>(L[4 * q + 1]),
                            residue_256_byte<LIMBS>(L[4 * q + 2]),
                            residue_256_byte<LIMBS>(L[4 * q + 3]));
  } else {
    const double p = tab->p[t], ip = tab->inv_p[t];
    const double* pw = tab->powL[t];
#pragma unroll
    for (int q = 0; q < EPT / 4; ++q)
      w[q] = pack_low_bytes(residue_odd<LIMBS>(L[4 * q], pw, p, ip),
                            residue_odd<LIMBS>(L[4 * q + 1], pw, p, ip),
                            residue_odd<LIMBS>(L[4 * q + 2], pw, p, ip),
                            residue_odd<LIMBS>(L[4 * q + 3], pw, p, ip));
  }
}

// Streaming accesses: the residue planes (N bytes per entry, far beyond the
// caches) are written once here and read by the GEMM much later, and the
// strided operand is read once; non-temporal loads and stores keep them from
// displacing other lines (measured 12% faster for the strided kernel, 2.5%
// for the contiguous one's stores; non-temporal loads slow the contiguous
// kernel's 64-byte-per-lane reads, so it keeps ordinary loads).
typedef unsigned int nt_u4 __attribute__((ext_vector_type(4)));
typedef unsigned int nt_u2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void nt_store(int8_t* dst, uint4 v) {
  __builtin_nontemporal_store(nt_u4{v.x, v.y, v.z, v.w}, reinterpret_cast<nt_u4*>(dst));
}
__device__ __forceinline__ void nt_store(int8_t* dst, uint2 v) {
  __builtin_nontemporal_store(nt_u2{v.x, v.y}, reinterpret_cast<nt_u2*>(dst));
}
__device__ __forceinline__ void nt_store(int8_t* dst, uint32_t v) {
  __builtin_nontemporal_store(v, reinterpret_cast<uint32_t*>(dst));
}
template <typename T>
__device__ __forceinline__ double nt_load(const T* p) {
  return (double)__builtin_nontemporal_load(p);
}

// NT = false (small problems): ordinary loads and stores, so that the
// operands stay in the caches for the next kernel that reads them and the
// residue planes for the GEMM.
template <bool NT, typename V>
__device__ __forceinline__ void store_out(int8_t* dst, V v) {
  if constexpr (NT) nt_store(dst, v);
  else *reinterpret_cast<V*>(dst) = v;
}
template <bool NT, typename T>
__device__ __forceinline__ double load_in(const T* p) {
  if constexpr (NT) return nt_load(p);
  else return (double)*p;
}

template <int EPT, bool NT = true>
__device__ __forceinline__ void store_packed(int8_t* dst, const uint32_t (&w)[EPT / 4]) {
  if constexpr (EPT == 4) store_out<NT>(dst, w[0]);
  else if constexpr (EPT == 8) store_out<NT>(dst, make_uint2(w[0], w[1]));
  else store_out<NT>(dst, make_uint4(w[0], w[1], w[2], w[3]));
}

// Strided vectors (rows of column-major A): entry h of vector v at
// X[v + h ld].  A block of 256 lanes covers VB vectors x (256 / VB) * EPS
// entries: lane = (vector tid % VB, entry group tid / VB), so each load
// instruction reads VB consecutive entries of a column per group; every lane
// converts EPS entries (16; 8 for small problems, twice the blocks).  Per
// plane the block's residue bytes are staged in LDS (rows padded by one
// group: conflict-free writes; two buffers, one barrier per plane) and
// written out as whole rows of (256 / VB) * EPS bytes.
constexpr int kK2VB = 32;                       // vectors per strided block
constexpr int kK2HB = (256 / kK2VB) * 16;       // entries per strided block (EPS 16)
constexpr int kK2HBSmall = (256 / kK2VB) * 8;   // (EPS 8)

template <int EPS>
struct K2Chunk;
template <>
struct K2Chunk<16> {
  typedef uint4 type;
  static __device__ __forceinline__ uint4 make(const uint32_t (&w)[4]) {
    return make_uint4(w[0], w[1], w[2], w[3]);
  }
};
template <>
struct K2Chunk<8> {
  typedef uint2 type;
  static __device__ __forceinline__ uint2 make(const uint32_t (&w)[2]) {
    return make_uint2(w[0], w[1]);
  }
};

template <typename T, int LIMBS, int VB = kK2VB, int EPS = 16, bool NT = true>
__device__ __forceinline__ void k2_split_strided_body(
    const T* __restrict__ X, int64_t ld, int64_t nvec, int64_t k,
    const int32_t* __restrict__ e, const ModTable* __restrict__ tab, int N,
    int8_t* __restrict__ R, int64_t Vp, int64_t Kp, int64_t bx, int64_t by) {
  constexpr int G = 256 / VB, HB = G * EPS;
  static_assert(VB * G == 256 && (VB * HB / EPS) == 256, "one write-out pass");
  typedef typename K2Chunk<EPS>::type Chunk;
  __shared__ Chunk stage[2][VB][G + 1];
  const int vl = threadIdx.x % VB, g = threadIdx.x / VB;
  const int64_t v0 = bx * VB, v = v0 + vl;
  const int64_t h0 = by * HB + g * EPS;
  const int32_t ev = v < nvec ? e[v] : 0;
  Limbs<LIMBS> L[EPS];
  {
    double a[EPS];
#pragma unroll
    for (int i = 0; i < EPS; ++i)
      a[i] = (v < nvec && h0 + i < k) ? load_in<NT>(X + v + (h0 + i) * ld) : 0.0;
#pragma unroll
    for (int i = 0; i < EPS; ++i) L[i] = make_limbs<LIMBS>(a[i], ev);
  }
  const int64_t plane = Vp * Kp;
  const int orow = threadIdx.x / G, ochunk = threadIdx.x % G;  // write-out mapping
  int8_t* out = R + (v0 + orow) * Kp + by * HB + ochunk * EPS;
  for (int t = 0; t < N; ++t) {
    const int sb = t & 1;
    uint32_t w[EPS / 4];
    pack_residues<LIMBS, EPS>(L, t, tab, w);
    stage[sb][vl][g] = K2Chunk<EPS>::make(w);
    __syncthreads();
    store_out<NT>(out + (int64_t)t * plane, stage[sb][orow][ochunk]);
  }
}

template <typename T, int LIMBS>
__global__ __launch_bounds__(256) void k2_split_strided(
    const T* __restrict__ X, int64_t ld, int64_t nvec, int64_t k,
    const int32_t* __restrict__ e, const ModTable* __restrict__ tab, int N,
    int8_t* __restrict__ R, int64_t Vp, int64_t Kp) {
  k2_split_strided_body<T, LIMBS>(X, ld, nvec, k, e, tab, N, R, Vp, Kp, blockIdx.x, blockIdx.y);
}

// Contiguous vectors (columns of column-major B): entry h of vector v at
// X[h + v ld].  One lane per (vector, group of EPT consecutive entries):
// neighbouring lanes read and write neighbouring groups, EPT-byte stores.
constexpr int kK2EPT = 8;

template <typename T, int LIMBS, int EPT = kK2EPT, bool NT = true>
__device__ __forceinline__ void k2_split_contig_body(
    const T* __restrict__ X, int64_t ld, int64_t nvec, int64_t k,
    const int32_t* __restrict__ e, const ModTable* __restrict__ tab, int N,
    int8_t* __restrict__ R, int64_t Vp, int64_t Kp, int64_t bx) {
  const int64_t groups = Kp / EPT;
  const int64_t gi = bx * 256 + threadIdx.x;
  if (gi >= Vp * groups) return;
  const int64_t v = gi / groups;
  const int64_t h0 = (gi - v * groups) * EPT;
  const int32_t ev = v < nvec ? e[v] : 0;
  Limbs<LIMBS> L[EPT];
  {
    double a[EPT];
    const T* p = X + v * ld + h0;
#pragma unroll
    for (int i = 0; i < EPT; ++i) a[i] = (v < nvec && h0 + i < k) ? (double)p[i] : 0.0;
#pragma unroll
    for (int i = 0; i < EPT; ++i) L[i] = make_limbs<LIMBS>(a[i], ev);
  }
  int8_t* out = R + v * Kp + h0;
  const int64_t plane = Vp * Kp;
  for (int t = 0; t < N; ++t) {
    uint32_t w[EPT / 4];
    pack_residues<LIMBS, EPT>(L, t, tab, w);
    store_packed<EPT, NT>(out + (int64_t)t * plane, w);
  }
}

template <typename T, int LIMBS>
__global__ __launch_bounds__(256) void k2_split_contig(
    const T* __restrict__ X, int64_t ld, int64_t nvec, int64_t k,
    const int32_t* __restrict__ e, const ModTable* __restrict__ tab, int N,
    int8_t* __restrict__ R, int64_t Vp, int64_t Kp) {
  k2_split_contig_body<T, LIMBS>(X, ld, nvec, k, e, tab, N, R, Vp, Kp, blockIdx.x);
}

// Both operands in one launch: blocks [0, nA) run the strided kernel's
// blocks for A (nA = gAx x Kp / kK2HB, gAx = Mp / kK2VB), the others the
// contiguous kernel's blocks for B.
template <typename T, int LIMBS, int EPS = 16, bool NT = true>
__global__ __launch_bounds__(256) void k2_split_ab(
    const T* __restrict__ A, int64_t lda, int64_t m, const int32_t* __restrict__ eA,
    int8_t* __restrict__ RA, int64_t Mp, const T* __restrict__ B, int64_t ldb, int64_t n,
    const int32_t* __restrict__ eB, int8_t* __restrict__ RB, int64_t Np, int64_t k,
    const ModTable* __restrict__ tab, int N, int64_t Kp, int64_t gAx, int64_t nA) {
  const int64_t b = blockIdx.x;
  if (b < nA)
    k2_split_strided_body<T, LIMBS, kK2VB, EPS, NT>(A, lda, m, k, eA, tab, N, RA, Mp, Kp,
                                                    b % gAx, b / gAx);
  else
    k2_split_contig_body<T, LIMBS, kK2EPT, NT>(B, ldb, n, k, eB, tab, N, RB, Np, Kp, b - nA);
}

// Accurate mode: abar = ceil(|a| 2^e') in [0, 64] (Section 2.3), one int8
// plane in the GEMM layout.  Vectors with exponent kExpZero or
// kExpNonFinite give zeros.
OZ2_HD int8_t bar_value(double a, int32_t e) {
  if (e == kExpZero || e == kExpNonFinite) return 0;
  double v = ceil(ldexp(fabs(a), e));
  return (int8_t)(v == v ? v : 0.0);
}

// Bar plane of the strided operand: the geometry of k2_split_strided (VB
// vectors x (256 / VB) 16 entries per block, one LDS staging pass).
template <typename T, int VB = kK2VB>
__global__ __launch_bounds__(256) void k2_bar_strided(
    const T* __restrict__ X, int64_t ld, int64_t nvec, int64_t k,
    const int32_t* __restrict__ e, int8_t* __restrict__ R, int64_t Vp, int64_t Kp) {
  constexpr int G = 256 / VB, HB = G * 16;
  __shared__ uint4 stage[VB][G + 1];
  const int vl = threadIdx.x % VB, g = threadIdx.x / VB;
  const int64_t v0 = (int64_t)blockIdx.x * VB, v = v0 + vl;
  const int64_t h0 = (int64_t)blockIdx.y * HB + g * 16;
  const int32_t ev = v < nvec ? e[v] : kExpZero;
  double a[16];
#pragma unroll
  for (int i = 0; i < 16; ++i)
    a[i] = (v < nvec && h0 + i < k) ? (double)X[v + (h0 + i) * ld] : 0.0;
  uint32_t w[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    uint32_t b = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) b |= (uint32_t)(uint8_t)bar_value(a[4 * q + i], ev) << (8 * i);
    w[q] = b;
  }
  stage[vl][g] = make_uint4(w[0], w[1], w[2], w[3]);
  __syncthreads();
  const int orow = threadIdx.x / G, ochunk = threadIdx.x % G;
  *reinterpret_cast<uint4*>(R + (v0 + orow) * Kp + (int64_t)blockIdx.y * HB + ochunk * 16) =
      stage[orow][ochunk];
}

// Bar plane of the contiguous operand: one lane per kK2EPT consecutive
// entries, as k2_split_contig.
template <typename T, int EPT = kK2EPT>
__global__ __launch_bounds__(256) void k2_bar_contig(
    const T* __restrict__ X, int64_t ld, int64_t nvec, int64_t k,
    const int32_t* __restrict__ e, int8_t* __restrict__ R, int64_t Vp, int64_t Kp) {
  const int64_t groups = Kp / EPT;
  const int64_t gi = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (gi >= Vp * groups) return;
  const int64_t v = gi / groups;
  const int64_t h0 = (gi - v * groups) * EPT;
  const int32_t ev = v < nvec ? e[v] : kExpZero;
  double a[EPT];
  const T* p = X + v * ld + h0;
#pragma unroll
  for (int i = 0; i < EPT; ++i) a[i] = (v < nvec && h0 + i < k) ? (double)p[i] : 0.0;
  uint32_t w[EPT / 4];
#pragma unroll
  for (int q = 0; q < EPT / 4; ++q) {
    uint32_t b = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) b |= (uint32_t)(uint8_t)bar_value(a[4 * q + i], ev) << (8 * i);
    w[q] = b;
  }
  store_packed<EPT>(R + v * Kp + h0, w);
}

}  // namespace oz2
