// oz2_k3_gemm.hpp -- K3: the N INT8 matrix products of Step 3,
//   C_t = rmod(A', p_t) rmod(B', p_t)   (INT8 x INT8 -> exact INT32),
// on gfx950 MFMA (v_mfma_i32_32x32x32_i8); all planes and tiles of a call
// in one 1-D grid.
//
// Operands: plane t of RA is Mp x Kp and plane t of RB is Np x Kp, both with
// the k index contiguous, so C_t = RA_t RB_t^T.  A workgroup of 256 lanes
// (2 x 2 waves) computes a BM x BN tile; each wave owns (BM/2) x (BN/2) as
// TM x TN blocks of 32 x 32.  Slabs of BK bytes of k are staged through LDS
// (double-buffered; 16-byte chunks XOR-swizzled by row so that the 16-byte
// fragment reads of a 32-row block hit distinct banks) and the next slab's
// global loads are in flight while the current one feeds the MFMAs.
//
// Epilogue: for odd p_t, |C_t| <= k 127^2 < 2^31 for k <= 2^17 (Section 2.2),
// so the INT32 sum is exact; plane 0 (p = 256, residues in [-128, 127]) can
// reach k 128^2 = 2^31 there and is exact modulo 2^32, which keeps its low
// byte -- all that is used of it -- exact.  The product is reduced to U_t = rmod(C_t, p_t) in [-(p_t-1)/2, (p_t-1)/2] (for
// p_t = 256 the low byte, in [-128, 127]) and stored as one signed byte
// per entry, in 32 x 32 blocks laid out in the MFMA accumulator order: block
// (bi, bj) of plane t is 1024 contiguous bytes at ((t Nb + bj) Mb + bi) * 1024
// (Mb = Mp/32, Nb = Np/32), lane l's 16 accumulators at byte 16 l.  K4 reads
// the same order, so the stores and loads are 16 contiguous bytes per lane.
// Other epilogues (EPI): 1 stores the raw INT32 product of one plane (test
// hook); 2 (accurate mode's scale GEMM on the bar planes, Section 2.3) does
// not store the product at all: it folds it into row and column maxima with
// integer atomicMax (entries are >= 0, and the maxima start at 0); 3 is EPI 0
// for a later block of k (k > 2^17 is split into blocks whose INT32 products
// are exact): U_t = rmod(U_t + rmod(C_t, p_t), p_t).
#pragma once

#include <type_traits>

#include "oz2_math.hpp"
#include "oz2_tables.hpp"

namespace oz2 {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// Accumulator layout of a 32 x 32 INT32 MFMA block: register r of lane l
// holds row acc_row(r, l), column acc_col(l).
OZ2_HD int acc_row(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }
OZ2_HD int acc_col(int lane) { return lane & 31; }

// 16-byte chunk swizzle inside an LDS row of BK bytes.
template <int BK>
__device__ __forceinline__ int swz_chunk(int row, int chunk) {
  if constexpr (BK == 128) return chunk ^ ((row >> 1) & 7);
  else return chunk ^ ((row >> 2) & 3);
}

// Map a workgroup id to (plane, tile).  Workgroups are dispatched
// round-robin over the 8 XCDs of MI355X (id mod 8), each XCD with its own L2,
// all sharing the MALL (Infinity Cache).  When the tile grid allows it, ids
// are taken in rounds of 256: in a round XCD x computes an 8 x 4 group of
// tiles (32 tiles sharing 8 row panels of A and 4 column panels of B in its
// L2), and the 8 groups of the round form one (8 XM) x (4 XN) block of tiles
// of the same plane (XM XN = 8; 32 x 8 preferred, else 16 x 16, else
// 8 x 32), so the XCDs fetch neighbouring panels at the same time and share
// them through the MALL.  Rounds sweep a band of 8 XM tile rows column block
// by column block, then the next band, then the next plane.  Other grids
// fall back to giving each XCD one contiguous range of the (plane, tile)
// sequence, walked in groups of 8 tile rows.
template <int XM>
__device__ __forceinline__ bool tile_of_rounds(int id, int tiles_m, int tiles_n, int* plane,
                                               int* tm, int* tn) {
  constexpr int XN = 8 / XM;
  if (tiles_m % (8 * XM) != 0 || tiles_n % (4 * XN) != 0) return false;
  const int x = id & 7, slot = id >> 3, r = slot >> 5, s = slot & 31;
  const int rpp = tiles_m * tiles_n / 256;    // rounds per plane
  const int rpb = tiles_n / (4 * XN);         // rounds per band
  *plane = r / rpp;
  const int rr = r - *plane * rpp, band = rr / rpb, c = rr - band * rpb;
  *tm = band * 8 * XM + (x / XN) * 8 + (s & 7);
  *tn = c * 4 * XN + (x % XN) * 4 + (s >> 3);
  return true;
}

__device__ __forceinline__ void tile_of(int id, int total, int tiles_m, int tiles_n,
                                        int* plane, int* tm, int* tn) {
  if (tile_of_rounds<4>(id, tiles_m, tiles_n, plane, tm, tn)) return;
  if (tile_of_rounds<2>(id, tiles_m, tiles_n, plane, tm, tn)) return;
  if (tile_of_rounds<1>(id, tiles_m, tiles_n, plane, tm, tn)) return;
  const int xcd = id & 7, slot = id >> 3;
  const int per = total >> 3, extra = total & 7;
  const int lin = (xcd < extra) ? xcd * (per + 1) + slot
                                : extra * (per + 1) + (xcd - extra) * per + slot;
  const int tiles = tiles_m * tiles_n;
  *plane = lin / tiles;
  const int in_plane = lin - *plane * tiles;
  constexpr int GM = 8;
  const int group = in_plane / (GM * tiles_n);
  const int first_m = group * GM;
  const int gm = tiles_m - first_m < GM ? tiles_m - first_m : GM;
  const int in = in_plane - group * GM * tiles_n;
  *tm = first_m + in % gm;
  *tn = in / gm;
}

// Global -> LDS copy of 16 bytes per lane without a register round trip
// (global_load_lds_dwordx4): lane l of the wave writes dst + 16 l, dst being
// wave-uniform.  The asm waits carry a memory clobber so that the compiler
// does not move LDS reads across them.
__device__ __forceinline__ void load_lds16(const int8_t* src, int8_t* dst) {
#if defined(__HIP_DEVICE_COMPILE__)
  __builtin_amdgcn_global_load_lds(src, dst, 16, 0, 0);
#endif
}
__device__ __forceinline__ void wait_vmem_all() {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
#endif
}
template <int N>
__device__ __forceinline__ void wait_vmem_n() {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
#endif
}
__device__ __forceinline__ void wait_vmem_lds_all() {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");
#endif
}

// The epilogue of a BM x BN tile whose wave (wm, wn) holds the exact INT32
// products of its (BM/2) x (BN/2) part in acc (TM x TN blocks of 32 x 32 in
// the MFMA accumulator layout): EPI 0 stores U_t = C_t mod p_t, EPI 1 the raw
// product, EPI 2 folds it into row and column maxima, EPI 3 adds C_t mod p_t
// to U_t (see the top of this file).
template <int BM, int BN, int EPI>
__device__ __forceinline__ void tile_epilogue(
    const v16i (&acc)[BM / 64][BN / 64], uint8_t* __restrict__ U, int32_t* __restrict__ aux0,
    int32_t* __restrict__ aux1, int64_t m, int64_t n, int64_t Mp, int64_t Np,
    const ModTable* __restrict__ tab, int t, int tm, int tn, int wm, int wn, int lane) {
  constexpr int TM = BM / 64, TN = BN / 64;
  const int64_t Mb = Mp / 32;
  if constexpr (EPI == 1) {
    int32_t* Craw = aux0;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int64_t col = (int64_t)tn * BN + wn * (BN / 2) + j * 32 + acc_col(lane);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int64_t row = (int64_t)tm * BM + wm * (BM / 2) + i * 32 + acc_row(r, lane);
          if (row < m && col < n) Craw[row + col * m] = acc[i][j][r];
        }
      }
    return;
  }
  if constexpr (EPI == 2) {
    int32_t* rmax = aux0;   // per row of the product (Mp entries)
    int32_t* cmax = aux1;   // per column (Np entries)
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        int v = acc[i][0][r];
#pragma unroll
        for (int j = 1; j < TN; ++j) v = v > acc[i][j][r] ? v : acc[i][j][r];
#pragma unroll
        for (int o = 1; o < 32; o <<= 1) {
          int u = __shfl_xor(v, o);
          v = v > u ? v : u;
        }
        if ((lane & 31) == 0)
          atomicMax(rmax + (int64_t)tm * BM + wm * (BM / 2) + i * 32 + acc_row(r, lane), v);
      }
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      int v = acc[0][j][0];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int r = 0; r < 16; ++r) v = v > acc[i][j][r] ? v : acc[i][j][r];
      int u = __shfl_xor(v, 32);
      v = v > u ? v : u;
      if (lane < 32) atomicMax(cmax + (int64_t)tn * BN + wn * (BN / 2) + j * 32 + acc_col(lane), v);
    }
    return;
  }
  const int64_t Nb = Np / 32;
  const bool is256 = (t == 0);
  const double p = tab->p[t], ip = tab->inv_p[t];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      uint32_t w[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        uint32_t u[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int c = acc[i][j][4 * q + e];
          if (is256) {
            u[e] = (uint32_t)c;                   // the low byte is kept
          } else {
            // symmetric residue, |r| <= (p-1)/2 (one instruction fewer per
            // entry than rounding c / p and converting the remainder back);
            // its two's-complement byte is kept
            u[e] = residue_sym_i32(c, p, ip);
          }
        }
        w[q] = pack_low_bytes(u[0], u[1], u[2], u[3]);
      }
      const int64_t bi = (int64_t)tm * (BM / 32) + wm * (TM) + i;
      const int64_t bj = (int64_t)tn * (BN / 32) + wn * (TN) + j;
      uint8_t* dst = U + (((int64_t)t * Nb + bj) * Mb + bi) * 1024 + lane * 16;
      if constexpr (EPI == 3) {
        // a later k block: U = rmod(U + rmod(C, p), p), byte by byte (the
        // low byte of the sum for p = 256)
        const uint4 o = *reinterpret_cast<const uint4*>(dst);
        const uint32_t ow[4] = {o.x, o.y, o.z, o.w};
        const int pi = (int)p, half = (int)p >> 1;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          uint32_t b = 0;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            int v = (int)(int8_t)(ow[q] >> (8 * e)) + (int)(int8_t)(w[q] >> (8 * e));
            if (!is256) v = v > half ? v - pi : (v < -half ? v + pi : v);
            b |= ((uint32_t)v & 0xFFu) << (8 * e);
          }
          w[q] = b;
        }
      }
      *reinterpret_cast<uint4*>(dst) = make_uint4(w[0], w[1], w[2], w[3]);
    }
}

// One BM x BN output tile of plane t (tile row tm, tile column tn).
//
// Main loop: one BK-byte k slab per iteration (128 bytes for the plain tiles,
// 64 for the batched one), two LDS buffers, BK / 32 MFMA k steps per slab.
// The instruction order is fixed explicitly (a scheduling fence after every
// MFMA and the memory operations paired with it), because with one wave per
// SIMD every stall of the in-order issue is a bubble of the matrix core:
//   * in k step kk, the TM + TN fragment reads of step kk + 1 follow the
//     first TM + TN MFMAs, one after each, in the order the i-major MFMAs
//     consume them;
//   * EARLY_BARRIER (the default for 256 x 256 tiles): in the last k step,
//     after a few MFMAs, the wave waits for its own loads and LDS reads and
//     meets the others at the slab barrier; the next slab is then complete in
//     LDS and the current buffer is free, and the next slab's step-0 fragment
//     reads follow the remaining MFMAs.  The next slab's global->LDS loads:
//     LX = 8 of them ride on MFMAs of the previous slab's last k step right
//     after its barrier (their buffer is free from then on), the others on
//     k steps 0 and 1, so they have two to four k steps to land (measured
//     1-4% faster than issuing all of them in k steps 0 and 1).  So no k step
//     waits for a fragment read issued less than a step earlier, and the
//     barrier sits among MFMAs instead of in front of them;
//   * otherwise (the smaller tiles: fewer MFMAs per k step, two or three
//     workgroups per CU) the barrier is at the top of the slab and the next
//     slab's loads are spread over LSTEPS k steps (measured best for them).
// Lane l of wave w in load round i fills LDS slot 16 (i 256 + 64 w + l); the
// slot's row and swizzled chunk decide which 16 source bytes it fetches.  The
// last slabs are separate copies of the body without the loads (and reads
// ahead) that have no slab to target, so that every slab body is one basic
// block without conditional loads.
//
// PF (persistent callers, barrier at the slab top only): the tile starts in
// LDS buffer buf0, its first slab already loaded there if `loaded`; during
// its last slab it issues the first slab of the caller's next tile (nA, nB:
// that tile's row panels of A and B; nKp its row length; null: no next tile)
// into the other buffer, which no wave reads any more once all have passed
// the last slab's barrier, so those loads fly during the last MFMAs and the
// epilogue.  Returns the buffer holding the next tile's first slab.
template <int BM, int BN, int BK, int EPI, bool EARLY_BARRIER = (BM >= 256 && BN >= 256),
          int LSTEPS = (EARLY_BARRIER ? 2 : 3), int LX = (EARLY_BARRIER ? 8 : 0), bool PF = false>
__device__ __forceinline__ int gemm_tile(
    const int8_t* __restrict__ RA, const int8_t* __restrict__ RB,
    uint8_t* __restrict__ U, int32_t* __restrict__ aux0, int32_t* __restrict__ aux1,
    int64_t m, int64_t n, int64_t Mp, int64_t Np, int64_t Kp,
    const ModTable* __restrict__ tab, int t, int tm, int tn,
    int8_t (*__restrict__ lds)[(BM + BN) * BK], int64_t k0 = 0, int64_t klen = -1,
    int buf0 = 0, bool loaded = false, const int8_t* nA = nullptr, const int8_t* nB = nullptr,
    int64_t nKp = 0) {
  static_assert(!PF || !EARLY_BARRIER, "prefetch across tiles needs the slab-top barrier");
  constexpr int TM = BM / 64, TN = BN / 64;      // 32x32 blocks per wave
  constexpr int CH = BK / 16;                    // 16-byte chunks per row
  constexpr int A_LOADS = BM * CH / 256, B_LOADS = BN * CH / 256;
  constexpr int KS = BK / 32;                    // MFMA k steps per slab
  static_assert(A_LOADS * 256 == BM * CH && B_LOADS * 256 == BN * CH, "tile");

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  // k columns [k0, k0 + klen) of the planes (rows of Kp bytes); klen < 0: all
  const int8_t* gA = RA + (int64_t)t * Mp * Kp + (int64_t)tm * BM * Kp + k0;
  const int8_t* gB = RB + (int64_t)t * Np * Kp + (int64_t)tn * BN * Kp + k0;
  if (klen < 0) klen = Kp;

  v16i acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = v16i{0};

  // Source offset of each of this lane's load slots (fixed across slabs).
  int64_t offA[A_LOADS], offB[B_LOADS];
#pragma unroll
  for (int i = 0; i < A_LOADS; ++i) {
    const int s = i * 256 + tid, row = s / CH;
    offA[i] = (int64_t)row * Kp + swz_chunk<BK>(row, s % CH) * 16;  // XOR: an involution
  }
#pragma unroll
  for (int i = 0; i < B_LOADS; ++i) {
    const int s = i * 256 + tid, row = s / CH;
    offB[i] = (int64_t)row * Kp + swz_chunk<BK>(row, s % CH) * 16;
  }
  // Load round i (A rounds first, then B) of slab k0 into buffer buf.
  auto gload1 = [&](int buf, int64_t k0, int i) {
    if (i < A_LOADS)
      load_lds16(gA + offA[i] + k0, lds[buf] + (i * 256 + wave * 64) * 16);
    else
      load_lds16(gB + offB[i - A_LOADS] + k0,
                 lds[buf] + BM * BK + ((i - A_LOADS) * 256 + wave * 64) * 16);
  };

  // Load round i of the caller's next tile's first slab into buffer buf.
  auto gload_next1 = [&](int buf, int i) {
    if (i < A_LOADS) {
      const int s = i * 256 + tid, row = s / CH;
      load_lds16(nA + (int64_t)row * nKp + swz_chunk<BK>(row, s % CH) * 16,
                 lds[buf] + (i * 256 + wave * 64) * 16);
    } else {
      const int s = (i - A_LOADS) * 256 + tid, row = s / CH;
      load_lds16(nB + (int64_t)row * nKp + swz_chunk<BK>(row, s % CH) * 16,
                 lds[buf] + BM * BK + ((i - A_LOADS) * 256 + wave * 64) * 16);
    }
  };

  // Fragment q (TM blocks of A, then TN blocks of B) of k step kk of LDS
  // buffer buf into register set F.
  v4i fa[2][TM], fb[2][TN];
  auto fread_q = [&](int buf, int kk, int F, int q) {
    const int ch = kk * 2 + (lane >> 5);
    if (q < TM) {
      const int8_t* sA = lds[buf] + (wm * (BM / 2)) * BK;
      const int row = q * 32 + (lane & 31);
      fa[F][q] = *reinterpret_cast<const v4i*>(sA + row * BK + swz_chunk<BK>(row, ch) * 16);
    } else {
      const int8_t* sB = lds[buf] + BM * BK + (wn * (BN / 2)) * BK;
      const int row = (q - TM) * 32 + (lane & 31);
      fb[F][q - TM] = *reinterpret_cast<const v4i*>(sB + row * BK + swz_chunk<BK>(row, ch) * 16);
    }
  };
  // The r-th read of a k step: in the order the MFMAs (i-major) consume the
  // fragments -- A0, B0 .. B(TN-1), then A1 .. A(TM-1).
  auto fread1 = [&](int buf, int kk, int F, int r) {
    fread_q(buf, kk, F, r == 0 ? 0 : (r <= TN ? TM + r - 1 : r - TN));
  };

  // LX (early-barrier mode only): the first LX loads of slab kt + 2 are
  // issued in slab kt's last k step right after the barrier (the buffer of
  // slab kt is free from then on), giving them about four k steps to land;
  // the other LOADS - LX loads of a slab go out in k steps 0..LSTEPS-1 of the
  // slab before it.
  constexpr int NM = TM * TN, NF = TM + TN, LOADS = A_LOADS + B_LOADS;
  constexpr int LY = LOADS - LX;                      // loads in steps 0..LSTEPS-1
  constexpr int PER = (LY + LSTEPS - 1) / LSTEPS;     // loads per loading step
  constexpr int SP = PER > 0 ? NM / PER : NM;         // MFMAs per load
  constexpr int BAR = (NM - NF) < 5 ? ((NM - NF) > 0 ? (NM - NF) : 0) : 5;  // MFMAs before it
  static_assert(KS % 2 == 0 && (!EARLY_BARRIER || BAR + NF <= NM), "schedule shape");
  static_assert(LSTEPS <= (EARLY_BARRIER ? KS - 1 : KS), "loads land before the barrier");
  static_assert(SP >= 1 && PER * LSTEPS >= LY, "loads fit the MFMA slots");
  static_assert(LX == 0 || (EARLY_BARRIER && LX <= NM - BAR - 1 && LX <= 63), "early loads");

  const int nk = (int)(klen / BK);
  if (!PF || !loaded) {
#pragma unroll
    for (int i = 0; i < LOADS; ++i) gload1(PF ? buf0 : 0, 0, i);
  }
  if constexpr (EARLY_BARRIER) {
    if (LX > 0 && nk > 1) {
#pragma unroll
      for (int i = 0; i < LX; ++i) gload1(1, BK, i);
      wait_vmem_n<LX>();  // slab 0 has landed; slab 1's first loads may not
    } else {
      wait_vmem_all();
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NF; ++q) fread1(0, 0, 0, q);
  }
  // One slab.  MORE: a next slab exists (load the rest of it, meet at the
  // barrier, read ahead); MORE2: a slab after that exists (its first LX
  // loads); NEXT (last slab, PF): load the next tile's first slab.
  // Separate copies, so that each stays one basic block.
  int buf = PF ? buf0 : 0;
  auto slab = [&](int kt, auto more_tag, auto more2_tag, auto next_tag) {
    constexpr bool MORE = decltype(more_tag)::value;
    constexpr bool MORE2 = decltype(more2_tag)::value;
    constexpr bool NEXT = decltype(next_tag)::value;
    const int64_t knext = (int64_t)(kt + 1) * BK;
    if constexpr (!EARLY_BARRIER) {
      // Barrier at the top of the slab: slab kt is in LDS and every wave is
      // done with the buffer the next loads overwrite.
      wait_vmem_lds_all();
      __syncthreads();
#pragma unroll
      for (int q = 0; q < NF; ++q) fread1(buf, 0, 0, q);
    }
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
      const int F = kk & 1;
#pragma unroll
      for (int idx = 0; idx < NM; ++idx) {
        if (MORE && EARLY_BARRIER && kk == KS - 1 && idx == BAR) {
          wait_vmem_lds_all();
          __syncthreads();
        }
        const int i = idx / TN, j = idx % TN;
        acc[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[F][i], fb[F][j], acc[i][j], 0, 0, 0);
        if (kk + 1 < KS) {
          // next step's fragments: one after each MFMA, the rest after the last
          if (idx + 1 < NM) {
            if (idx < NF) fread1(buf, kk + 1, F ^ 1, idx);
          } else {
#pragma unroll
            for (int q = idx; q < NF; ++q) fread1(buf, kk + 1, F ^ 1, q);
          }
        }
        if (MORE && kk < LSTEPS && PER > 0 && idx % SP == SP - 1) {
          const int g = LX + kk * PER + idx / SP;
          if (g < LOADS) gload1(buf ^ 1, knext, g);
        }
        if (NEXT && kk < LSTEPS && PER > 0 && idx % SP == SP - 1) {
          const int g = kk * PER + idx / SP;
          if (g < LOADS) gload_next1(buf ^ 1, g);
        }
        if (MORE && EARLY_BARRIER && kk == KS - 1 && idx >= BAR && idx < BAR + NF)
          fread1(buf ^ 1, 0, 0, idx - BAR);
        if (MORE2 && LX > 0 && kk == KS - 1 && idx > BAR && idx <= BAR + LX)
          gload1(buf, knext + BK, idx - BAR - 1);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    buf ^= 1;
  };
  int kt = 0;
  for (; kt + 2 < nk; ++kt) slab(kt, std::true_type{}, std::true_type{}, std::false_type{});
  if (nk >= 2) slab(nk - 2, std::true_type{}, std::false_type{}, std::false_type{});
  if (PF && nA) {
    slab(nk - 1, std::false_type{}, std::false_type{}, std::bool_constant<PF>{});
  } else {
    slab(nk - 1, std::false_type{}, std::false_type{}, std::false_type{});
    wait_vmem_all();  // no load may still target LDS when the tile returns
  }

  tile_epilogue<BM, BN, EPI>(acc, U, aux0, aux1, m, n, Mp, Np, tab, t, tm, tn, wm, wn, lane);
  return buf;
}

template <int BM, int BN, int BK, int EPI>
__global__ __launch_bounds__(256) void k3_gemm_i8(
    const int8_t* __restrict__ RA, const int8_t* __restrict__ RB,
    uint8_t* __restrict__ U, int32_t* __restrict__ aux0, int32_t* __restrict__ aux1,
    int64_t m, int64_t n, int64_t Mp, int64_t Np, int64_t Kp,
    const ModTable* __restrict__ tab, int t_raw, int64_t k0, int64_t klen) {
  __shared__ __attribute__((aligned(16))) int8_t lds[2][(BM + BN) * BK];
  const int tiles_m = (int)(Mp / BM), tiles_n = (int)(Np / BN);
  int plane, tm, tn;
  tile_of(blockIdx.x, gridDim.x, tiles_m, tiles_n, &plane, &tm, &tn);
  const int t = (EPI == 1 || EPI == 2) ? t_raw : plane;
  gemm_tile<BM, BN, BK, EPI>(RA, RB, U, aux0, aux1, m, n, Mp, Np, Kp, tab, t, tm, tn, lds, k0,
                             klen);
}

}  // namespace oz2
