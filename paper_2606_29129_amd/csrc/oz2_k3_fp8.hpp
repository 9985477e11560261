// oz2_k3_fp8.hpp -- the residue products of Step 3 on the FP8 (E4M3) matrix
// engine: v_mfma_f32_32x32x64_f8f6f4 with binary32 accumulation.
//
// The paper notes that its scaling carries over to Ozaki scheme II on FP8
// engines (Section 1) and leaves that extension open (Section 6).  Here the
// scaling, the integers, the INT8 residues, the CRT and the unscaling are
// those of the INT8 path; only the products C_t = RA_t RB_t^T change engine,
// and they come out identical, so C is bit-identical to the INT8 path's.
//
// Digits.  E4M3 holds every integer up to 16 in magnitude, a residue reaches
// 128, so each residue r is split as r = 16 h + l, l = ((r + 8) mod 16) - 8
// in [-8, 7], h in [-8, 8]; the engine operands are the E4M3 values 16 h and
// l.  Then r_A r_B = (16h_A)(16h_B) + (16h_A) l_B + l_A (16h_B) + l_A l_B:
// four MFMAs per 64 indices of k into one binary32 accumulator.  The four
// terms of one index add up in magnitude to at most 136^2, so after 512
// indices every partial sum, in whatever order the engine adds, is an
// integer below 512 * 136^2 < 2^24: exact.  Every 512 indices (8 slabs) the
// accumulator is converted (exactly) to INT32 and added to the INT32
// product, which the INT8 path's epilogues then reduce and store.
//
// Digit planes.  Plane t of operand X (Vp rows) is Vp x 2Kp bytes: for each
// 64 indices c of k, 64 codes of 16 h then 64 codes of l (a 128-byte chunk
// holding both digit operands of those indices).  k_fp8_digits writes them
// from the INT8 residue planes.
//
// Operand layout.  A lane gives the MFMA 32 bytes of its row (A) or column
// (B); the 64 indices of a step are split between the two lane halves.
// Whatever index each byte position stands for, A and B use the same
// position for the same index (both fragments are read from the same chunk
// offsets), so the engine sums exactly the 64 products of the step.
#pragma once

#include "oz2_k3_gemm.hpp"

namespace oz2 {

typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int kF8Tile = 128;      // BM = BN of the FP8 GEMM tile
constexpr int kF8SlabK = 64;      // indices of k per LDS slab (128 bytes per row)
constexpr int kF8DumpSlabs = 8;   // slabs per exact binary32 block (512 indices)

// E4M3 code of an integer digit v in [-8, 8] (shift 0) or of 16 v (shift 4:
// the exponent field is 4 higher; 0 stays 0).  Codes of the magnitudes
// 0..7 as bytes of one word: 0x00, 0x38 (1), 0x40 (2), 0x44 (3), 0x48 (4),
// 0x4A (5), 0x4C (6), 0x4E (7); 8 is 0x50.
OZ2_HD uint32_t e4m3_small(int v, int shift) {
  const uint32_t a = (uint32_t)(v < 0 ? -v : v);
  uint32_t c = a == 8 ? 0x50u : (uint32_t)((0x4E4C4A4844403800ull >> (8 * a)) & 0xFFu);
  if (c) c += (uint32_t)shift << 3;
  return c | (v < 0 ? 0x80u : 0u);
}

// INT8 residue planes (planes x Vp x Kp, k contiguous) to digit planes
// (planes x Vp x 2Kp, layout above).  One thread per 16 residues.
__global__ __launch_bounds__(256) void k_fp8_digits(const int8_t* __restrict__ R,
                                                    uint8_t* __restrict__ F, int64_t rows,
                                                    int64_t Kp) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;   // group of 16 residues
  const int64_t per_row = Kp / 16;
  if (g >= rows * per_row) return;
  const int64_t row = g / per_row, kb = (g - row * per_row) * 16;
  const v4i in = __builtin_nontemporal_load(reinterpret_cast<const v4i*>(R + row * Kp + kb));
  const uint32_t w[4] = {(uint32_t)in[0], (uint32_t)in[1], (uint32_t)in[2], (uint32_t)in[3]};
  uint32_t hw[4], lw[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    uint32_t hb = 0, lb = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = (int)(int8_t)(uint8_t)(w[q] >> (8 * e));
      const int l = ((r + 8) & 15) - 8;
      const int h = (r - l) >> 4;
      hb |= e4m3_small(h, 4) << (8 * e);
      lb |= e4m3_small(l, 0) << (8 * e);
    }
    hw[q] = hb;
    lw[q] = lb;
  }
  uint8_t* out = F + row * 2 * Kp + (kb / kF8SlabK) * 128 + (kb % kF8SlabK);
  __builtin_nontemporal_store(v4i{(int)hw[0], (int)hw[1], (int)hw[2], (int)hw[3]},
                              reinterpret_cast<v4i*>(out));
  __builtin_nontemporal_store(v4i{(int)lw[0], (int)lw[1], (int)lw[2], (int)lw[3]},
                              reinterpret_cast<v4i*>(out + 64));
}

// One 128 x 128 output tile of plane t on the FP8 engine: 4 waves (2 x 2),
// each 64 x 64 as 2 x 2 blocks of 32 x 32.  Slabs of 64 indices (128 bytes
// per row: both digit operands) are staged through LDS, double-buffered, the
// next slab's global->LDS loads in flight while the current one feeds the
// MFMAs; the barrier sits at the top of each slab.  k columns [k0, k0 + klen)
// of the residue index (klen a multiple of 64, at most 2^17).
template <int EPI>
__device__ __forceinline__ void gemm_tile_f8(const uint8_t* __restrict__ FA,
                                             const uint8_t* __restrict__ FB,
                                             uint8_t* __restrict__ U, int32_t* __restrict__ aux0,
                                             int64_t m, int64_t n, int64_t Mp, int64_t Np,
                                             int64_t Kp, const ModTable* __restrict__ tab, int t,
                                             int tm, int tn, uint8_t (*__restrict__ lds)[2 * kF8Tile * 128],
                                             int64_t k0, int64_t klen) {
  constexpr int BM = kF8Tile, BN = kF8Tile, TM = 2, TN = 2, ROWB = 128, CH = ROWB / 16;
  constexpr int LOADS = (BM + BN) * CH / 256;   // 16-byte loads per lane per slab
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t rowbytes = 2 * Kp;
  const uint8_t* gA = FA + (int64_t)t * Mp * rowbytes + (int64_t)tm * BM * rowbytes + 2 * k0;
  const uint8_t* gB = FB + (int64_t)t * Np * rowbytes + (int64_t)tn * BN * rowbytes + 2 * k0;

  // Load slot i of this lane: LDS chunk s = i 256 + tid (rows 0..BM-1 of A,
  // then BN rows of B), source chunk swizzled by row (an involution).
  int64_t off[LOADS];
#pragma unroll
  for (int i = 0; i < LOADS; ++i) {
    const int s = i * 256 + tid, row = s / CH, r = row < BM ? row : row - BM;
    off[i] = (int64_t)r * rowbytes + swz_chunk<ROWB>(r, s % CH) * 16;
  }
  auto gload = [&](int buf, int64_t kb) {   // kb: byte offset of the slab in a row
#pragma unroll
    for (int i = 0; i < LOADS; ++i) {
      const int s = i * 256 + tid, row = s / CH;
      const uint8_t* src = (row < BM ? gA : gB) + off[i] + kb;
      load_lds16(reinterpret_cast<const int8_t*>(src),
                 reinterpret_cast<int8_t*>(lds[buf] + (i * 256 + wave * 64) * 16));
    }
  };
  // 32-byte fragment of digit d (0: 16h, 1: l) of block q of A (q < TM) or
  // B: chunks 4 d + 2 (lane / 32) and the one after it of its row.
  auto frag = [&](int buf, int q, int d) -> v8i {
    const int half = lane >> 5;
    int row;
    const uint8_t* base;
    if (q < TM) {
      row = wm * (BM / 2) + q * 32 + (lane & 31);
      base = lds[buf];
    } else {
      row = wn * (BN / 2) + (q - TM) * 32 + (lane & 31);
      base = lds[buf] + BM * ROWB;
    }
    const int c0 = 4 * d + 2 * half;
    const v4i lo = *reinterpret_cast<const v4i*>(base + row * ROWB + swz_chunk<ROWB>(row, c0) * 16);
    const v4i hi =
        *reinterpret_cast<const v4i*>(base + row * ROWB + swz_chunk<ROWB>(row, c0 + 1) * 16);
    return v8i{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
  };

  v16i acc[TM][TN];
  v16f accf[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      acc[i][j] = v16i{0};
      accf[i][j] = v16f{0.0f};
    }

  const int nk = (int)(klen / kF8SlabK);
  gload(0, 0);
  int buf = 0;
  for (int kt = 0; kt < nk; ++kt) {
    wait_vmem_lds_all();
    __syncthreads();   // slab kt is in LDS; every wave is done with the other buffer
    if (kt + 1 < nk) gload(buf ^ 1, (int64_t)(kt + 1) * ROWB);
    v8i fa[TM][2], fb[TN][2];
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      fa[i][0] = frag(buf, i, 0);
      fa[i][1] = frag(buf, i, 1);
    }
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      fb[j][0] = frag(buf, TM + j, 0);
      fb[j][1] = frag(buf, TM + j, 1);
    }
#pragma unroll
    for (int da = 0; da < 2; ++da)
#pragma unroll
      for (int db = 0; db < 2; ++db)
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
            accf[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                fa[i][da], fb[j][db], accf[i][j], 0, 0, 0, 0, 0, 0);
    if ((kt + 1) % kF8DumpSlabs == 0 || kt + 1 == nk) {
      // the block's sums are integers below 2^24: exact in binary32 and here
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
#pragma unroll
          for (int r = 0; r < 16; ++r) acc[i][j][r] += (int)accf[i][j][r];
          accf[i][j] = v16f{0.0f};
        }
    }
    buf ^= 1;
  }
  wait_vmem_all();
  tile_epilogue<BM, BN, EPI>(acc, U, aux0, nullptr, m, n, Mp, Np, tab, t, tm, tn, wm, wn, lane);
}

// All planes (EPI 0, 3) or plane t_raw (EPI 1) of one launch; tiles mapped
// to XCDs as the INT8 GEMM maps them.
template <int EPI>
__global__ __launch_bounds__(256) void k3_gemm_f8(const uint8_t* __restrict__ FA,
                                                  const uint8_t* __restrict__ FB,
                                                  uint8_t* __restrict__ U,
                                                  int32_t* __restrict__ aux0, int64_t m, int64_t n,
                                                  int64_t Mp, int64_t Np, int64_t Kp,
                                                  const ModTable* __restrict__ tab, int t_raw,
                                                  int64_t k0, int64_t klen) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[2][2 * kF8Tile * 128];
  const int tiles_m = (int)(Mp / kF8Tile), tiles_n = (int)(Np / kF8Tile);
  int plane, tm, tn;
  tile_of(blockIdx.x, gridDim.x, tiles_m, tiles_n, &plane, &tm, &tn);
  const int t = (EPI == 1) ? t_raw : plane;
  gemm_tile_f8<EPI>(FA, FB, U, aux0, m, n, Mp, Np, Kp, tab, t, tm, tn, lds, k0, klen);
}

}  // namespace oz2
