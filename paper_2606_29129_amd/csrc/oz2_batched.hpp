// oz2_batched.hpp -- many independent emulated GEMMs of uneven shapes in a
// handful of launches (captured once into a HIP graph by the host side).
//
// Every problem keeps its own workspace regions and constants table (its own
// N).  The element-wise stages run as one 1-D grid per kernel: a block reads
// its problem from a host-built block-to-problem table, its place inside the
// problem from a prefix sum of per-problem block counts, and runs the same
// body as the single-problem kernel.  The INT8 GEMM runs as a persistent
// kernel over a list of (problem, plane, tile) items sorted by decreasing k,
// dealt out round-robin to the workgroups.
#pragma once

#include "oz2_k1_norm.hpp"
#include "oz2_k2_split.hpp"
#include "oz2_k3_gemm.hpp"
#include "oz2_k4_crt.hpp"

namespace oz2 {

constexpr int kBatchTile = 128;   // GEMM tile of the batched path (BM = BN)

struct BatchProb {
  const double* A;
  const double* B;
  double* C;
  int64_t m, n, k, lda, ldb, ldc;
  int64_t Mp, Np, Kp, nch;
  int N, mode;
  const ModTable* tab;
  int32_t *eA, *eB;
  double *partA, *partB, *maxA, *maxB, *SA, *SB;
  int8_t *RA, *RB;
  uint8_t* U;
  int64_t k1a_gx;  // K1 strided grid width (height is ceil(nch/4))
};

// k slab of the batched GEMM tile (bytes).
constexpr int kBatchBK = 64;

// The fast modes need at most 2 limbs of 40 bits for |a'| (< 2^79 at N = 20).
constexpr int kBatchLimbs = 2;

// Stages with a per-problem block count.
enum BatchStage { kB_K1A = 0, kB_K1B, kB_FOLDA, kB_FOLDB, kB_K2A, kB_K2B, kB_K4, kB_NSTAGES };

// One instantiation per stage, so that each gets the register budget (and
// occupancy) of its own body.
// A block finds its problem in a host-built table (one load) and its
// position inside the problem from the stage's block prefix sums.
template <int STAGE>
__global__ __launch_bounds__(256) void kb_stage(const BatchProb* __restrict__ probs,
                                                const int64_t* __restrict__ prefix,
                                                const uint16_t* __restrict__ owner, int batch,
                                                int* __restrict__ status) {
  const int64_t* pre = prefix + (int64_t)STAGE * (batch + 1);
  const int64_t b = blockIdx.x;
  const int p = owner[b];
  const int64_t local = b - pre[p];
  const BatchProb& P = probs[p];
  switch (STAGE) {
    case kB_K1A: {
      int64_t bx = local % P.k1a_gx, by = local / P.k1a_gx;
      k1_partials_strided_body<double>(P.A, P.lda, P.m, P.k, P.nch, P.partA, P.maxA, bx, by);
      break;
    }
    case kB_K1B:
      k1_partials_contig_body<double>(P.B, P.ldb, P.n, P.k, P.nch, P.partB, P.maxB, local);
      break;
    case kB_FOLDA:
      k1_fold_body(P.partA, P.maxA, P.nch, P.m, P.mode, P.tab, P.eA, P.SA, status, local);
      break;
    case kB_FOLDB:
      k1_fold_body(P.partB, P.maxB, P.nch, P.n, P.mode, P.tab, P.eB, P.SB, status, local);
      break;
    case kB_K2A: {
      const int64_t gx = P.Mp / kK2VB;
      int64_t bx = local % gx, by = local / gx;
      k2_split_strided_body<double, kBatchLimbs>(P.A, P.lda, P.m, P.k, P.eA, P.tab, P.N, P.RA, P.Mp,
                                       P.Kp, bx, by);
      break;
    }
    case kB_K2B:
      k2_split_contig_body<double, kBatchLimbs>(P.B, P.ldb, P.n, P.k, P.eB, P.tab, P.N, P.RB, P.Np, P.Kp,
                                      local);
      break;
    default:
      k4_crt_body<4, double>(P.U, P.eA, P.eB, P.tab, P.N, P.m, P.n, P.Mp, P.Np, P.C, P.ldc,
                             local);
      break;
  }
}

// Work item: problem (16 bits), plane (8 bits), tile row, tile column.
struct WorkItem {
  uint16_t p;
  uint16_t t;
  uint16_t tm;
  uint16_t tn;
};

// Persistent GEMM over the work list (each XCD's share sorted by decreasing
// k, the tiles of a plane kept on one XCD by the host's ordering).
// Workgroup b takes items b, b + G, b + 2G, ... (G = grid size): a sorted
// list dealt out round-robin balances like a greedy queue, without the
// contended atomic counter, and the next item is known in advance, so its
// descriptor is loaded while the current tile runs.
struct TileArgs {
  const int8_t* RA;
  const int8_t* RB;
  uint8_t* U;
  int64_t m, n, Mp, Np, Kp;
  const ModTable* tab;
  int t, tm, tn;
};

__device__ __forceinline__ TileArgs tile_args(const BatchProb* __restrict__ probs,
                                              const WorkItem* __restrict__ items, int i) {
  const WorkItem w = items[i];
  const BatchProb& P = probs[w.p];
  return TileArgs{P.RA, P.RB, P.U, P.m, P.n, P.Mp, P.Np, P.Kp, P.tab, w.t, w.tm, w.tn};
}

__global__ __launch_bounds__(256) void kb_gemm(const BatchProb* __restrict__ probs,
                                               const WorkItem* __restrict__ items, int nitems) {
  __shared__ __attribute__((aligned(16))) int8_t lds[2][2 * kBatchTile * kBatchBK];
  int i = blockIdx.x;
  if (i >= nitems) return;
  TileArgs cur = tile_args(probs, items, i);
  for (;;) {
    const int inext = i + (int)gridDim.x;
    const bool more = inext < nitems;
    const TileArgs nxt = tile_args(probs, items, more ? inext : i);
    // A 128 x 128 tile has only 4 MFMAs per k step per wave; with 64-byte
    // k slabs (32 KiB of LDS) three workgroups share a CU, hiding the
    // per-item latency of the small problems; barrier at the slab top.
    gemm_tile<kBatchTile, kBatchTile, kBatchBK, 0, false, 2>(cur.RA, cur.RB, cur.U, nullptr, nullptr,
                                                        cur.m, cur.n, cur.Mp, cur.Np, cur.Kp,
                                                        cur.tab, cur.t, cur.tm, cur.tn, lds);
    if (!more) break;
    __syncthreads();  // every wave is done with the LDS before the next prologue
    i = inext;
    cur = nxt;
  }
}

// Status word reset at the start of each replay (a kernel, not a memset, so
// that it can live in the captured graph).
__global__ void kb_reset(int* __restrict__ status) {
  if (threadIdx.x == 0) status[0] = 0;
}

}  // namespace oz2
