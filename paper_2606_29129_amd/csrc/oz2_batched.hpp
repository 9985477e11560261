// oz2_batched.hpp -- many independent emulated GEMMs of uneven shapes in a
// handful of launches (captured once into a HIP graph by the host side).
//
// Every problem keeps its own workspace regions and constants table (its own
// N).  The element-wise stages run as 1-D grids over the whole batch (the A
// and B halves of a step share one launch): a block reads its problem from
// a host-built block-to-problem table, its place inside the problem from a
// prefix sum of per-problem block counts, and runs the same body as the
// single-problem kernel.  The INT8 GEMM runs as a persistent
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

// The same descriptor as the device reads it: every pointer in the global
// address space (the table in the constant one; the kernels never write
// it).  Read through generic pointers, the element-wise bodies' loads and
// stores were flat accesses, which complete out of order, so every use of a
// loaded value waited for all outstanding memory operations; typed loads
// let the compiler emit global (and scalar) accesses and keep the bodies'
// own prefetching.
#define OZ2_GLOBAL __attribute__((address_space(1)))
struct BatchProbDev {
  const double OZ2_GLOBAL* A;
  const double OZ2_GLOBAL* B;
  double OZ2_GLOBAL* C;
  int64_t m, n, k, lda, ldb, ldc;
  int64_t Mp, Np, Kp, nch;
  int N, mode;
  __attribute__((address_space(4))) const ModTable* tab;
  int32_t OZ2_GLOBAL* eA;
  int32_t OZ2_GLOBAL* eB;
  double OZ2_GLOBAL* partA;
  double OZ2_GLOBAL* partB;
  double OZ2_GLOBAL* maxA;
  double OZ2_GLOBAL* maxB;
  double OZ2_GLOBAL* SA;
  double OZ2_GLOBAL* SB;
  int8_t OZ2_GLOBAL* RA;
  int8_t OZ2_GLOBAL* RB;
  uint8_t OZ2_GLOBAL* U;
  int64_t k1a_gx;
};
#undef OZ2_GLOBAL
static_assert(sizeof(BatchProbDev) == sizeof(BatchProb) &&
                  offsetof(BatchProbDev, tab) == offsetof(BatchProb, tab) &&
                  offsetof(BatchProbDev, U) == offsetof(BatchProb, U) &&
                  offsetof(BatchProbDev, k1a_gx) == offsetof(BatchProb, k1a_gx),
              "device view of the descriptor");

// k slab of the batched GEMM tile (bytes): 128 (Kp is a multiple of 128, so
// no more padding than 64) at two workgroups per CU (64 KiB of LDS each)
// measured 1-2% faster than 64-byte slabs at three.
constexpr int kBatchBK = 128;

// The fast modes need at most 2 limbs of 40 bits for |a'| (< 2^79 at N = 20).
constexpr int kBatchLimbs = 2;

// Stages with a per-problem block count.
enum BatchStage { kB_K1A = 0, kB_K1B, kB_FOLDA, kB_FOLDB, kB_K2A, kB_K2B, kB_K4, kB_NSTAGES };

// Block b of a stage (b counted from the stage's first block) finds its
// problem in a host-built table (one load) and its position inside the
// problem from the stage's block prefix sums.
template <int STAGE>
__device__ __forceinline__ void kb_stage_body(const BatchProb* __restrict__ probs,
                                              const int64_t* __restrict__ prefix,
                                              const uint16_t* __restrict__ owner, int batch,
                                              int* __restrict__ status, int64_t b) {
  const int64_t* pre = prefix + (int64_t)STAGE * (batch + 1);
  const int p = owner[b];
  const int64_t local = b - pre[p];
  const BatchProbDev& P = reinterpret_cast<const BatchProbDev*>(probs)[p];
  // Generic pointers for the bodies, each converted from its typed load (the
  // compiler carries the global address space into the inlined bodies).
  const double* A = (const double*)P.A;
  const double* B = (const double*)P.B;
  const ModTable* tab = (const ModTable*)P.tab;
  int32_t* eA = (int32_t*)P.eA;
  int32_t* eB = (int32_t*)P.eB;
  switch (STAGE) {
    case kB_K1A: {
      int64_t bx = local % P.k1a_gx, by = local / P.k1a_gx;
      k1_partials_strided_body<double>(A, P.lda, P.m, P.k, P.nch, (double*)P.partA,
                                       (double*)P.maxA, bx, by);
      break;
    }
    case kB_K1B:
      k1_partials_contig_body<double>(B, P.ldb, P.n, P.k, P.nch, (double*)P.partB,
                                      (double*)P.maxB, local);
      break;
    case kB_FOLDA:
      k1_fold_body((double*)P.partA, (double*)P.maxA, P.nch, P.m, P.mode, tab, eA,
                   (double*)P.SA, status, local);
      break;
    case kB_FOLDB:
      k1_fold_body((double*)P.partB, (double*)P.maxB, P.nch, P.n, P.mode, tab, eB,
                   (double*)P.SB, status, local);
      break;
    case kB_K2A: {
      const int64_t gx = P.Mp / kK2VB;
      int64_t bx = local % gx, by = local / gx;
      k2_split_strided_body<double, kBatchLimbs>(A, P.lda, P.m, P.k, eA, tab, P.N, (int8_t*)P.RA,
                                                 P.Mp, P.Kp, bx, by);
      break;
    }
    case kB_K2B:
      k2_split_contig_body<double, kBatchLimbs>(B, P.ldb, P.n, P.k, eB, tab, P.N, (int8_t*)P.RB,
                                                P.Np, P.Kp, local);
      break;
    default:
      k4_crt_body<4, double>((uint8_t*)P.U, eA, eB, tab, P.N, P.m, P.n, P.Mp, P.Np,
                             (double*)P.C, P.ldc, local);
      break;
  }
}

// One stage per launch (one instantiation per stage, so that each gets the
// register budget and occupancy of its own body).
template <int STAGE>
__global__ __launch_bounds__(256) void kb_stage(const BatchProb* __restrict__ probs,
                                                const int64_t* __restrict__ prefix,
                                                const uint16_t* __restrict__ owner, int batch,
                                                int* __restrict__ status) {
  kb_stage_body<STAGE>(probs, prefix, owner, batch, status, blockIdx.x);
}

// The A and the B half of one step (two independent stages) in one launch:
// blocks [0, nfirst) run stage S1, the others stage S2, whose owner entries
// follow S1's in the owner table.  The halves overlap instead of the second
// waiting for the first one's last blocks.
// Three blocks per CU: the norm pair's bodies keep a chunk's 64 loads in
// flight (174 registers, two waves per SIMD); capped at 168 registers (a
// few spilled) a third wave covers the others' waits on the batch's short
// vectors, 0.59 -> 0.51 ms for the 256-problem batch (the plain path's
// norm kernel, on long vectors, is slower so capped).  The other pairs'
// times do not change.
template <int S1, int S2>
__global__ __launch_bounds__(256, 3) void kb_stage_pair(const BatchProb* __restrict__ probs,
                                                     const int64_t* __restrict__ prefix,
                                                     const uint16_t* __restrict__ owner,
                                                     int batch, int64_t nfirst,
                                                     int* __restrict__ status) {
  const int64_t b = blockIdx.x;
  if (b < nfirst)
    kb_stage_body<S1>(probs, prefix, owner, batch, status, b);
  else
    kb_stage_body<S2>(probs, prefix, owner + nfirst, batch, status, b - nfirst);
}

// Work item: problem, plane, tile row, tile column (16 bits each).
struct __attribute__((aligned(8))) WorkItem {
  uint16_t p;
  uint16_t t;
  uint16_t tm;
  uint16_t tn;
};
// (read on the device as one little-endian 8-byte word: p in bits 0-15, t in
// 16-31, tm in 32-47, tn in 48-63)
static_assert(sizeof(WorkItem) == 8 && offsetof(WorkItem, t) == 2 && offsetof(WorkItem, tm) == 4 &&
                  offsetof(WorkItem, tn) == 6,
              "work item layout");

typedef __attribute__((address_space(1))) uint8_t GlobalU8;
typedef __attribute__((address_space(4))) const ModTable ConstTable;
struct TileArgs {
  const int8_t* RA;
  const int8_t* RB;
  GlobalU8* U;
  int64_t m, n, Mp, Np, Kp;
  ConstTable* tab;
  int t, tm, tn;
};

// The descriptor's pointers are generic; the ones the tile writes through
// (U) and reads its constants from (tab) are cast to the global and the
// constant address space (kept so across the loop, where a cast pair
// would fold away).  Through generic pointers the epilogue's stores
// were flat stores and its reads of p_t flat loads, and flat accesses
// complete out of order: every use of p_t then waited for all outstanding
// memory operations, the previous 16-byte store of the tile included, so
// each tile paid its store round trips one after another.  The work item is
// read as one 8-byte word through the constant address space (the list is
// not written by the kernel and i is the same in every lane), a scalar load.
__device__ __forceinline__ TileArgs tile_args(const BatchProb* __restrict__ probs,
                                              const WorkItem* __restrict__ items, int i) {
  typedef __attribute__((address_space(4))) const uint64_t ConstWord;
  const uint64_t raw = ((ConstWord*)items)[__builtin_amdgcn_readfirstlane(i)];
  const int p = (int)(raw & 0xFFFF), t = (int)((raw >> 16) & 0xFFFF);
  const int tm = (int)((raw >> 32) & 0xFFFF), tn = (int)(raw >> 48);
  const BatchProb& P = probs[p];
  return TileArgs{P.RA, P.RB, (GlobalU8*)P.U, P.m, P.n, P.Mp, P.Np, P.Kp, (ConstTable*)P.tab,
                  t, tm, tn};
}

// Persistent GEMM over the work list (each XCD's share sorted by decreasing
// k, the tiles of a plane kept on one XCD by the host's ordering).
// Workgroup b takes items b, b + G, b + 2G, ... (G = grid size): a sorted
// list dealt out round-robin balances like a greedy queue, without the
// contended atomic counter, and the next item is known in advance, so its
// descriptor is loaded while the current tile runs.
__global__ __launch_bounds__(256) void kb_gemm(const BatchProb* __restrict__ probs,
                                               const WorkItem* __restrict__ items, int nitems) {
  __shared__ __attribute__((aligned(16))) int8_t lds[2][2 * kBatchTile * kBatchBK];
  int i = blockIdx.x;
  if (i >= nitems) return;
  TileArgs cur = tile_args(probs, items, i);
  int buf = 0;
  bool loaded = false;
  for (;;) {
    const int inext = i + (int)gridDim.x;
    const bool more = inext < nitems;
    const TileArgs nxt = tile_args(probs, items, more ? inext : i);
    // the next item's row panels (its first slab is loaded during this
    // item's last slab)
    const int8_t* nA =
        more ? nxt.RA + ((int64_t)nxt.t * nxt.Mp + (int64_t)nxt.tm * kBatchTile) * nxt.Kp : nullptr;
    const int8_t* nB =
        more ? nxt.RB + ((int64_t)nxt.t * nxt.Np + (int64_t)nxt.tn * kBatchTile) * nxt.Kp : nullptr;
    // A 128 x 128 tile has only 4 MFMAs per k step per wave; two
    // workgroups share a CU (64 KiB of LDS each), hiding part of the
    // per-item latency of the small problems; barrier at the slab top.
    // No barrier between items: the epilogue does not touch the LDS, and the
    // next item's first barrier orders its loads after every wave's last
    // reads of this item.
    buf = gemm_tile<kBatchTile, kBatchTile, kBatchBK, 0, false, 2, 0, true>(
        cur.RA, cur.RB, (uint8_t*)cur.U, nullptr, nullptr, cur.m, cur.n, cur.Mp, cur.Np, cur.Kp,
        (const ModTable*)cur.tab, cur.t, cur.tm, cur.tn, lds, 0, -1, buf, loaded, nA, nB,
        nxt.Kp);
    if (!more) break;
    loaded = true;
    i = inext;
    cur = nxt;
  }
}

// Caller pointers of up to kBatchPtrChunk consecutive descriptors, passed as
// kernel arguments (1.5 KiB): a replay whose problems moved to new matrices
// rewrites only these fields, stream ordered, with no host buffer that has to
// outlive the call.
constexpr int kBatchPtrChunk = 64;
struct BatchPtrs {
  const double* A[kBatchPtrChunk];
  const double* B[kBatchPtrChunk];
  double* C[kBatchPtrChunk];
  int first, count;
};

__global__ void kb_set_ptrs(BatchProb* __restrict__ probs, BatchPtrs p) {
  const int c = threadIdx.x;
  if (c < p.count) {
    BatchProb& q = probs[p.first + c];
    q.A = p.A[c];
    q.B = p.B[c];
    q.C = p.C[c];
  }
}

// Status word reset at the start of each replay (a kernel, not a memset, so
// that it can live in the captured graph).
__global__ void kb_reset(int* __restrict__ status) {
  if (threadIdx.x == 0) status[0] = 0;
}

}  // namespace oz2
