// oz2_lib.hip -- libozaki2: the C ABI declared in include/ozaki2.h.
//
// One translation unit: host planning (argument checks, constant tables,
// workspace layout, stream, stage timing) and the four kernels K1-K4.
#include <hip/hip_runtime.h>

#include <limits.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "ozaki2.h"
#include "oz2_k1_norm.hpp"
#include "oz2_k2_split.hpp"
#include "oz2_k3_gemm.hpp"
#include "oz2_k3_fp8.hpp"
#include "oz2_k4_crt.hpp"
#include "oz2_tables.hpp"
#include "oz2_batched.hpp"
#include "oz2_complex.hpp"
#include "oz2_autotune.hpp"
#include "oz2_fused.hpp"

#include <algorithm>

using namespace oz2;

// Constant tables for every N (index 0: fast modes, 1: accurate mode limbs).
__device__ ModTable g_tables[2][kMaxN + 1];

// Workspace of ozaki2_dgemm_noalloc: fixed device memory, one copy per GPU
// (held until the process ends).  Host code never passes `scratch` itself
// (on the host it names a stand-in, not device memory); it uses the device
// address taken once per device with hipGetSymbolAddress (DevState).
static __device__ __align__(256) char scratch[OZ2_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kBM = 256, kBN = 256, kBK = 128;  // largest K3 tile (sizes the workspace)
constexpr int kMaxDevices = 64;

struct DevState {
  bool ready = false;
  ModTable* d_tables = nullptr;  // device address of g_tables
  void* ws = nullptr;            // library-owned workspace (OZ2_WORKSPACE_LIBRARY only)
  size_t ws_bytes = 0;
  char* scratch = nullptr;       // device address of `scratch` on this device
};

DevState g_dev[kMaxDevices];
hipStream_t g_stream = nullptr;
void* g_user_ws = nullptr;
size_t g_user_ws_bytes = 0;
int g_ws_policy = OZ2_WORKSPACE_CALLER;
// Advanced whenever workspace memory may have been written by anything but
// the batched path's own kernels (another entry point's call, a new or
// re-set workspace, a library reallocation): the batch's tables, which stay
// in the workspace between calls, are then written again before a replay.
uint64_t g_ws_epoch = 1;
ModTable g_host_tables[2][kMaxN + 1];
bool g_host_tables_ok[2][kMaxN + 1];
bool g_host_tables_built = false;
int g_timing = 0;
double g_stage_ms[OZ2_NUM_STAGES];
int g_timed_calls = 0;

void build_host_tables() {
  if (g_host_tables_built) return;
  for (int a = 0; a < 2; ++a)
    for (int N = 0; N <= kMaxN; ++N)
      g_host_tables_ok[a][N] = build_table(N, a == 1, &g_host_tables[a][N]);
  g_host_tables_built = true;
}

int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }
size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
  int64_t Mp, Np, Kp, nch;
  size_t eA, eB, SA, SB, partA, partB, maxA, maxB, RA, RB, U, status, total;
  size_t e1A, e1B, cmaxA, cmaxB, barA, barB;  // accurate mode only
  size_t FA, FB;                               // FP8 engine: digit planes
};

// GEMM tile configurations (OZ2_TILE_*): rows x columns of the output tile.
constexpr int kTileBM[4] = {0, 256, 128, 256};
constexpr int kTileBN[4] = {0, 256, 128, 64};
int g_tile_policy = OZ2_TILE_AUTO;

// Automatic tile choice: a cost model over the padded work and the number of
// workgroup rounds.  A 256 x 256 tile runs one workgroup per CU, the smaller
// tiles two.  Per CU and unit of padded output the smaller tiles are slower
// (128 x 128 at 0.75, 256 x 64 at 0.45 of the 256 x 256 rate), but with two
// workgroups per CU one's prologue and epilogue overlap the other's main
// loop, while a 256 x 256 round pays them in full (counted as 2 k slabs).
// The constants are the fit (autotune.fit_tile_model) to measured times of
// the three tiles (autotune_tiles.json) on 13 shapes
// (square 512..16384, k from 512 to 16384, n = 64..256 skinny) at N = 14
// and 20: the model's pick is never more than 0.6% slower than the best.
int choose_tile(int64_t m, int64_t n, int64_t k, int N) {
  constexpr double kRate[4] = {0.0, 1.0, 0.75, 0.45};
  constexpr int kPerCU[4] = {0, 1, 2, 2};
  constexpr double kFixed[4] = {0.0, 2.0, 0.0, 0.0};
  const double slabs = (double)((k + kBK - 1) / kBK);
  int best = OZ2_TILE_256x256;
  double best_t = 0.0;
  for (int c = OZ2_TILE_256x256; c <= OZ2_TILE_256x64; ++c) {
    const int64_t tiles = ((m + kTileBM[c] - 1) / kTileBM[c]) * ((n + kTileBN[c] - 1) / kTileBN[c]);
    const double rounds = ceil((double)(tiles * N) / (256.0 * kPerCU[c]));
    const double t =
        rounds * (double)kTileBM[c] * kTileBN[c] * kPerCU[c] * (slabs + kFixed[c]) / kRate[c];
    if (c == OZ2_TILE_256x256 || t < best_t) {
      best = c;
      best_t = t;
    }
  }
  return best;
}

int tile_config(int64_t m, int64_t n, int64_t k, int N) {
  return g_tile_policy == OZ2_TILE_AUTO ? choose_tile(m, n, k, N) : g_tile_policy;
}

// comps = 1 for real products; 3 for complex ones (three residue planes per
// modulus and operand, three uint8 product planes per modulus; the squared
// norms run over 2k components).
Layout make_layout(int64_t m, int64_t n, int64_t k, int N, int mode, int64_t bm = kBM,
                   int64_t bn = kBN, int comps = 1, bool fused = false) {
  const bool fp8 = (mode & OZ2_ENGINE_FP8) != 0;
  mode &= ~OZ2_ENGINE_FP8;
  Layout L;
  L.Mp = round_up(m > 0 ? m : 1, bm);
  L.Np = round_up(n > 0 ? n : 1, bn);
  L.Kp = round_up(k > 0 ? k : 1, kBK);
  L.nch = ((comps == 3 ? 2 * k : k) + kKC - 1) / kKC;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
  L.status = take(256);
  L.eA = take(4 * (size_t)L.Mp);
  L.eB = take(4 * (size_t)L.Np);
  L.SA = take(8 * (size_t)m);
  L.SB = take(8 * (size_t)n);
  L.partA = take(8 * (size_t)L.nch * m);
  L.partB = take(8 * (size_t)L.nch * n);
  const bool need_max = (mode == OZ2_MODE_ORIGINAL || mode == OZ2_MODE_ACCURATE);
  L.maxA = need_max ? take(8 * (size_t)L.nch * m) : 0;
  L.maxB = need_max ? take(8 * (size_t)L.nch * n) : 0;
  const bool acc = (mode == OZ2_MODE_ACCURATE);
  L.e1A = acc ? take(4 * (size_t)L.Mp) : 0;
  L.e1B = acc ? take(4 * (size_t)L.Np) : 0;
  L.cmaxA = acc ? take(4 * (size_t)L.Mp) : 0;
  L.cmaxB = acc ? take(4 * (size_t)L.Np) : 0;
  L.barA = acc ? take((size_t)L.Mp * L.Kp) : 0;
  L.barB = acc ? take((size_t)L.Np * L.Kp) : 0;
  // the fused path (n <= 64) keeps A's residues and the products in registers
  L.RA = take(fused ? 0 : (size_t)comps * N * L.Mp * L.Kp);
  L.RB = take((size_t)comps * N * L.Np * L.Kp);
  L.U = take(fused ? 0 : (size_t)comps * N * L.Mp * L.Np);
  L.FA = fp8 ? take((size_t)N * L.Mp * 2 * L.Kp) : 0;
  L.FB = fp8 ? take((size_t)N * L.Np * 2 * L.Kp) : 0;
  L.total = off;
  return L;
}

// BLAS-style argument checks shared by the GEMM entry points.
int check_args(int64_t m, int64_t n, int64_t k, const void* A, int64_t lda,
               const void* B, int64_t ldb, const void* C, int64_t ldc, int N, int mode,
               bool have_c) {
  if (m < 0) return -1;
  if (n < 0) return -2;
  if (k < 0) return -3;
  if (!A && m > 0 && k > 0) return -4;
  if (lda < (m > 1 ? m : 1)) return -5;
  if (!B && k > 0 && n > 0) return -6;
  if (ldb < (k > 1 ? k : 1)) return -7;
  if (have_c) {
    if (!C && m > 0 && n > 0) return -8;
    if (ldc < (m > 1 ? m : 1)) return -9;
  }
  if (N < OZ2_N_MIN || N > OZ2_N_MAX) return -10;
  mode &= ~OZ2_ENGINE_FP8;
  if (mode != OZ2_MODE_REVISED && mode != OZ2_MODE_ORIGINAL && mode != OZ2_MODE_ACCURATE &&
      mode != OZ2_MODE_EXACT)
    return -11;
  if (k > OZ2_K_MAX || (mode == OZ2_MODE_ACCURATE && k > OZ2_K_MAX_ACCURATE))
    return OZ2_ERR_K_TOO_LARGE;
  if (m > (int64_t)INT32_MAX / 2 || n > (int64_t)INT32_MAX / 2) return OZ2_ERR_TOO_LARGE;
  return 0;
}

int ensure_device(int* dev_out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return OZ2_ERR_HIP;
  if (dev < 0 || dev >= kMaxDevices) return OZ2_ERR_HIP;
  DevState& D = g_dev[dev];
  if (!D.ready) {
    build_host_tables();
    if (hipMemcpyToSymbol(HIP_SYMBOL(g_tables), g_host_tables, sizeof g_host_tables) != hipSuccess)
      return OZ2_ERR_HIP;
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(g_tables)) != hipSuccess) return OZ2_ERR_HIP;
    D.d_tables = reinterpret_cast<ModTable*>(p);
    void* sp = nullptr;
    if (hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)) != hipSuccess || !sp) return OZ2_ERR_HIP;
    D.scratch = reinterpret_cast<char*>(sp);
    D.ready = true;
  }
  *dev_out = dev;
  return 0;
}

// The caller's workspace if it is large enough.  Otherwise, under the
// default policy (OZ2_WORKSPACE_CALLER), OZ2_ERR_WORKSPACE: no call on the
// hot path allocates device memory.  Under OZ2_WORKSPACE_LIBRARY (an opt-in
// convenience) the library allocates, grows and keeps its own.
// Every call advances g_ws_epoch except those of the batched path
// (keeps_batch_tables), whose writes never reach the tables of a batch with
// the same signature.
int get_workspace(int dev, size_t bytes, char** out, bool keeps_batch_tables = false) {
  if (!keeps_batch_tables) ++g_ws_epoch;
  if (g_user_ws && g_user_ws_bytes >= bytes) {
    *out = reinterpret_cast<char*>(g_user_ws);
    return 0;
  }
  if (g_ws_policy != OZ2_WORKSPACE_LIBRARY) return OZ2_ERR_WORKSPACE;
  DevState& D = g_dev[dev];
  if (D.ws_bytes < bytes) {
    ++g_ws_epoch;
    if (D.ws) {
      if (hipDeviceSynchronize() != hipSuccess) return OZ2_ERR_HIP;
      (void)hipFree(D.ws);
      D.ws = nullptr;
      D.ws_bytes = 0;
    }
    size_t want = align256(bytes + bytes / 8);
    if (hipMalloc(&D.ws, want) != hipSuccess) {
      D.ws = nullptr;
      return OZ2_ERR_WORKSPACE;
    }
    D.ws_bytes = want;
  }
  *out = reinterpret_cast<char*>(D.ws);
  return 0;
}

// Stage timing: each timed call records OZ2_NUM_STAGES + 1 events on the
// stream; nothing waits for them until ozaki2_get_stage_times.
struct TimedCall {
  hipEvent_t ev[OZ2_NUM_STAGES + 1];
};
std::vector<TimedCall> g_pending;
std::vector<TimedCall> g_free;

struct StageClock {
  bool on;
  TimedCall tc;
  explicit StageClock(bool allowed = true) : on(allowed && g_timing != 0) {
    if (!on) return;
    if (!g_free.empty()) {
      tc = g_free.back();
      g_free.pop_back();
    } else {
      for (int i = 0; i <= OZ2_NUM_STAGES; ++i)
        if (hipEventCreate(&tc.ev[i]) != hipSuccess) { on = false; return; }
    }
  }
  void mark(int i) {
    if (on) (void)hipEventRecord(tc.ev[i], g_stream);
  }
  void finish() {
    if (on) g_pending.push_back(tc);
    on = false;
  }
  ~StageClock() {
    if (on) g_free.push_back(tc);  // abandoned on an error path
  }
};

struct Debug {
  int t;
  int32_t *eA, *eB, *Ct;
  double *SA, *SB;
  int8_t *RA, *RB;
};

// Small problems (K2 would launch fewer than 1024 blocks): K2 takes 8 entries
// of A per lane (twice the blocks for A).  Residue planes that fit in half
// the MALL (128 MiB): K1 and K2 use ordinary loads and stores, so that the
// operands stay in the caches for K2 and the planes for the GEMM.
bool small_problem(const Layout& L) {
  const int64_t nA = (L.Mp / kK2VB) * (L.Kp / kK2HB);
  const int64_t nB = (L.Np * (L.Kp / kK2EPT) + 255) / 256;
  return nA + nB < 4 * 256;
}
bool cache_resident(const Layout& L, int N) {
  return (int64_t)N * (L.Mp + L.Np) * L.Kp <= (int64_t(128) << 20);
}

template <typename T, int LIMBS>
void launch_split(const T* A, int64_t lda, const T* B, int64_t ldb, int64_t m, int64_t n,
                  int64_t k, const Layout& L, char* ws, const ModTable* tab, int N) {
  const int64_t gAx = L.Mp / kK2VB, nA = gAx * (L.Kp / kK2HB);
  const int64_t nB = (L.Np * (L.Kp / kK2EPT) + 255) / 256;
  if (small_problem(L)) {
    const int64_t nA8 = gAx * (L.Kp / kK2HBSmall);
    k2_split_ab<T, LIMBS, 8, false><<<(unsigned)(nA8 + nB), 256, 0, g_stream>>>(
        A, lda, m, (const int32_t*)(ws + L.eA), (int8_t*)(ws + L.RA), L.Mp, B, ldb, n,
        (const int32_t*)(ws + L.eB), (int8_t*)(ws + L.RB), L.Np, k, tab, N, L.Kp, gAx, nA8);
    return;
  }
  if (cache_resident(L, N)) {
    k2_split_ab<T, LIMBS, 16, false><<<(unsigned)(nA + nB), 256, 0, g_stream>>>(
        A, lda, m, (const int32_t*)(ws + L.eA), (int8_t*)(ws + L.RA), L.Mp, B, ldb, n,
        (const int32_t*)(ws + L.eB), (int8_t*)(ws + L.RB), L.Np, k, tab, N, L.Kp, gAx, nA);
    return;
  }
  k2_split_ab<T, LIMBS><<<(unsigned)(nA + nB), 256, 0, g_stream>>>(
      A, lda, m, (const int32_t*)(ws + L.eA), (int8_t*)(ws + L.RA), L.Mp, B, ldb, n,
      (const int32_t*)(ws + L.eB), (int8_t*)(ws + L.RB), L.Np, k, tab, N, L.Kp, gAx, nA);
}

// K3 over the planes given by (t, planes): EPI 0 runs all N planes (t
// ignored), EPI 1 and 2 one plane.
template <int EPI>
void launch_gemm(int cfg, const int8_t* RA, const int8_t* RB, uint8_t* U, int32_t* aux0,
                 int32_t* aux1, int64_t m, int64_t n, const Layout& L, const ModTable* tab,
                 int t, int planes, int64_t k0 = 0, int64_t klen = -1) {
  const unsigned tiles =
      (unsigned)((L.Mp / kTileBM[cfg]) * (L.Np / kTileBN[cfg]) * planes);
  if (klen < 0) klen = L.Kp;
  switch (cfg) {
    case OZ2_TILE_128x128:
      k3_gemm_i8<128, 128, kBK, EPI><<<tiles, 256, 0, g_stream>>>(
          RA, RB, U, aux0, aux1, m, n, L.Mp, L.Np, L.Kp, tab, t, k0, klen);
      break;
    case OZ2_TILE_256x64:
      k3_gemm_i8<256, 64, kBK, EPI><<<tiles, 256, 0, g_stream>>>(
          RA, RB, U, aux0, aux1, m, n, L.Mp, L.Np, L.Kp, tab, t, k0, klen);
      break;
    default:
      k3_gemm_i8<256, 256, kBK, EPI><<<tiles, 256, 0, g_stream>>>(
          RA, RB, U, aux0, aux1, m, n, L.Mp, L.Np, L.Kp, tab, t, k0, klen);
      break;
  }
}

// K3 over all N planes; k beyond OZ2_K_BLOCK in blocks of OZ2_K_BLOCK (each
// block's INT32 products are exact; later blocks add theirs modulo p_t).
void launch_gemm_blocked(int cfg, const int8_t* RA, const int8_t* RB, uint8_t* U, int64_t m,
                         int64_t n, const Layout& L, const ModTable* tab, int N) {
  for (int64_t k0 = 0; k0 < L.Kp; k0 += OZ2_K_BLOCK) {
    const int64_t klen = std::min<int64_t>(OZ2_K_BLOCK, L.Kp - k0);
    if (k0 == 0) launch_gemm<0>(cfg, RA, RB, U, nullptr, nullptr, m, n, L, tab, 0, N, k0, klen);
    else launch_gemm<3>(cfg, RA, RB, U, nullptr, nullptr, m, n, L, tab, 0, N, k0, klen);
  }
}

template <int S, typename TO>
void launch_crt(const Layout& L, char* ws, const ModTable* tab, int N, int64_t m, int64_t n,
                TO* C, int64_t ldc) {
  const int64_t blocks = ((m + 31) / 32) * ((n + 31) / 32);
  // four waves per 32 x 32 block when two would leave fewer than four
  // waves per SIMD (1024 SIMDs)
  if (blocks * kK4WavesPerBlock < 4 * 1024) {
    const int64_t waves = blocks * kK4WavesPerBlockSmall;
    k4_crt<S, TO, kK4WavesPerBlockSmall><<<(unsigned)((waves + 3) / 4), 256, 0, g_stream>>>(
        (const uint8_t*)(ws + L.U), (const int32_t*)(ws + L.eA), (const int32_t*)(ws + L.eB),
        tab, N, m, n, L.Mp, L.Np, C, ldc);
  } else {
    const int64_t waves = blocks * kK4WavesPerBlock;
    k4_crt<S, TO><<<(unsigned)((waves + 3) / 4), 256, 0, g_stream>>>(
        (const uint8_t*)(ws + L.U), (const int32_t*)(ws + L.eA), (const int32_t*)(ws + L.eB),
        tab, N, m, n, L.Mp, L.Np, C, ldc);
  }
}

// fixed_ws: the device's `scratch` array as the workspace (no stage events,
// no allocation of any kind); a call that needs more returns
// OZ2_ERR_SCRATCH_TOO_SMALL before launching anything.
template <typename T, typename TO>
int run_gemm(int64_t m, int64_t n, int64_t k, const T* A, int64_t lda, const T* B,
             int64_t ldb, TO* C, int64_t ldc, int N, int mode, const Debug* dbg,
             bool fixed_ws = false) {
  int rc = check_args(m, n, k, A, lda, B, ldb, C, ldc, N, mode, dbg == nullptr);
  if (rc) return rc;
  if (dbg && (dbg->t < 0 || dbg->t >= N)) return -10;
  if (dbg && dbg->Ct && k > OZ2_K_BLOCK) return OZ2_ERR_UNSUPPORTED;  // INT32 of one block
  const bool fp8 = (mode & OZ2_ENGINE_FP8) != 0;
  mode &= ~OZ2_ENGINE_FP8;
  if (fp8 && mode == OZ2_MODE_ACCURATE) return OZ2_ERR_UNSUPPORTED;
  if (m == 0 || n == 0) return 0;
  int dev;
  if ((rc = ensure_device(&dev))) return rc;
  DevState& D = g_dev[dev];
  if (k == 0) {
    if (dbg) return 0;
    k_zero<TO><<<(unsigned)((m * n + 255) / 256), 256, 0, g_stream>>>(C, m, n, ldc);
    return hipGetLastError() == hipSuccess ? 0 : OZ2_ERR_HIP;
  }
  build_host_tables();
  const int acc_tab = (mode == OZ2_MODE_ACCURATE) ? 1 : 0;
  if (!g_host_tables_ok[acc_tab][N]) return OZ2_ERR_UNSUPPORTED;
  const ModTable& HT = g_host_tables[acc_tab][N];
  const ModTable* tab = D.d_tables + acc_tab * (kMaxN + 1) + N;

  const int cfg = tile_config(m, n, k, N);
  // Narrow B: conversion of A, products and CRT in one kernel (automatic
  // tile choice only; a forced tile keeps the separate kernels).
  const bool fused = !dbg && !fp8 && g_tile_policy == OZ2_TILE_AUTO && n <= kFuseCols &&
                     N <= kFuseMaxN && mode != OZ2_MODE_ACCURATE && k <= OZ2_K_BLOCK &&
                     HT.limbs == 2;
  Layout L = fused ? make_layout(m, n, k, N, mode, kFuseRows, kFuseCols, 1, true)
             : fp8 ? make_layout(m, n, k, N, mode | OZ2_ENGINE_FP8, kF8Tile, kF8Tile)
                   : make_layout(m, n, k, N, mode, kTileBM[cfg], kTileBN[cfg]);
  char* ws = nullptr;
  if (fixed_ws) {
    if (L.total > (size_t)OZ2_NOALLOC_SCRATCH_BYTES) return OZ2_ERR_SCRATCH_TOO_SMALL;
    ws = D.scratch;
  } else if ((rc = get_workspace(dev, L.total, &ws))) {
    return rc;
  }

  StageClock clk(!fixed_ws);
  clk.mark(0);
  // K1: squared norms and exponents.
  {
    double* pmA = L.maxA ? (double*)(ws + L.maxA) : nullptr;
    double* pmB = L.maxB ? (double*)(ws + L.maxB) : nullptr;
    dim3 gA((unsigned)((m + 63) / 64), (unsigned)((L.nch + 3) / 4));
    int64_t work = n * L.nch;
    {
      // both operands' partial sums (and the status word's reset) in one launch
      const int64_t nA = (int64_t)gA.x * gA.y, nB = (work + 255) / 256;
      if (small_problem(L) || cache_resident(L, N))
        k1_partials_ab<T, false><<<(unsigned)(nA + nB), 256, 0, g_stream>>>(
            A, lda, m, B, ldb, n, k, L.nch, (double*)(ws + L.partA), pmA,
            (double*)(ws + L.partB), pmB, (int64_t)gA.x, nA, (int*)(ws + L.status));
      else
        k1_partials_ab<T><<<(unsigned)(nA + nB), 256, 0, g_stream>>>(
            A, lda, m, B, ldb, n, k, L.nch, (double*)(ws + L.partA), pmA,
            (double*)(ws + L.partB), pmB, (int64_t)gA.x, nA, (int*)(ws + L.status));
    }
    if (mode != OZ2_MODE_ACCURATE) {
      const int64_t fA = (m + 255) / 256, fB = (n + 255) / 256;
      k1_fold_ab<<<(unsigned)(fA + fB), 256, 0, g_stream>>>(
          (double*)(ws + L.partA), pmA, m, (int32_t*)(ws + L.eA), (double*)(ws + L.SA),
          (double*)(ws + L.partB), pmB, n, (int32_t*)(ws + L.eB), (double*)(ws + L.SB), L.nch,
          mode, tab, (int*)(ws + L.status), fA);
      if (mode == OZ2_MODE_EXACT) {
        // Fallback for the vectors whose squared norm overflowed: the partial
        // sums again over the scaled-down entries (other vectors exit at
        // once), then their fold.
        k1_partials_strided<T, true><<<gA, 256, 0, g_stream>>>(
            A, lda, m, k, L.nch, (double*)(ws + L.partA), nullptr, (const int32_t*)(ws + L.eA));
        k1_partials_contig<T, true><<<(unsigned)((work + 255) / 256), 256, 0, g_stream>>>(
            B, ldb, n, k, L.nch, (double*)(ws + L.partB), nullptr, (const int32_t*)(ws + L.eB));
        k1_fold_rescale<<<(unsigned)((m + 255) / 256), 256, 0, g_stream>>>(
            (double*)(ws + L.partA), L.nch, m, tab, (int32_t*)(ws + L.eA), (double*)(ws + L.SA),
            (int*)(ws + L.status));
        k1_fold_rescale<<<(unsigned)((n + 255) / 256), 256, 0, g_stream>>>(
            (double*)(ws + L.partB), L.nch, n, tab, (int32_t*)(ws + L.eB), (double*)(ws + L.SB),
            (int*)(ws + L.status));
      }
    } else {
      // Accurate mode (Section 2.3): first scale from the maxima, bar
      // matrices, one INT8 GEMM reduced to row/column maxima, exponents.
      int32_t* e1A = (int32_t*)(ws + L.e1A);
      int32_t* e1B = (int32_t*)(ws + L.e1B);
      k1_fold_first<<<(unsigned)((m + 255) / 256), 256, 0, g_stream>>>(
          (double*)(ws + L.partA), pmA, L.nch, m, e1A, (int*)(ws + L.status));
      k1_fold_first<<<(unsigned)((n + 255) / 256), 256, 0, g_stream>>>(
          (double*)(ws + L.partB), pmB, L.nch, n, e1B, (int*)(ws + L.status));
      dim3 gb((unsigned)(L.Mp / kK2VB), (unsigned)(L.Kp / kK2HB));
      k2_bar_strided<T><<<gb, 256, 0, g_stream>>>(A, lda, m, k, e1A, (int8_t*)(ws + L.barA),
                                                  L.Mp, L.Kp);
      int64_t wb = L.Np * (L.Kp / kK2EPT);
      k2_bar_contig<T><<<(unsigned)((wb + 255) / 256), 256, 0, g_stream>>>(
          B, ldb, n, k, e1B, (int8_t*)(ws + L.barB), L.Np, L.Kp);
      int32_t* cmA = (int32_t*)(ws + L.cmaxA);
      int32_t* cmB = (int32_t*)(ws + L.cmaxB);
      k_fill_i32<<<(unsigned)((L.Mp + 255) / 256), 256, 0, g_stream>>>(cmA, L.Mp, 0);
      k_fill_i32<<<(unsigned)((L.Np + 255) / 256), 256, 0, g_stream>>>(cmB, L.Np, 0);
      launch_gemm<2>(cfg, (const int8_t*)(ws + L.barA), (const int8_t*)(ws + L.barB), nullptr,
                     cmA, cmB, m, n, L, tab, 0, 1);
      k1_accurate_exponent<<<(unsigned)((m + 255) / 256), 256, 0, g_stream>>>(
          e1A, cmA, m, tab, (int32_t*)(ws + L.eA));
      k1_accurate_exponent<<<(unsigned)((n + 255) / 256), 256, 0, g_stream>>>(
          e1B, cmB, n, tab, (int32_t*)(ws + L.eB));
      // no squared norms in this mode: report zeros
      k_fill_i32<<<(unsigned)((2 * m + 255) / 256), 256, 0, g_stream>>>((int32_t*)(ws + L.SA),
                                                                         2 * m, 0);
      k_fill_i32<<<(unsigned)((2 * n + 255) / 256), 256, 0, g_stream>>>((int32_t*)(ws + L.SB),
                                                                         2 * n, 0);
    }
  }
  clk.mark(1);
  if (fused) {
    // K2 for B only, then the fused kernel (stage 2: conversion of A,
    // products, CRT and unscaling).
    const int64_t work = L.Np * (L.Kp / kK2EPT);
    k2_split_contig<T, 2><<<(unsigned)((work + 255) / 256), 256, 0, g_stream>>>(
        B, ldb, n, k, (const int32_t*)(ws + L.eB), tab, N, (int8_t*)(ws + L.RB), L.Np, L.Kp);
    clk.mark(2);
    const unsigned grid = (unsigned)((m + kFuseRows - 1) / kFuseRows);
    const int32_t* eA = (const int32_t*)(ws + L.eA);
    const int32_t* eB = (const int32_t*)(ws + L.eB);
    const int8_t* RB = (const int8_t*)(ws + L.RB);
    switch (N) {
#define OZ2_FUSED(NP)                                                                     \
  case NP:                                                                                \
    k234_fused<T, TO, NP><<<grid, 256, 0, g_stream>>>(A, lda, m, n, k, eA, eB, RB, L.Np,  \
                                                       L.Kp, tab, C, ldc);                \
    break;
      OZ2_FUSED(2) OZ2_FUSED(3) OZ2_FUSED(4) OZ2_FUSED(5) OZ2_FUSED(6) OZ2_FUSED(7)
      OZ2_FUSED(8) OZ2_FUSED(9) OZ2_FUSED(10) OZ2_FUSED(11) OZ2_FUSED(12) OZ2_FUSED(13)
      OZ2_FUSED(14) OZ2_FUSED(15) OZ2_FUSED(16)
#undef OZ2_FUSED
      default: return OZ2_ERR_UNSUPPORTED;
    }
    clk.mark(3);
    clk.mark(4);
    clk.mark(5);
    if (hipGetLastError() != hipSuccess) return OZ2_ERR_HIP;
    clk.finish();
    return 0;
  }
  // K2: integers and residues.
  switch (HT.limbs) {
    case 2: launch_split<T, 2>(A, lda, B, ldb, m, n, k, L, ws, tab, N); break;
    case 3: launch_split<T, 3>(A, lda, B, ldb, m, n, k, L, ws, tab, N); break;
    default: launch_split<T, 4>(A, lda, B, ldb, m, n, k, L, ws, tab, N); break;
  }
  if (fp8) {
    // the two E4M3 digit planes of every residue plane
    const int64_t ga = N * L.Mp * (L.Kp / 16), gb = N * L.Np * (L.Kp / 16);
    k_fp8_digits<<<(unsigned)((ga + 255) / 256), 256, 0, g_stream>>>(
        (const int8_t*)(ws + L.RA), (uint8_t*)(ws + L.FA), N * L.Mp, L.Kp);
    k_fp8_digits<<<(unsigned)((gb + 255) / 256), 256, 0, g_stream>>>(
        (const int8_t*)(ws + L.RB), (uint8_t*)(ws + L.FB), N * L.Np, L.Kp);
  }
  clk.mark(2);
  // K3: N residue products (INT8 engine, or the FP8 one).
  if (fp8) {
    const uint8_t* FA = (const uint8_t*)(ws + L.FA);
    const uint8_t* FB = (const uint8_t*)(ws + L.FB);
    const unsigned tiles = (unsigned)((L.Mp / kF8Tile) * (L.Np / kF8Tile));
    if (dbg) {
      if (dbg->Ct)
        k3_gemm_f8<1><<<tiles, 256, 0, g_stream>>>(FA, FB, nullptr, dbg->Ct, m, n, L.Mp, L.Np,
                                                   L.Kp, tab, dbg->t, 0, L.Kp);
    } else {
      for (int64_t k0 = 0; k0 < L.Kp; k0 += OZ2_K_BLOCK) {
        const int64_t klen = std::min<int64_t>(OZ2_K_BLOCK, L.Kp - k0);
        if (k0 == 0)
          k3_gemm_f8<0><<<tiles * N, 256, 0, g_stream>>>(FA, FB, (uint8_t*)(ws + L.U), nullptr,
                                                         m, n, L.Mp, L.Np, L.Kp, tab, 0, k0, klen);
        else
          k3_gemm_f8<3><<<tiles * N, 256, 0, g_stream>>>(FA, FB, (uint8_t*)(ws + L.U), nullptr,
                                                         m, n, L.Mp, L.Np, L.Kp, tab, 0, k0, klen);
      }
    }
  } else if (dbg) {
    if (dbg->Ct)
      launch_gemm<1>(cfg, (const int8_t*)(ws + L.RA), (const int8_t*)(ws + L.RB), nullptr,
                     dbg->Ct, nullptr, m, n, L, tab, dbg->t, 1);
  } else {
    launch_gemm_blocked(cfg, (const int8_t*)(ws + L.RA), (const int8_t*)(ws + L.RB),
                        (uint8_t*)(ws + L.U), m, n, L, tab, N);
  }
  clk.mark(3);
  // K4: CRT and unscaling.
  if (!dbg) {
    switch (HT.slices) {
      case 1: launch_crt<1, TO>(L, ws, tab, N, m, n, C, ldc); break;
      case 2: launch_crt<2, TO>(L, ws, tab, N, m, n, C, ldc); break;
      case 3: launch_crt<3, TO>(L, ws, tab, N, m, n, C, ldc); break;
      default: launch_crt<4, TO>(L, ws, tab, N, m, n, C, ldc); break;
    }
  }
  clk.mark(4);
  clk.mark(5);
  if (hipGetLastError() != hipSuccess) return OZ2_ERR_HIP;
  if (dbg) {
    hipStream_t s = g_stream;
    bool ok = true;
    if (dbg->eA) ok &= hipMemcpyAsync(dbg->eA, ws + L.eA, 4 * m, hipMemcpyDeviceToDevice, s) == hipSuccess;
    if (dbg->eB) ok &= hipMemcpyAsync(dbg->eB, ws + L.eB, 4 * n, hipMemcpyDeviceToDevice, s) == hipSuccess;
    if (dbg->SA) ok &= hipMemcpyAsync(dbg->SA, ws + L.SA, 8 * m, hipMemcpyDeviceToDevice, s) == hipSuccess;
    if (dbg->SB) ok &= hipMemcpyAsync(dbg->SB, ws + L.SB, 8 * n, hipMemcpyDeviceToDevice, s) == hipSuccess;
    for (int t = 0; t < N && ok; ++t) {
      if (dbg->RA)
        ok &= hipMemcpy2DAsync(dbg->RA + (size_t)t * m * k, k, ws + L.RA + (size_t)t * L.Mp * L.Kp,
                               L.Kp, k, m, hipMemcpyDeviceToDevice, s) == hipSuccess;
      if (dbg->RB)
        ok &= hipMemcpy2DAsync(dbg->RB + (size_t)t * n * k, k, ws + L.RB + (size_t)t * L.Np * L.Kp,
                               L.Kp, k, n, hipMemcpyDeviceToDevice, s) == hipSuccess;
    }
    if (!ok || hipStreamSynchronize(s) != hipSuccess) return OZ2_ERR_HIP;
  }
  clk.finish();
  return 0;
}

// Complex products (ZGEMM: T = double, CGEMM: T = float).  A, B and C hold
// interleaved (re, im) pairs, column-major, leading dimensions in complex
// entries.  Revised and original fast modes.
template <typename T>
int run_complex(int64_t m, int64_t n, int64_t k, const T* A, int64_t lda, const T* B,
                int64_t ldb, T* C, int64_t ldc, int N, int mode) {
  int rc = check_args(m, n, k, A, lda, B, ldb, C, ldc, N, mode, true);
  if (rc) return rc;
  if (mode == OZ2_MODE_ACCURATE || (mode & OZ2_ENGINE_FP8)) return OZ2_ERR_UNSUPPORTED;
  const uintptr_t align = 2 * sizeof(T) - 1;   // one complex entry
  if (reinterpret_cast<uintptr_t>(A) & align) return -4;
  if (reinterpret_cast<uintptr_t>(B) & align) return -6;
  if (reinterpret_cast<uintptr_t>(C) & align) return -8;
  if (m == 0 || n == 0) return 0;
  int dev;
  if ((rc = ensure_device(&dev))) return rc;
  DevState& D = g_dev[dev];
  if (k == 0) {
    k_zero<T><<<(unsigned)((2 * m * n + 255) / 256), 256, 0, g_stream>>>(C, 2 * m, n, 2 * ldc);
    return hipGetLastError() == hipSuccess ? 0 : OZ2_ERR_HIP;
  }
  build_host_tables();
  if (!g_host_tables_ok[0][N]) return OZ2_ERR_UNSUPPORTED;
  const ModTable& HT = g_host_tables[0][N];
  const ModTable* tab = D.d_tables + N;

  const int cfg = tile_config(m, n, k, N);
  Layout L = make_layout(m, n, k, N, mode, kTileBM[cfg], kTileBN[cfg], 3);
  char* ws = nullptr;
  if ((rc = get_workspace(dev, L.total, &ws))) return rc;

  StageClock clk;
  clk.mark(0);
  // K1: squared norms over the 2k components and exponents.
  k_clear_status<<<1, 64, 0, g_stream>>>((int*)(ws + L.status));
  {
    double* pmA = L.maxA ? (double*)(ws + L.maxA) : nullptr;
    double* pmB = L.maxB ? (double*)(ws + L.maxB) : nullptr;
    dim3 gA((unsigned)((m + 63) / 64), (unsigned)((L.nch + 3) / 4));
    k1_partials_strided_cplx<T><<<gA, 256, 0, g_stream>>>(A, lda, m, k, L.nch,
                                                          (double*)(ws + L.partA), pmA);
    int64_t work = n * L.nch;
    k1_partials_contig<T><<<(unsigned)((work + 255) / 256), 256, 0, g_stream>>>(
        B, 2 * ldb, n, 2 * k, L.nch, (double*)(ws + L.partB), pmB);
    k1_fold<<<(unsigned)((m + 255) / 256), 256, 0, g_stream>>>(
        (double*)(ws + L.partA), pmA, L.nch, m, mode, tab, (int32_t*)(ws + L.eA),
        (double*)(ws + L.SA), (int*)(ws + L.status));
    k1_fold<<<(unsigned)((n + 255) / 256), 256, 0, g_stream>>>(
        (double*)(ws + L.partB), pmB, L.nch, n, mode, tab, (int32_t*)(ws + L.eB),
        (double*)(ws + L.SB), (int*)(ws + L.status));
    if (mode == OZ2_MODE_EXACT) {
      k1_partials_strided_cplx<T, true><<<gA, 256, 0, g_stream>>>(
          A, lda, m, k, L.nch, (double*)(ws + L.partA), nullptr, (const int32_t*)(ws + L.eA));
      k1_partials_contig<T, true><<<(unsigned)((work + 255) / 256), 256, 0, g_stream>>>(
          B, 2 * ldb, n, 2 * k, L.nch, (double*)(ws + L.partB), nullptr,
          (const int32_t*)(ws + L.eB));
      k1_fold_rescale<<<(unsigned)((m + 255) / 256), 256, 0, g_stream>>>(
          (double*)(ws + L.partA), L.nch, m, tab, (int32_t*)(ws + L.eA), (double*)(ws + L.SA),
          (int*)(ws + L.status));
      k1_fold_rescale<<<(unsigned)((n + 255) / 256), 256, 0, g_stream>>>(
          (double*)(ws + L.partB), L.nch, n, tab, (int32_t*)(ws + L.eB), (double*)(ws + L.SB),
          (int*)(ws + L.status));
    }
  }
  clk.mark(1);
  // K2: integers and the residues of the three components.
  {
    const int64_t gx = L.Mp / kK2CVB;
    const int64_t blocksA = gx * (L.Kp / kK2CHB);
    const int64_t workB = L.Np * (L.Kp / kK2CEPL);
    const int32_t* eA = (const int32_t*)(ws + L.eA);
    const int32_t* eB = (const int32_t*)(ws + L.eB);
    int8_t* RA = (int8_t*)(ws + L.RA);
    int8_t* RB = (int8_t*)(ws + L.RB);
    if (HT.limbs == 2) {
      k2_split_strided_cplx<T, 2><<<(unsigned)blocksA, 256, 0, g_stream>>>(
          A, lda, m, k, eA, tab, N, RA, L.Mp, L.Kp, gx);
      k2_split_contig_cplx<T, 2><<<(unsigned)((workB + 255) / 256), 256, 0, g_stream>>>(
          B, ldb, n, k, eB, tab, N, RB, L.Np, L.Kp);
    } else {
      k2_split_strided_cplx<T, 3><<<(unsigned)blocksA, 256, 0, g_stream>>>(
          A, lda, m, k, eA, tab, N, RA, L.Mp, L.Kp, gx);
      k2_split_contig_cplx<T, 3><<<(unsigned)((workB + 255) / 256), 256, 0, g_stream>>>(
          B, ldb, n, k, eB, tab, N, RB, L.Np, L.Kp);
    }
  }
  clk.mark(2);
  // K3: 3N INT8 GEMMs, one launch (per k block) for each component.
  for (int c = 0; c < 3; ++c)
    launch_gemm_blocked(cfg, (const int8_t*)(ws + L.RA) + (size_t)c * N * L.Mp * L.Kp,
                        (const int8_t*)(ws + L.RB) + (size_t)c * N * L.Np * L.Kp,
                        (uint8_t*)(ws + L.U) + (size_t)c * N * L.Mp * L.Np, m, n, L, tab, N);
  clk.mark(3);
  // K4: both parts, CRT and unscaling.
  {
    const int64_t blocks = ((m + 31) / 32) * ((n + 31) / 32);
    const unsigned grid = (unsigned)((blocks + 3) / 4);
    const uint8_t* U = (const uint8_t*)(ws + L.U);
    const int32_t* eA = (const int32_t*)(ws + L.eA);
    const int32_t* eB = (const int32_t*)(ws + L.eB);
    switch (HT.slices) {
      case 1: k4_crt_cplx<1, T><<<grid, 256, 0, g_stream>>>(U, eA, eB, tab, N, m, n, L.Mp, L.Np, C, ldc); break;
      case 2: k4_crt_cplx<2, T><<<grid, 256, 0, g_stream>>>(U, eA, eB, tab, N, m, n, L.Mp, L.Np, C, ldc); break;
      case 3: k4_crt_cplx<3, T><<<grid, 256, 0, g_stream>>>(U, eA, eB, tab, N, m, n, L.Mp, L.Np, C, ldc); break;
      default: k4_crt_cplx<4, T><<<grid, 256, 0, g_stream>>>(U, eA, eB, tab, N, m, n, L.Mp, L.Np, C, ldc); break;
    }
  }
  clk.mark(4);
  clk.mark(5);
  if (hipGetLastError() != hipSuccess) return OZ2_ERR_HIP;
  clk.finish();
  return 0;
}

// ---------------------------------------------------------------------------
// Batched path: graph built once per batch signature, replayed per call.
// ---------------------------------------------------------------------------

struct BatchState {
  bool valid = false;
  uint64_t sig = 0;
  int dev = -1;
  char* ws = nullptr;               // workspace the graph's kernels address
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap = nullptr;
  std::vector<BatchProb> uploaded;  // descriptors as last written to the device
  uint64_t epoch = 0;               // g_ws_epoch when the tables were written
};
BatchState g_batch;

uint64_t mix64(uint64_t h, uint64_t v) {
  h ^= v + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
  return h;
}

void batch_release() {
  if (g_batch.exec) (void)hipGraphExecDestroy(g_batch.exec);
  if (g_batch.graph) (void)hipGraphDestroy(g_batch.graph);
  g_batch.exec = nullptr;
  g_batch.graph = nullptr;
  g_batch.valid = false;
}

// Scratch of the phi estimate (operand descriptors and per-block partial
// statistics) for `ns` operands; it sits right after the status word of the
// workspace.
size_t tune_scratch_bytes(size_t ns) {
  return align256(sizeof(StatSrc) * ns) + align256(sizeof(double) * 2 * kStatBlocks * ns);
}

// phi of each operand (pooled within-vector variance of log|x|,
// oz2_autotune.hpp): one
// launch for all of them on the library stream into the workspace scratch
// at `scratch`, then a synchronising copy of the per-block partials.
int estimate_phis(char* scratch, const std::vector<StatSrc>& srcs, std::vector<double>* phis) {
  const size_t ns = srcs.size();
  phis->assign(ns, 0.0);
  if (ns == 0) return 0;
  const size_t off_part = align256(sizeof(StatSrc) * ns);
  std::vector<double> part(2 * kStatBlocks * ns);
  if (hipMemcpyAsync(scratch, srcs.data(), sizeof(StatSrc) * ns, hipMemcpyHostToDevice,
                     g_stream) != hipSuccess)
    return OZ2_ERR_HIP;
  k_logstats<<<(unsigned)(ns * kStatBlocks), 256, 0, g_stream>>>(
      reinterpret_cast<const StatSrc*>(scratch), reinterpret_cast<double*>(scratch + off_part));
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(part.data(), scratch + off_part, sizeof(double) * part.size(),
                     hipMemcpyDeviceToHost, g_stream) != hipSuccess ||
      hipStreamSynchronize(g_stream) != hipSuccess)
    return OZ2_ERR_HIP;
  for (size_t i = 0; i < ns; ++i) (*phis)[i] = phi_from_partials(part.data() + 2 * kStatBlocks * i);
  return 0;
}

// Everything a batch needs, planned on the host: the problems that run (m, n,
// k > 0), their workspace layouts, the per-stage block tables and the regions
// of the batch's workspace:
//   [status | phi scratch | descriptors | block prefixes | work items |
//    block owners | per-problem regions (Layout of each problem)]
struct BatchPlan {
  std::vector<int> act;            // index into the problem array
  std::vector<Layout> lay;
  std::vector<size_t> base;        // offset of each active problem's region
  std::vector<int64_t> prefix;     // (na + 1) per stage
  int64_t blocks[kB_NSTAGES];
  int64_t owner_off[kB_NSTAGES];
  int64_t total_blocks = 0, nitems = 0;
  size_t off_tune = 256, off_probs = 0, off_prefix = 0, off_items = 0, off_owner = 0;
  size_t total = 0;
  uint64_t sig = 0;
};

// Validates the batch (every N resolved, 2..20) and plans it.  `tune_ops`
// reserves phi scratch for that many operands.
int plan_batch(int batch, const oz2_problem* P, int mode, size_t tune_ops, BatchPlan* pl,
               int* bad) {
  if (bad) *bad = -1;
  if (batch < 0) return -1;
  if (batch > 0 && !P) return -2;
  if (mode != OZ2_MODE_REVISED && mode != OZ2_MODE_ORIGINAL) return -3;   // fast modes only
  if (batch > 65535) return OZ2_ERR_TOO_LARGE;
  build_host_tables();
  for (int i = 0; i < batch; ++i) {
    const oz2_problem& q = P[i];
    int rc = check_args(q.m, q.n, q.k, q.A, q.lda, q.B, q.ldb, q.C, q.ldc, q.N, mode, true);
    if (!rc && q.k > OZ2_K_BLOCK) rc = OZ2_ERR_K_TOO_LARGE;  // no k blocking in a batch
    if (!rc && (q.m > 65535 * (int64_t)kBatchTile || q.n > 65535 * (int64_t)kBatchTile))
      rc = OZ2_ERR_TOO_LARGE;
    if (!rc && q.m > 0 && q.n > 0 && q.k > 0 &&
        (!g_host_tables_ok[0][q.N] || g_host_tables[0][q.N].limbs > kBatchLimbs))
      rc = OZ2_ERR_UNSUPPORTED;
    if (rc) {
      if (bad) *bad = i;
      return rc;
    }
  }
  pl->act.clear();
  for (int i = 0; i < batch; ++i)
    if (P[i].m > 0 && P[i].n > 0 && P[i].k > 0) pl->act.push_back(i);
  const int na = (int)pl->act.size();
  pl->lay.assign(na, Layout());
  pl->base.assign(na, 0);
  pl->nitems = 0;
  uint64_t sig = mix64(0, (uint64_t)na);
  sig = mix64(sig, (uint64_t)mode);
  for (int a = 0; a < na; ++a) {
    const oz2_problem& q = P[pl->act[a]];
    pl->lay[a] = make_layout(q.m, q.n, q.k, q.N, mode, kBatchTile, kBatchTile);
    pl->nitems += (int64_t)q.N * (pl->lay[a].Mp / kBatchTile) * (pl->lay[a].Np / kBatchTile);
    sig = mix64(mix64(mix64(mix64(sig, (uint64_t)q.m), (uint64_t)q.n), (uint64_t)q.k),
                (uint64_t)q.N);
  }
  if (pl->nitems > INT32_MAX) return OZ2_ERR_TOO_LARGE;
  pl->prefix.assign((size_t)(na + 1) * kB_NSTAGES, 0);
  for (int st = 0; st < kB_NSTAGES; ++st) {
    int64_t acc = 0;
    for (int a = 0; a < na; ++a) {
      const oz2_problem& q = P[pl->act[a]];
      const Layout& L = pl->lay[a];
      int64_t c = 0;
      switch (st) {
        case kB_K1A: c = ((q.m + 63) / 64) * ((L.nch + 3) / 4); break;
        case kB_K1B: c = (q.n * L.nch + 255) / 256; break;
        case kB_FOLDA: c = (q.m + 255) / 256; break;
        case kB_FOLDB: c = (q.n + 255) / 256; break;
        case kB_K2A: c = (L.Mp / kK2VB) * (L.Kp / kK2HB); break;
        case kB_K2B: c = (L.Np * (L.Kp / kK2EPT) + 255) / 256; break;
        default: c = (((q.m + 31) / 32) * ((q.n + 31) / 32) * kK4WavesPerBlock + 3) / 4; break;
      }
      pl->prefix[(size_t)st * (na + 1) + a] = acc;
      acc += c;
    }
    pl->prefix[(size_t)st * (na + 1) + na] = acc;
    pl->blocks[st] = acc;
    if (acc > INT32_MAX) return OZ2_ERR_TOO_LARGE;
  }
  // the A and B halves of a step share one launch
  for (int st : {kB_K1A, kB_FOLDA, kB_K2A})
    if (pl->blocks[st] + pl->blocks[st + 1] > INT32_MAX) return OZ2_ERR_TOO_LARGE;
  pl->total_blocks = 0;
  for (int st = 0; st < kB_NSTAGES; ++st) {
    pl->owner_off[st] = pl->total_blocks;
    pl->total_blocks += pl->blocks[st];
  }
  pl->off_tune = 256;
  pl->off_probs = pl->off_tune + tune_scratch_bytes(tune_ops);
  pl->off_prefix = pl->off_probs + align256(sizeof(BatchProb) * na);
  pl->off_items = pl->off_prefix + align256(sizeof(int64_t) * (na + 1) * kB_NSTAGES);
  pl->off_owner = pl->off_items + align256(sizeof(WorkItem) * (size_t)pl->nitems);
  size_t off = pl->off_owner + align256(sizeof(uint16_t) * (size_t)pl->total_blocks);
  for (int a = 0; a < na; ++a) {
    pl->base[a] = off;
    off += pl->lay[a].total;
  }
  pl->total = off;
  // where the tables and regions sit (they move with the phi scratch)
  pl->sig = mix64(mix64(sig, (uint64_t)pl->off_probs), (uint64_t)pl->total);
  return 0;
}

// The work list of the persistent GEMM: (problem, plane, tile) items sorted
// by decreasing k, regrouped for the XCDs.
std::vector<WorkItem> batch_items(const oz2_problem* P, const BatchPlan& pl) {
  const int na = (int)pl.act.size();
  std::vector<int> order(na);
  for (int a = 0; a < na; ++a) order[a] = a;
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return P[pl.act[x]].k > P[pl.act[y]].k; });
  std::vector<WorkItem> items;
  items.reserve((size_t)pl.nitems);
  for (int a : order) {
    const oz2_problem& q = P[pl.act[a]];
    const int tmn = (int)(pl.lay[a].Mp / kBatchTile), tnn = (int)(pl.lay[a].Np / kBatchTile);
    for (int t = 0; t < q.N; ++t)
      for (int tn = 0; tn < tnn; ++tn)
        for (int tm = 0; tm < tmn; ++tm)
          items.push_back(WorkItem{(uint16_t)a, (uint16_t)t, (uint16_t)tm, (uint16_t)tn});
  }
  // XCD-local order.  Workgroups are dispatched round-robin over the 8
  // XCDs (each with its own L2) and workgroup b takes items b, b + G, ...
  // (G = 2 * CUs, a multiple of 8, for any list of that many items or
  // more), so item i runs on XCD i % 8.  Items are regrouped so that the tiles of one
  // plane of one problem run on one XCD, at about the same time, and
  // share their row and column panels in its L2 (dealt round-robin they
  // were spread over all 8, each L2 fetching nearly every panel):
  // planes (runs of one plane's tiles, in the list's order of
  // decreasing k) go to the XCD with the least work so far that still
  // has room, split where an XCD is full; per-XCD lengths are exactly
  // nitems / 8 (+1 for the first nitems % 8); item i of the list is
  // position i / 8 of XCD i % 8's sequence.  Measured on the 256-problem
  // batch: 4% less time for the whole call.
  const int64_t NI = (int64_t)items.size();
  std::vector<std::vector<WorkItem>> seq(8);
  std::vector<int64_t> cap(8), work(8, 0);
  for (int x = 0; x < 8; ++x) cap[x] = NI / 8 + (x < NI % 8 ? 1 : 0);
  size_t pos = 0;
  while (pos < items.size()) {
    size_t end = pos;
    while (end < items.size() && items[end].p == items[pos].p && items[end].t == items[pos].t) ++end;
    const int64_t nk = pl.lay[items[pos].p].Kp / kBatchBK;
    while (pos < end) {
      int best = -1;
      for (int x = 0; x < 8; ++x)
        if ((int64_t)seq[x].size() < cap[x] && (best < 0 || work[x] < work[best])) best = x;
      const int64_t room = cap[best] - (int64_t)seq[best].size();
      const size_t take = (size_t)std::min<int64_t>(room, (int64_t)(end - pos));
      for (size_t q = 0; q < take; ++q) seq[best].push_back(items[pos + q]);
      work[best] += (int64_t)take * nk;
      pos += take;
    }
  }
  for (int64_t i = 0; i < NI; ++i) items[(size_t)i] = seq[(size_t)(i % 8)][(size_t)(i / 8)];
  return items;
}

// The batch's kernels on stream s: status reset, the per-stage grids, the
// persistent GEMM, the CRT grid.  With a StageClock (direct launches on the
// library stream) events separate the stages as in ozaki2_dgemm.
void enqueue_batch(hipStream_t s, const BatchPlan& pl, char* ws, int64_t gemm_grid,
                   StageClock* clk) {
  const int na = (int)pl.act.size();
  const BatchProb* d_probs = (const BatchProb*)(ws + pl.off_probs);
  const int64_t* d_prefix = (const int64_t*)(ws + pl.off_prefix);
  const uint16_t* d_owner = (const uint16_t*)(ws + pl.off_owner);
  int* d_status = (int*)ws;
  if (clk) clk->mark(0);
  kb_reset<<<1, 64, 0, s>>>(d_status);
#define OZ2_STAGE(ST)                                                                   \
  if (pl.blocks[ST] > 0)                                                                \
    kb_stage<ST><<<(unsigned)pl.blocks[ST], 256, 0, s>>>(d_probs, d_prefix,               \
                                                       d_owner + pl.owner_off[ST], na, d_status);
#define OZ2_STAGE_PAIR(S1, S2)                                                            \
  static_assert(S2 == S1 + 1, "owner entries of S2 follow S1's");                       \
  if (pl.blocks[S1] + pl.blocks[S2] > 0)                                                \
    kb_stage_pair<S1, S2><<<(unsigned)(pl.blocks[S1] + pl.blocks[S2]), 256, 0, s>>>(       \
        d_probs, d_prefix, d_owner + pl.owner_off[S1], na, pl.blocks[S1], d_status);
  OZ2_STAGE_PAIR(kB_K1A, kB_K1B)
  OZ2_STAGE_PAIR(kB_FOLDA, kB_FOLDB)
  if (clk) clk->mark(1);
  OZ2_STAGE_PAIR(kB_K2A, kB_K2B)
  if (clk) clk->mark(2);
  kb_gemm<<<(unsigned)gemm_grid, 256, 0, s>>>(d_probs, (const WorkItem*)(ws + pl.off_items),
                                              (int)pl.nitems);
  if (clk) clk->mark(3);
  OZ2_STAGE(kB_K4)
#undef OZ2_STAGE_PAIR
#undef OZ2_STAGE
  if (clk) {
    clk->mark(4);
    clk->mark(5);
  }
}

// Batched path with every N given.  All device data of the batch (status,
// descriptors, block tables, work list, per-problem regions) lives in the
// workspace; the first call with a new signature (shapes, N, mode, device,
// workspace address) writes the tables, synchronises and captures the
// graph; later calls only refresh the caller pointers that changed (kernel
// arguments of kb_set_ptrs, no host buffer to keep alive) and replay it.
int run_batched_resolved(int batch, const oz2_problem* P, int mode, size_t tune_ops, int* bad) {
  BatchPlan pl;
  int rc = plan_batch(batch, P, mode, tune_ops, &pl, bad);
  if (rc) return rc;
  if (batch == 0) return 0;
  int dev;
  if ((rc = ensure_device(&dev))) return rc;
  DevState& D = g_dev[dev];
  char* ws = nullptr;
  if (!pl.act.empty() && (rc = get_workspace(dev, pl.total, &ws, true))) return rc;

  for (int i = 0; i < batch; ++i) {
    const oz2_problem& q = P[i];
    if (q.m > 0 && q.n > 0 && q.k == 0)
      k_zero<double><<<(unsigned)((q.m * q.n + 255) / 256), 256, 0, g_stream>>>(q.C, q.m, q.n,
                                                                                q.ldc);
  }
  if (pl.act.empty()) return hipGetLastError() == hipSuccess ? 0 : OZ2_ERR_HIP;
  const int na = (int)pl.act.size();

  int cus = 256;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  // two resident workgroups per CU (64 KiB of LDS each; 64-byte slabs at
  // three per CU measured 1-2% slower, four at <= 128 registers 6% slower)
  const int64_t gemm_grid = std::min<int64_t>(pl.nitems, (int64_t)cus * 2);

  const uint64_t sig = mix64(mix64(pl.sig, (uint64_t)dev), (uint64_t)(uintptr_t)ws);
  std::vector<BatchProb> probs(na);
  for (int a = 0; a < na; ++a) {
    const oz2_problem& q = P[pl.act[a]];
    const Layout& L = pl.lay[a];
    char* w = ws + pl.base[a];
    BatchProb& B = probs[a];
    B.A = q.A;
    B.B = q.B;
    B.C = q.C;
    B.m = q.m; B.n = q.n; B.k = q.k;
    B.lda = q.lda; B.ldb = q.ldb; B.ldc = q.ldc;
    B.Mp = L.Mp; B.Np = L.Np; B.Kp = L.Kp; B.nch = L.nch;
    B.N = q.N;
    B.mode = mode;
    B.tab = D.d_tables + q.N;
    B.eA = (int32_t*)(w + L.eA);
    B.eB = (int32_t*)(w + L.eB);
    B.partA = (double*)(w + L.partA);
    B.partB = (double*)(w + L.partB);
    B.maxA = L.maxA ? (double*)(w + L.maxA) : nullptr;
    B.maxB = L.maxB ? (double*)(w + L.maxB) : nullptr;
    B.SA = (double*)(w + L.SA);
    B.SB = (double*)(w + L.SB);
    B.RA = (int8_t*)(w + L.RA);
    B.RB = (int8_t*)(w + L.RB);
    B.U = (uint8_t*)(w + L.U);
    B.k1a_gx = (q.m + 63) / 64;
  }

  // Tables (descriptors, block prefixes and owners, work list): written in
  // stream order after any earlier work on this workspace, and waited for
  // (the host vectors are pageable memory).
  auto upload_tables = [&]() -> int {
    std::vector<WorkItem> items = batch_items(P, pl);
    std::vector<uint16_t> owner((size_t)pl.total_blocks);
    for (int st = 0; st < kB_NSTAGES; ++st)
      for (int a = 0; a < na; ++a)
        for (int64_t bb = pl.prefix[(size_t)st * (na + 1) + a];
             bb < pl.prefix[(size_t)st * (na + 1) + a + 1]; ++bb)
          owner[(size_t)(pl.owner_off[st] + bb)] = (uint16_t)a;
    if (hipMemcpyAsync(ws + pl.off_probs, probs.data(), sizeof(BatchProb) * na,
                       hipMemcpyHostToDevice, g_stream) != hipSuccess ||
        hipMemcpyAsync(ws + pl.off_prefix, pl.prefix.data(), pl.prefix.size() * sizeof(int64_t),
                       hipMemcpyHostToDevice, g_stream) != hipSuccess ||
        hipMemcpyAsync(ws + pl.off_owner, owner.data(), owner.size() * sizeof(uint16_t),
                       hipMemcpyHostToDevice, g_stream) != hipSuccess ||
        hipMemcpyAsync(ws + pl.off_items, items.data(), items.size() * sizeof(WorkItem),
                       hipMemcpyHostToDevice, g_stream) != hipSuccess ||
        hipStreamSynchronize(g_stream) != hipSuccess)
      return OZ2_ERR_HIP;
    g_batch.uploaded = probs;
    g_batch.epoch = g_ws_epoch;
    return 0;
  };

  if (!g_batch.valid || g_batch.sig != sig) {
    batch_release();
    g_batch.uploaded.clear();
    if (!g_batch.cap && hipStreamCreateWithFlags(&g_batch.cap, hipStreamNonBlocking) != hipSuccess)
      return OZ2_ERR_HIP;
    if ((rc = upload_tables())) return rc;
    hipStream_t cs = g_batch.cap;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return OZ2_ERR_HIP;
    enqueue_batch(cs, pl, ws, gemm_grid, nullptr);
    hipError_t e1 = hipStreamEndCapture(cs, &g_batch.graph);
    if (e1 != hipSuccess || !g_batch.graph) return OZ2_ERR_HIP;
    if (hipGraphInstantiate(&g_batch.exec, g_batch.graph, nullptr, nullptr, 0) != hipSuccess)
      return OZ2_ERR_HIP;
    g_batch.sig = sig;
    g_batch.dev = dev;
    g_batch.ws = ws;
    g_batch.valid = true;
  } else if (g_batch.epoch != g_ws_epoch) {
    // Same signature, but the workspace was used by other calls since the
    // tables were written (their regions overlap the tables): write them
    // again; the captured graph addresses the same places.
    if ((rc = upload_tables())) return rc;
  } else {
    // Same signature and untouched tables: refresh the caller pointers that
    // changed, in chunks carried as kernel arguments (stream ordered after
    // the previous replay).
    BatchPtrs chunk;
    for (int a0 = 0; a0 < na; a0 += kBatchPtrChunk) {
      const int cnt = std::min(kBatchPtrChunk, na - a0);
      bool changed = false;
      for (int c = 0; c < cnt; ++c) {
        const BatchProb& nw = probs[a0 + c];
        const BatchProb& old = g_batch.uploaded[a0 + c];
        changed |= nw.A != old.A || nw.B != old.B || nw.C != old.C;
        chunk.A[c] = nw.A;
        chunk.B[c] = nw.B;
        chunk.C[c] = nw.C;
      }
      if (!changed) continue;
      chunk.first = a0;
      chunk.count = cnt;
      kb_set_ptrs<<<1, 64, 0, g_stream>>>((BatchProb*)(ws + pl.off_probs), chunk);
      for (int c = 0; c < cnt; ++c) g_batch.uploaded[a0 + c] = probs[a0 + c];
    }
  }

  if (g_timing) {
    // Timed calls launch the same kernels directly, with stage events.
    StageClock clk;
    enqueue_batch(g_stream, pl, ws, gemm_grid, &clk);
    if (hipGetLastError() != hipSuccess) return OZ2_ERR_HIP;
    clk.finish();
    return 0;
  }
  if (hipGraphLaunch(g_batch.exec, g_stream) != hipSuccess) return OZ2_ERR_HIP;
  return hipGetLastError() == hipSuccess ? 0 : OZ2_ERR_HIP;
}

// Upper bound of a batch's workspace: problems with N = 0 are planned with
// OZ2_N_MAX, and phi scratch is reserved for two operands per such problem.
int batch_bound_plan(int batch, const oz2_problem* problems, int mode, BatchPlan* pl,
                     size_t* tune_ops, std::vector<oz2_problem>* Q, int* bad) {
  if (batch < 0) return -1;
  if (batch > 0 && !problems) return -2;
  Q->assign(problems, problems + batch);
  size_t ops = 0;
  for (auto& q : *Q)
    if (q.N == 0) {
      q.N = OZ2_N_MAX;
      if (q.m > 0 && q.n > 0 && q.k > 0) ops += 2;
    }
  *tune_ops = ops;
  return plan_batch(batch, Q->data(), mode, ops, pl, bad);
}

}  // namespace

extern "C" {

int ozaki2_dgemm_batched(int batch, oz2_problem* problems, int mode, double target_max_rel_err,
                         int* bad_index) {
  if (bad_index) *bad_index = -1;
  if (batch < 0) return -1;
  if (batch > 0 && !problems) return -2;
  if (mode != OZ2_MODE_REVISED && mode != OZ2_MODE_ORIGINAL) return -3;
  bool any_auto = false;
  for (int i = 0; i < batch; ++i) any_auto |= problems[i].N == 0;
  if (any_auto && !(target_max_rel_err > 0.0 && target_max_rel_err <= 1.0)) return -4;
  // Validate (and size the workspace) with OZ2_N_MAX for the problems that
  // leave N to the library, so that nothing is launched for an invalid batch
  // and the workspace bound is the one ozaki2_dgemm_batched_workspace_size
  // reports.
  BatchPlan bound;
  size_t tune_ops = 0;
  std::vector<oz2_problem> Q;
  int rc = batch_bound_plan(batch, problems, mode, &bound, &tune_ops, &Q, bad_index);
  if (rc) return rc;
  if (any_auto && tune_ops > 0) {
    std::vector<StatSrc> srcs;
    std::vector<int> who;
    for (int i = 0; i < batch; ++i) {
      const oz2_problem& q = problems[i];
      if (q.N != 0 || q.m == 0 || q.n == 0 || q.k == 0) continue;
      srcs.push_back(stat_src(q.A, q.m, q.k, q.lda, 0));   // the rows of A
      srcs.push_back(stat_src(q.B, q.k, q.n, q.ldb, 1));   // the columns of B
      who.push_back(i);
    }
    int dev;
    if ((rc = ensure_device(&dev))) return rc;
    char* ws = nullptr;
    // the phi scratch ends where this plan's tables begin
    if ((rc = get_workspace(dev, bound.total, &ws, true))) return rc;
    std::vector<double> phis;
    if ((rc = estimate_phis(ws + bound.off_tune, srcs, &phis))) return rc;
    for (size_t w = 0; w < who.size(); ++w)
      Q[who[w]].N = tune_pick_N(Q[who[w]].k, std::max(phis[2 * w], phis[2 * w + 1]),
                                target_max_rel_err);
  }
  for (int i = 0; i < batch; ++i) {
    const oz2_problem& q = problems[i];
    problems[i].N_used = (q.N == 0 && (q.m == 0 || q.n == 0 || q.k == 0)) ? 0 : Q[i].N;
  }
  return run_batched_resolved(batch, Q.data(), mode, tune_ops, bad_index);
}

int ozaki2_dgemm_batched_workspace_size(int batch, const oz2_problem* problems, int mode,
                                        size_t* bytes) {
  if (batch < 0) return -1;
  if (batch > 0 && !problems) return -2;
  if (mode != OZ2_MODE_REVISED && mode != OZ2_MODE_ORIGINAL) return -3;
  if (!bytes) return -4;
  BatchPlan bound;
  size_t tune_ops = 0;
  std::vector<oz2_problem> Q;
  int rc = batch_bound_plan(batch, problems, mode, &bound, &tune_ops, &Q, nullptr);
  if (rc) return rc;
  *bytes = bound.act.empty() && tune_ops == 0 ? 0 : bound.total;
  return 0;
}

int ozaki2_autotune_N(int64_t k, double phi, double target_max_rel_err, int* N) {
  if (k < 0) return -1;
  if (!(phi >= 0.0 && phi <= 1e300)) return -2;
  if (!(target_max_rel_err > 0.0 && target_max_rel_err <= 1.0)) return -3;
  if (!N) return -4;
  *N = tune_pick_N(k, phi, target_max_rel_err);
  return 0;
}

int ozaki2_estimate_phi(int64_t rows, int64_t cols, const double* X, int64_t ld, int vectors,
                        double* phi) {
  if (rows < 0) return -1;
  if (cols < 0) return -2;
  if (!X && rows > 0 && cols > 0) return -3;
  if (ld < (rows > 1 ? rows : 1)) return -4;
  if (vectors != 0 && vectors != 1) return -5;
  if (!phi) return -6;
  *phi = 0.0;
  if (rows == 0 || cols == 0) return 0;
  int dev, rc;
  if ((rc = ensure_device(&dev))) return rc;
  char* ws = nullptr;
  if ((rc = get_workspace(dev, 256 + tune_scratch_bytes(1), &ws))) return rc;
  std::vector<double> phis;
  if ((rc = estimate_phis(ws + 256, {stat_src(X, rows, cols, ld, vectors)}, &phis))) return rc;
  *phi = phis[0];
  return 0;
}


int ozaki2_dgemm(int64_t m, int64_t n, int64_t k, const double* A, int64_t lda,
                 const double* B, int64_t ldb, double* C, int64_t ldc, int N, int mode) {
  return run_gemm<double, double>(m, n, k, A, lda, B, ldb, C, ldc, N, mode, nullptr);
}

int ozaki2_dgemm_noalloc(int64_t m, int64_t n, int64_t k, const double* A, int64_t lda,
                         const double* B, int64_t ldb, double* C, int64_t ldc, int N, int mode) {
  return run_gemm<double, double>(m, n, k, A, lda, B, ldb, C, ldc, N, mode, nullptr, true);
}

int ozaki2_sgemm(int64_t m, int64_t n, int64_t k, const float* A, int64_t lda,
                 const float* B, int64_t ldb, float* C, int64_t ldc, int N, int mode) {
  return run_gemm<float, float>(m, n, k, A, lda, B, ldb, C, ldc, N, mode, nullptr);
}

int ozaki2_zgemm(int64_t m, int64_t n, int64_t k, const double* A, int64_t lda,
                 const double* B, int64_t ldb, double* C, int64_t ldc, int N, int mode) {
  return run_complex<double>(m, n, k, A, lda, B, ldb, C, ldc, N, mode);
}

int ozaki2_cgemm(int64_t m, int64_t n, int64_t k, const float* A, int64_t lda,
                 const float* B, int64_t ldb, float* C, int64_t ldc, int N, int mode) {
  return run_complex<float>(m, n, k, A, lda, B, ldb, C, ldc, N, mode);
}

int ozaki2_zgemm_workspace_size(int64_t m, int64_t n, int64_t k, int N, int mode,
                                size_t* bytes) {
  int rc = check_args(m, n, k, (const void*)16, m > 1 ? m : 1, (const void*)16, k > 1 ? k : 1,
                      (const void*)16, m > 1 ? m : 1, N, mode, true);
  if (rc) return rc;
  if (mode == OZ2_MODE_ACCURATE || (mode & OZ2_ENGINE_FP8)) return OZ2_ERR_UNSUPPORTED;
  if (!bytes) return -6;
  *bytes = (m == 0 || n == 0 || k == 0) ? 0 : make_layout(m, n, k, N, mode, kBM, kBN, 3).total;
  return 0;
}

int ozaki2_set_stream(void* stream) {
  g_stream = reinterpret_cast<hipStream_t>(stream);
  return 0;
}

int ozaki2_workspace_size(int64_t m, int64_t n, int64_t k, int N, int mode, size_t* bytes) {
  int rc = check_args(m, n, k, (const void*)1, m > 1 ? m : 1, (const void*)1, k > 1 ? k : 1,
                      (const void*)1, m > 1 ? m : 1, N, mode, true);
  if (rc) return rc;
  if (!bytes) return -6;
  if ((mode & OZ2_ENGINE_FP8) && (mode & ~OZ2_ENGINE_FP8) == OZ2_MODE_ACCURATE)
    return OZ2_ERR_UNSUPPORTED;
  // the largest tile's padding: an upper bound for every tile the call may pick
  *bytes = (m == 0 || n == 0 || k == 0) ? 0 : make_layout(m, n, k, N, mode).total;
  return 0;
}

int ozaki2_set_workspace(void* ptr, size_t bytes) {
  if (reinterpret_cast<uintptr_t>(ptr) & 255) return -1;
  if (ptr != g_user_ws || (ptr ? bytes : 0) != g_user_ws_bytes) ++g_ws_epoch;
  g_user_ws = ptr;
  g_user_ws_bytes = ptr ? bytes : 0;
  return 0;
}

int ozaki2_set_workspace_policy(int policy) {
  if (policy != OZ2_WORKSPACE_CALLER && policy != OZ2_WORKSPACE_LIBRARY) return -1;
  g_ws_policy = policy;
  return 0;
}

int ozaki2_get_device_status(int* status) {
  int dev;
  int rc = ensure_device(&dev);
  if (rc) return rc;
  if (!status) return -1;
  *status = 0;
  if (hipStreamSynchronize(g_stream) != hipSuccess) return OZ2_ERR_HIP;
  // The status word lives at offset 0 of whichever workspace the last call
  // used; every candidate is checked and cleared.
  void* cands[3] = {g_user_ws, g_dev[dev].ws, g_dev[dev].scratch};
  for (void* p : cands) {
    if (!p) continue;
    int v = 0;
    if (hipMemcpy(&v, p, 4, hipMemcpyDeviceToHost) != hipSuccess) return OZ2_ERR_HIP;
    *status |= v;
    int z = 0;
    if (hipMemcpy(p, &z, 4, hipMemcpyHostToDevice) != hipSuccess) return OZ2_ERR_HIP;
  }
  return 0;
}

const char* ozaki2_status_string(int code) {
  if (code < 0) return "invalid argument (the negated return value is its 1-based position)";
  switch (code) {
    case OZ2_SUCCESS: return "success";
    case OZ2_ERR_K_TOO_LARGE:
      return "k exceeds the limit (2^22; 2^18 in accurate mode; 2^17 per problem of a batch)";
    case OZ2_ERR_WORKSPACE:
      return "workspace missing or too small (ozaki2_set_workspace), or its allocation failed";
    case OZ2_ERR_HIP: return "HIP runtime error";
    case OZ2_ERR_UNSUPPORTED: return "unsupported request";
    case OZ2_ERR_TOO_LARGE: return "problem size too large";
    case OZ2_ERR_SCRATCH_TOO_SMALL:
      return "ozaki2_dgemm_noalloc: the problem needs more workspace than the library's fixed "
             "device scratch (OZ2_NOALLOC_SCRATCH_BYTES)";
    default: return "unknown status";
  }
}

const char* ozaki2_version(void) {
  return "ozaki2 0.3 gfx950 kc=64 slice=39 limb=40 log2=rn32(log2_f64) "
         "tiles=256x256x128,128x128x128,256x64x128(auto) batched=128x128x128 "
         "fp8=e4m3x2digits,128x128x64,kb512";
}

int ozaki2_finalize(void) {
  (void)hipStreamSynchronize(g_stream);
  batch_release();
  if (g_batch.cap) (void)hipStreamDestroy(g_batch.cap);
  g_batch = BatchState();
  for (auto& tc : g_pending) g_free.push_back(tc);
  g_pending.clear();
  for (auto& tc : g_free)
    for (int i = 0; i <= OZ2_NUM_STAGES; ++i) (void)hipEventDestroy(tc.ev[i]);
  g_free.clear();
  for (int d = 0; d < kMaxDevices; ++d) {
    DevState& D = g_dev[d];
    if (!D.ready) continue;
    if (hipSetDevice(d) != hipSuccess) continue;
    (void)hipDeviceSynchronize();
    if (D.ws) (void)hipFree(D.ws);
    D = DevState();
  }
  return 0;
}

int ozaki2_query_constants(int N, int32_t* moduli, float* p_prime_prop, float* p_prime_fast,
                           float* delta, double* log2_P) {
  if (N < OZ2_N_MIN || N > OZ2_N_MAX) return -1;
  build_host_tables();
  if (!g_host_tables_ok[0][N]) return OZ2_ERR_UNSUPPORTED;
  const ModTable& T = g_host_tables[0][N];
  if (moduli)
    for (int t = 0; t < N; ++t) moduli[t] = (int32_t)T.p[t];
  if (p_prime_prop) *p_prime_prop = T.p_prop;
  if (p_prime_fast) *p_prime_fast = T.p_fast;
  if (delta) *delta = T.delta;
  if (log2_P) *log2_P = T.log2P;
  return 0;
}

int ozaki2_set_tile(int tile) {
  if (tile < OZ2_TILE_AUTO || tile > OZ2_TILE_256x64) return -1;
  g_tile_policy = tile;
  return 0;
}

int ozaki2_get_tile(int64_t m, int64_t n, int64_t k, int N, int* tile) {
  if (m < 0) return -1;
  if (n < 0) return -2;
  if (k < 0) return -3;
  if (N < OZ2_N_MIN || N > OZ2_N_MAX) return -4;
  if (!tile) return -5;
  *tile = tile_config(m, n, k, N);
  return 0;
}

int ozaki2_set_timing(int enable) {
  if (hipStreamSynchronize(g_stream) != hipSuccess) return OZ2_ERR_HIP;
  for (auto& tc : g_pending) g_free.push_back(tc);
  g_pending.clear();
  g_timing = enable;
  for (double& v : g_stage_ms) v = 0.0;
  g_timed_calls = 0;
  return 0;
}

int ozaki2_get_stage_times(double* ms, int* calls) {
  if (hipStreamSynchronize(g_stream) != hipSuccess) return OZ2_ERR_HIP;
  for (auto& tc : g_pending) {
    if (hipEventSynchronize(tc.ev[OZ2_NUM_STAGES]) != hipSuccess) return OZ2_ERR_HIP;
    for (int s = 0; s < OZ2_NUM_STAGES; ++s) {
      float v = 0.f;
      if (hipEventElapsedTime(&v, tc.ev[s], tc.ev[s + 1]) == hipSuccess) g_stage_ms[s] += v;
    }
    ++g_timed_calls;
    g_free.push_back(tc);
  }
  g_pending.clear();
  for (int s = 0; s < OZ2_NUM_STAGES; ++s) {
    if (ms) ms[s] = g_stage_ms[s];
    g_stage_ms[s] = 0.0;
  }
  if (calls) *calls = g_timed_calls;
  g_timed_calls = 0;
  return 0;
}

int ozaki2_debug_stages(int64_t m, int64_t n, int64_t k, const double* A, int64_t lda,
                        const double* B, int64_t ldb, int N, int mode, int t, int32_t* eA,
                        int32_t* eB, double* SA, double* SB, int8_t* RA, int8_t* RB,
                        int32_t* Ct) {
  Debug d{t, eA, eB, Ct, SA, SB, RA, RB};
  return run_gemm<double, double>(m, n, k, A, lda, B, ldb, (double*)nullptr, 1, N, mode, &d);
}

int ozaki2_debug_log2f(const float* x, float* y, int64_t n) {
  if (n < 0) return -3;
  if (n == 0) return 0;
  if (!x) return -1;
  if (!y) return -2;
  int dev;
  int rc = ensure_device(&dev);
  if (rc) return rc;
  k_log2f<<<(unsigned)((n + 255) / 256), 256, 0, g_stream>>>(x, y, n);
  if (hipGetLastError() != hipSuccess) return OZ2_ERR_HIP;
  return hipStreamSynchronize(g_stream) == hipSuccess ? 0 : OZ2_ERR_HIP;
}

}  // extern "C"
