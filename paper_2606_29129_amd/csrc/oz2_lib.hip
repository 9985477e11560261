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
#include "oz2_k4_crt.hpp"
#include "oz2_tables.hpp"

using namespace oz2;

// Constant tables for every N (index 0: fast modes, 1: accurate mode limbs).
__device__ ModTable g_tables[2][kMaxN + 1];

namespace {

constexpr int kBM = 256, kBN = 256, kBK = 128;  // K3 tile
constexpr int kMaxDevices = 64;

struct DevState {
  bool ready = false;
  ModTable* d_tables = nullptr;  // device address of g_tables
  void* ws = nullptr;            // library-owned workspace
  size_t ws_bytes = 0;
};

DevState g_dev[kMaxDevices];
hipStream_t g_stream = nullptr;
void* g_user_ws = nullptr;
size_t g_user_ws_bytes = 0;
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
};

Layout make_layout(int64_t m, int64_t n, int64_t k, int N, int mode) {
  Layout L;
  L.Mp = round_up(m > 0 ? m : 1, kBM);
  L.Np = round_up(n > 0 ? n : 1, kBN);
  L.Kp = round_up(k > 0 ? k : 1, kBK);
  L.nch = (k + kKC - 1) / kKC;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
  L.status = take(256);
  L.eA = take(4 * (size_t)L.Mp);
  L.eB = take(4 * (size_t)L.Np);
  L.SA = take(8 * (size_t)m);
  L.SB = take(8 * (size_t)n);
  L.partA = take(8 * (size_t)L.nch * m);
  L.partB = take(8 * (size_t)L.nch * n);
  const bool need_max = (mode == OZ2_MODE_ORIGINAL);
  L.maxA = need_max ? take(8 * (size_t)L.nch * m) : 0;
  L.maxB = need_max ? take(8 * (size_t)L.nch * n) : 0;
  L.RA = take((size_t)N * L.Mp * L.Kp);
  L.RB = take((size_t)N * L.Np * L.Kp);
  L.U = take((size_t)N * L.Mp * L.Np);
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
  if (mode != OZ2_MODE_REVISED && mode != OZ2_MODE_ORIGINAL && mode != OZ2_MODE_ACCURATE)
    return -11;
  if (k > OZ2_K_MAX) return OZ2_ERR_K_TOO_LARGE;
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
    D.ready = true;
  }
  *dev_out = dev;
  return 0;
}

int get_workspace(int dev, size_t bytes, char** out) {
  if (g_user_ws && g_user_ws_bytes >= bytes) {
    *out = reinterpret_cast<char*>(g_user_ws);
    return 0;
  }
  DevState& D = g_dev[dev];
  if (D.ws_bytes < bytes) {
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
  StageClock() : on(g_timing != 0) {
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

template <typename T, int LIMBS>
void launch_split(const T* A, int64_t lda, const T* B, int64_t ldb, int64_t m, int64_t n,
                  int64_t k, const Layout& L, char* ws, const ModTable* tab, int N) {
  dim3 gA((unsigned)(L.Mp / 64), (unsigned)(L.Kp / 128));
  k2_split_strided<T, LIMBS><<<gA, 256, 0, g_stream>>>(
      A, lda, m, k, (const int32_t*)(ws + L.eA), tab, N, (int8_t*)(ws + L.RA), L.Mp, L.Kp);
  int64_t work = L.Np * (L.Kp / 16);
  k2_split_contig<T, LIMBS><<<(unsigned)((work + 255) / 256), 256, 0, g_stream>>>(
      B, ldb, n, k, (const int32_t*)(ws + L.eB), tab, N, (int8_t*)(ws + L.RB), L.Np, L.Kp);
}

template <int S, typename TO>
void launch_crt(const Layout& L, char* ws, const ModTable* tab, int N, int64_t m, int64_t n,
                TO* C, int64_t ldc) {
  int64_t blocks = ((m + 31) / 32) * ((n + 31) / 32);
  k4_crt<S, TO><<<(unsigned)((blocks + 3) / 4), 256, 0, g_stream>>>(
      (const uint8_t*)(ws + L.U), (const int32_t*)(ws + L.eA), (const int32_t*)(ws + L.eB),
      tab, N, m, n, L.Mp, L.Np, C, ldc);
}

template <typename T, typename TO>
int run_gemm(int64_t m, int64_t n, int64_t k, const T* A, int64_t lda, const T* B,
             int64_t ldb, TO* C, int64_t ldc, int N, int mode, const Debug* dbg) {
  int rc = check_args(m, n, k, A, lda, B, ldb, C, ldc, N, mode, dbg == nullptr);
  if (rc) return rc;
  if (dbg && (dbg->t < 0 || dbg->t >= N)) return -10;
  if (mode == OZ2_MODE_ACCURATE) return OZ2_ERR_UNSUPPORTED;
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

  Layout L = make_layout(m, n, k, N, mode);
  char* ws = nullptr;
  if ((rc = get_workspace(dev, L.total, &ws))) return rc;

  StageClock clk;
  clk.mark(0);
  // K1: squared norms and exponents.
  k_clear_status<<<1, 64, 0, g_stream>>>((int*)(ws + L.status));
  {
    double* pmA = L.maxA ? (double*)(ws + L.maxA) : nullptr;
    double* pmB = L.maxB ? (double*)(ws + L.maxB) : nullptr;
    dim3 gA((unsigned)((m + 63) / 64), (unsigned)((L.nch + 3) / 4));
    k1_partials_strided<T><<<gA, 256, 0, g_stream>>>(A, lda, m, k, L.nch,
                                                     (double*)(ws + L.partA), pmA);
    int64_t work = n * L.nch;
    k1_partials_contig<T><<<(unsigned)((work + 255) / 256), 256, 0, g_stream>>>(
        B, ldb, n, k, L.nch, (double*)(ws + L.partB), pmB);
    k1_fold<<<(unsigned)((m + 255) / 256), 256, 0, g_stream>>>(
        (double*)(ws + L.partA), pmA, L.nch, m, mode, tab, (int32_t*)(ws + L.eA),
        (double*)(ws + L.SA), (int*)(ws + L.status));
    k1_fold<<<(unsigned)((n + 255) / 256), 256, 0, g_stream>>>(
        (double*)(ws + L.partB), pmB, L.nch, n, mode, tab, (int32_t*)(ws + L.eB),
        (double*)(ws + L.SB), (int*)(ws + L.status));
  }
  clk.mark(1);
  // K2: integers and residues.
  switch (HT.limbs) {
    case 2: launch_split<T, 2>(A, lda, B, ldb, m, n, k, L, ws, tab, N); break;
    case 3: launch_split<T, 3>(A, lda, B, ldb, m, n, k, L, ws, tab, N); break;
    default: launch_split<T, 4>(A, lda, B, ldb, m, n, k, L, ws, tab, N); break;
  }
  clk.mark(2);
  // K3: N INT8 GEMMs.
  const int tiles = (int)((L.Mp / kBM) * (L.Np / kBN));
  if (dbg) {
    if (dbg->Ct)
      k3_gemm_i8<kBM, kBN, kBK, true><<<(unsigned)tiles, 256, 0, g_stream>>>(
          (const int8_t*)(ws + L.RA), (const int8_t*)(ws + L.RB), nullptr, dbg->Ct, m, n, L.Mp,
          L.Np, L.Kp, tab, dbg->t);
  } else {
    k3_gemm_i8<kBM, kBN, kBK, false><<<(unsigned)(tiles * N), 256, 0, g_stream>>>(
        (const int8_t*)(ws + L.RA), (const int8_t*)(ws + L.RB), (uint8_t*)(ws + L.U), nullptr,
        m, n, L.Mp, L.Np, L.Kp, tab, 0);
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

}  // namespace

extern "C" {

int ozaki2_dgemm(int64_t m, int64_t n, int64_t k, const double* A, int64_t lda,
                 const double* B, int64_t ldb, double* C, int64_t ldc, int N, int mode) {
  return run_gemm<double, double>(m, n, k, A, lda, B, ldb, C, ldc, N, mode, nullptr);
}

int ozaki2_sgemm(int64_t m, int64_t n, int64_t k, const float* A, int64_t lda,
                 const float* B, int64_t ldb, float* C, int64_t ldc, int N, int mode) {
  return run_gemm<float, float>(m, n, k, A, lda, B, ldb, C, ldc, N, mode, nullptr);
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
  *bytes = (m == 0 || n == 0 || k == 0) ? 0 : make_layout(m, n, k, N, mode).total;
  return 0;
}

int ozaki2_set_workspace(void* ptr, size_t bytes) {
  if (reinterpret_cast<uintptr_t>(ptr) & 255) return -1;
  g_user_ws = ptr;
  g_user_ws_bytes = ptr ? bytes : 0;
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
  // used; both candidates are checked and cleared.
  void* cands[2] = {g_user_ws, g_dev[dev].ws};
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
    case OZ2_ERR_K_TOO_LARGE: return "k exceeds 2^17 (INT32 accumulation limit)";
    case OZ2_ERR_WORKSPACE: return "workspace allocation failed";
    case OZ2_ERR_HIP: return "HIP runtime error";
    case OZ2_ERR_UNSUPPORTED: return "unsupported request";
    case OZ2_ERR_TOO_LARGE: return "problem size too large";
    default: return "unknown status";
  }
}

const char* ozaki2_version(void) {
  return "ozaki2 0.1 gfx950 kc=64 slice=39 limb=26 log2=rn32(log2_f64) tile=256x256x128";
}

int ozaki2_finalize(void) {
  (void)hipStreamSynchronize(g_stream);
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
