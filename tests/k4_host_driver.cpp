// Host build of K4's per-entry arithmetic (test infrastructure): reads cases
// "N E U_0 ... U_{N-1}" (residues of C'' as K3 writes them) from stdin, forms
// the slice sums sum_t w_ts U_t from the library's Step 1 table as K4 does,
// and prints the binary64 and binary32 results of crt_unscale as bit
// patterns (hex), one case per line.
#include <cstdio>
#include <cstdint>

#include "oz2_k4_crt.hpp"

using namespace oz2;

template <int S>
static void one(const ModTable& T, int E, const int* U) {
  double acc[S];
  for (int s = 0; s < S; ++s) acc[s] = 0.0;
  for (int t = 0; t < T.N; ++t)
    for (int s = 0; s < S; ++s) acc[s] = fma(T.w[t][s], (double)U[t], acc[s]);
  const double d = crt_unscale<S, 53, -1074>(acc, T, E);
  const float f = (float)crt_unscale<S, 24, -149>(acc, T, E);
  printf("%016llx %08x\n", (unsigned long long)f64_to_bits(d), (unsigned)f32_to_bits(f));
}

int main() {
  static ModTable tabs[kMaxN + 1];
  static bool built[kMaxN + 1];
  int N, E;
  while (scanf("%d %d", &N, &E) == 2) {
    if (N < 2 || N > kMaxN) return 2;
    if (!built[N]) {
      if (!build_table(N, false, &tabs[N])) return 3;
      built[N] = true;
    }
    int U[kMaxN];
    for (int t = 0; t < N; ++t)
      if (scanf("%d", &U[t]) != 1) return 4;
    const ModTable& T = tabs[N];
    switch (T.slices) {
      case 1: one<1>(T, E, U); break;
      case 2: one<2>(T, E, U); break;
      case 3: one<3>(T, E, U); break;
      default: one<4>(T, E, U); break;
    }
  }
  return 0;
}
