/* Directed-rounding reference computed by the host FPU under fesetround().
 * Independent of the oracle's exact-rational rounding: each function sets the
 * IEEE 754 rounding mode and lets the hardware round one operation. */
#include <fenv.h>
#include <math.h>
#include <stdint.h>

#pragma STDC FENV_ACCESS ON

double ru_square(double a) {
  int old = fegetround(); fesetround(FE_UPWARD);
  volatile double x = a; volatile double r = x * x;
  fesetround(old); return r;
}
double ru_add(double a, double b) {
  int old = fegetround(); fesetround(FE_UPWARD);
  volatile double x = a, y = b; volatile double r = x + y;
  fesetround(old); return r;
}
float f64_to_f32(double a, int up) {
  int old = fegetround(); fesetround(up ? FE_UPWARD : FE_DOWNWARD);
  volatile double x = a; volatile float r = (float)x;
  fesetround(old); return r;
}
/* Sum of squares in chunks of kc, every square and addition rounded up. */
double ru_norm_chunked(const double* v, int64_t k, int64_t kc) {
  int old = fegetround(); fesetround(FE_UPWARD);
  volatile double total = 0.0;
  for (int64_t c = 0; c < k; c += kc) {
    volatile double part = 0.0;
    for (int64_t h = c; h < k && h < c + kc; ++h) {
      volatile double sq = v[h] * v[h];
      part = part + sq;
    }
    total = total + part;
  }
  fesetround(old); return total;
}
