// Host check of the in-register DFTs of fft_lds.h against the DFT's
// definition.  dft_tw<R, N, SIGN>(x, u) must give
//   y[f] = sum_r x[r] (u exp(SIGN 2 pi i f / N))^r,
// the input twiddles u^r of a Stockham stage folded into the transform, and
// dft<R, N, SIGN>(x) the same with u = 1.  The reference sums run in long
// double from the same rounded inputs (u's modulus, one up to rounding, is
// kept as it is).  Prints "ok" when every case is within its bound.
#include "fft_lds.h"

#include <cmath>
#include <cstdio>
#include <random>

using namespace pc;

template <typename R, int N, int SIGN, bool TW>
static bool check(std::mt19937_64& g, double bound) {
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  double worst = 0.0;
  for (int trial = 0; trial < 500; ++trial) {
    const double ang = U(g) * M_PI;
    const cpx<R> u = TW ? cpx<R>{(R)std::cos(ang), (R)std::sin(ang)} : cpx<R>{R(1), R(0)};
    cpx<R> x[N];
    long double xr[N], xi[N];
    for (int r = 0; r < N; ++r) {
      x[r] = {(R)U(g), (R)U(g)};
      xr[r] = x[r].x;
      xi[r] = x[r].y;
    }
    if (TW)
      dft_tw<R, N, SIGN>(x, u);
    else
      dft<R, N, SIGN>(x);
    const long double mod = std::hypot((long double)u.x, (long double)u.y);
    const long double arg = std::atan2((long double)u.y, (long double)u.x);
    double err = 0.0, mag = 0.0;
    for (int f = 0; f < N; ++f) {
      long double yr = 0.0L, yi = 0.0L;
      for (int r = 0; r < N; ++r) {
        const long double a = r * (arg + SIGN * 2.0L * (long double)M_PI * f / N);
        const long double m = std::pow(mod, (long double)r);
        yr += m * (xr[r] * std::cos(a) - xi[r] * std::sin(a));
        yi += m * (xr[r] * std::sin(a) + xi[r] * std::cos(a));
      }
      err = std::max(err, (double)std::hypot(yr - x[f].x, yi - x[f].y));
      mag = std::max(mag, (double)std::hypot(yr, yi));
    }
    worst = std::max(worst, err / mag);
  }
  const bool ok = worst <= bound;
  std::printf("%s N=%d sign=%+d %s: max error / max output %.3g (bound %.1g)%s\n",
              sizeof(R) == 4 ? "f32" : "f64", N, SIGN, TW ? "twiddled" : "plain", worst, bound,
              ok ? "" : "  FAIL");
  return ok;
}

template <typename R, int SIGN>
static bool all_sizes(std::mt19937_64& g, double bound) {
  bool ok = true;
  ok &= check<R, 2, SIGN, true>(g, bound);
  ok &= check<R, 4, SIGN, true>(g, bound);
  ok &= check<R, 8, SIGN, true>(g, bound);
  ok &= check<R, 16, SIGN, true>(g, bound);
  ok &= check<R, 4, SIGN, false>(g, bound);
  ok &= check<R, 16, SIGN, false>(g, bound);
  return ok;
}

int main() {
  std::mt19937_64 g(20240601);
  bool ok = true;
  ok &= all_sizes<double, +1>(g, 1e-13);
  ok &= all_sizes<double, -1>(g, 1e-13);
  ok &= all_sizes<float, +1>(g, 2e-6);
  ok &= all_sizes<float, -1>(g, 2e-6);
  std::printf(ok ? "ok\n" : "FAILED\n");
  return ok ? 0 : 1;
}
