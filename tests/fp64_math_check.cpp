// Host check of log1p_unit (the binary64 log(1 + y), 0 <= y <= 1, of the
// FP64 path) against a long double reference: prints the largest error in
// units in the last place over a sweep of the range, for the host's exact
// reciprocal and for reciprocal estimates off by 2^-23 relative either way
// (twice the largest error measured for the device's v_rcp_f64 estimate on
// the range the function uses).
#include "fp64_math.h"

#include <cfloat>
#include <cmath>
#include <cstdio>
#include <random>

int main() {
  double max_ulp = 0.0, worst = 0.0;
  long bad = 0;
  const double skew[3] = {0.0, std::ldexp(1.0, -23), -std::ldexp(1.0, -23)};
  auto check = [&](double y) {
    const long double ref = log1pl((long double)y);
    for (double e : skew) {
      const double got = e == 0.0 ? lingam::log1p_unit(y)
                                  : lingam::log1p_unit_with(y, [e](double x) { return (1.0 / x) * (1.0 + e); });
      if (ref == 0.0L) {
        if (got != 0.0) ++bad;
        continue;
      }
      const double ulp = std::ldexp(1.0, std::ilogb((double)ref) - 52);
      const double err = (double)fabsl((long double)got - ref) / ulp;
      if (!(err <= max_ulp)) {
        max_ulp = err;
        worst = y;
      }
    }
  };
  std::mt19937_64 g(20210928);
  std::uniform_real_distribution<double> unit(0.0, 1.0), expo(0.0, 745.0);
  for (int i = 0; i < 1000000; ++i) check(unit(g));
  for (int i = 0; i < 1000000; ++i) check(std::exp(-expo(g)));  // y = e^{-2|u|} as the kernels form it
  const double edges[] = {0.0, 1.0, 0.41421356237309503, 0.4142135623730951, 0.41421356237309515,
                          DBL_MIN, 4.9e-324, DBL_EPSILON, 0.5 * DBL_EPSILON, 1.0 - DBL_EPSILON / 2};
  for (double y : edges) check(y);
  std::printf("%.6f %.17g %ld\n", max_ulp, worst, bad);
  return 0;
}
