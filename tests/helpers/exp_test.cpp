// Host harness for vegas::exp_f64: prints x and exp_f64(x) for x read from stdin.
#include <cstdio>

#include "vegas_math.hpp"

int main() {
  double x;
  while (std::scanf("%lf", &x) == 1) std::printf("%.17g %.17g\n", x, vegas::exp_f64(x));
  return 0;
}
