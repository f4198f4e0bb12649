// Host harness for the binary64 functions of vegas_math.hpp: reads lines
// "e x", "l x", "p x a", "s u" or "c u" from stdin and prints exp_f64(x),
// log_f64(x), pow_pos(x, a), or the sine or cosine of sincos_turns_f64(u)
// with 17 significant digits.
#include <cstdio>

#include "vegas_math.hpp"

int main() {
  char op;
  double x, a;
  while (std::scanf(" %c %lf", &op, &x) == 2) {
    double y = 0.0;
    if (op == 'e') {
      y = vegas::exp_f64(x);
    } else if (op == 'l') {
      y = vegas::log_f64(x);
    } else if (op == 'p' && std::scanf("%lf", &a) == 1) {
      y = vegas::pow_pos(x, a);
    } else if (op == 's' || op == 'c') {
      double sn, cs;
      vegas::sincos_turns_f64(x, &sn, &cs);
      y = op == 's' ? sn : cs;
    } else {
      return 1;
    }
    std::printf("%.17g\n", y);
  }
  return 0;
}
