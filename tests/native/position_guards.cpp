// Host check of the position helpers shared with the particle kernels: every
// coordinate, finite or not, in range or far outside, must give a node index
// inside the lattice, and ordinary positions must be unchanged.
#include <cmath>
#include <cstdio>
#include <limits>

#include "../../paper_1306_0788_amd/csrc/lbmd_internal.h"

int main() {
  const double inf = std::numeric_limits<double>::infinity(), nan = std::numeric_limits<double>::quiet_NaN();
  const double xs[] = {0.0, 0.5, 31.999999, 32.0, -1e-17, -0.5, 63.7, -40.2, 1e12, -1e12, 1e30, -1e30, 1.7e308,
                       -1.7e308, inf, -inf, nan, 5e15, -5e15};
  int bad = 0;
  for (int n : {1, 3, 32, 37, 256}) {
    for (double x : xs) {
      const double w = lbmd::wrapd(x, double(n));
      if (std::isfinite(x) && !(w >= 0.0 && w < double(n))) {
        printf("wrapd(%g, %d) = %g outside [0, n)\n", x, n, w);
        ++bad;
      }
      if (std::isnan(x) && !std::isnan(w)) {
        printf("wrapd(nan) lost the NaN\n");
        ++bad;
      }
      for (double f : {std::floor(x), std::floor(w), x}) {
        const int c = lbmd::cell_coord(f, n);
        if (c < 0 || c >= n) {
          printf("cell_coord(%g, %d) = %d\n", f, n, c);
          ++bad;
        }
      }
    }
    // positions inside the box keep their value and cell
    for (double x : {0.0, 0.25, double(n) - 0.5}) {
      if (x >= n) continue;
      if (lbmd::wrapd(x, n) != x || lbmd::cell_coord(std::floor(x), n) != int(std::floor(x))) {
        printf("ordinary position %g changed\n", x);
        ++bad;
      }
    }
    if (lbmd::wrapd(double(n) + 0.25, n) != 0.25 || lbmd::wrapd(-0.25, n) != double(n) - 0.25) {
      printf("one-period wrap changed at n = %d\n", n);
      ++bad;
    }
  }
  printf("%s\n", bad ? "FAIL" : "OK");
  return bad ? 1 : 0;
}
