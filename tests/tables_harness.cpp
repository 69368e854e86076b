// Test driver of the host stencil tables (tables.hpp), run by
// tests/test_host_tables.py on the CPU.  For each deflation level 2..6 prints
// "level R", then the (2R+1)^2 Laplace and wavenumber tables (row-major [b][a])
// and the 1-D factors t and m (2R+1 each), one value per line, %.17g.
#include <cstdio>
#include <vector>

#include "../paper_2412_04980_amd/csrc/tables.hpp"

int main() {
  for (int level = 2; level <= 6; ++level) {
    int R = 0, R1 = 0;
    std::vector<double> lap, wav, t1, m1;
    hm::coarse_tables(level, &R, lap, wav);
    hm::coarse_tables_1d(level, &R1, t1, m1);
    if (R1 != R) return 1;
    std::printf("%d %d\n", level, R);
    for (double v : lap) std::printf("%.17g\n", v);
    for (double v : wav) std::printf("%.17g\n", v);
    for (double v : t1) std::printf("%.17g\n", v);
    for (double v : m1) std::printf("%.17g\n", v);
  }
  return 0;
}
