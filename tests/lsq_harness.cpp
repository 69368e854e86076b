// Test driver of the host least-squares code (lsq.hpp), run by
// tests/test_host_lsq.py on the CPU.  Reads "m beta" and then the m Hessenberg
// columns (column j: j+2 complex entries as re im pairs) from stdin; prints the
// residual estimate after every column and then the solution y (m entries).
#include <cstdio>
#include <vector>

#include "../paper_2412_04980_amd/csrc/lsq.hpp"

int main() {
  int m = 0;
  double beta = 0;
  if (std::scanf("%d %lf", &m, &beta) != 2 || m < 1) return 1;
  hm::LSQ lsq;
  lsq.init(m, beta);
  for (int j = 0; j < m; ++j) {
    std::vector<hm::c128> col(j + 2);
    for (auto& v : col)
      if (std::scanf("%lf %lf", &v.re, &v.im) != 2) return 1;
    std::printf("%.17g\n", lsq.add(j, col.data()));
  }
  std::vector<hm::c128> y;
  lsq.solve(m, y);
  for (const auto& v : y) std::printf("%.17g %.17g\n", v.re, v.im);
  return 0;
}
