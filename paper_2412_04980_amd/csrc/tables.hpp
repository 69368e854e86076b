// Exact coarse-level stencil tables (host).
//
// Sec. 3.3 of the paper obtains the coarse-level Laplace and wavenumber
// stencils by Galerkin coarsening of the 5-point stencils with the
// higher-order deflation vectors (printed for the third level and, in
// Appendix A, for levels four to six).  The 2-D products separate into 1-D
// factors: Laplace_l = h^-2 (t_l (x) m_l + m_l (x) t_l), wavenumber_l = m_l (x) m_l,
// with t_1 = [-1 2 -1], m_1 = [1] and the 1-D Galerkin step
// s_{l+1}[D] = sum_{a,b} p_a p_b s_l[2D + b - a],  p = [1 4 6 4 1] / 8.
// Entries are kept as exact integers over a power of two and rounded to
// double once.
#pragma once
#include <cstdint>
#include <vector>

namespace hm {

struct Table1D {
  std::vector<__int128> num;   // centred, odd length
  int shift = 0;               // value = num / 2^shift
};

inline Table1D galerkin_step(const Table1D& s) {
  static const int p[5] = {1, 4, 6, 4, 1};   // / 8
  const int r = (int)s.num.size() / 2;
  const int rc = (r + 4) / 2;
  Table1D c;
  c.shift = s.shift + 6;
  for (int D = -rc; D <= rc; ++D) {
    __int128 acc = 0;
    for (int a = -2; a <= 2; ++a)
      for (int b = -2; b <= 2; ++b) {
        const int idx = 2 * D + b - a;
        if (idx >= -r && idx <= r) acc += (__int128)(p[a + 2] * p[b + 2]) * s.num[idx + r];
      }
    c.num.push_back(acc);
  }
  while (c.num.size() > 1 && c.num.front() == 0 && c.num.back() == 0) {
    c.num.erase(c.num.begin());
    c.num.pop_back();
  }
  return c;
}

// 2-D tables of deflation level `level` >= 2: Laplace (without the h^-2) and
// wavenumber, (2R+1)^2 row-major [b][a], R = radius.
inline void coarse_tables(int level, int* R, std::vector<double>& lap, std::vector<double>& wav) {
  Table1D t, m;
  t.num = {-1, 2, -1};
  m.num = {1};
  for (int l = 1; l < level; ++l) {
    t = galerkin_step(t);
    m = galerkin_step(m);
  }
  const int n = (int)(t.num.size() > m.num.size() ? t.num.size() : m.num.size());
  auto pad = [n](const Table1D& v) {
    std::vector<__int128> out(n, 0);
    const int off = (n - (int)v.num.size()) / 2;
    for (size_t i = 0; i < v.num.size(); ++i) out[off + i] = v.num[i];
    return out;
  };
  const std::vector<__int128> tp = pad(t), mp = pad(m);
  // both 1-D tables share the same denominator 2^(6(level-1))
  const int sh = t.shift + m.shift;
  const double den = __builtin_ldexp(1.0, sh);
  *R = n / 2;
  lap.assign(n * n, 0.0);
  wav.assign(n * n, 0.0);
  for (int b = 0; b < n; ++b)
    for (int a = 0; a < n; ++a) {
      const __int128 L = tp[a] * mp[b] + mp[a] * tp[b];
      const __int128 K = mp[a] * mp[b];
      // one rounding to double (power-of-two scaling is exact)
      lap[b * n + a] = (double)L / den;
      wav[b * n + a] = (double)K / den;
    }
}

// 1-D factors t_l, m_l of deflation level `level` (centred, length 2R+1).
inline void coarse_tables_1d(int level, int* R, std::vector<double>& t1, std::vector<double>& m1) {
  Table1D t, m;
  t.num = {-1, 2, -1};
  m.num = {1};
  for (int l = 1; l < level; ++l) {
    t = galerkin_step(t);
    m = galerkin_step(m);
  }
  const int n = (int)(t.num.size() > m.num.size() ? t.num.size() : m.num.size());
  *R = n / 2;
  t1.assign(n, 0.0);
  m1.assign(n, 0.0);
  const int ot = (n - (int)t.num.size()) / 2, om = (n - (int)m.num.size()) / 2;
  for (size_t i = 0; i < t.num.size(); ++i) t1[ot + i] = (double)t.num[i] / __builtin_ldexp(1.0, t.shift);
  for (size_t i = 0; i < m.num.size(); ++i) m1[om + i] = (double)m.num[i] / __builtin_ldexp(1.0, m.shift);
}

}  // namespace hm
