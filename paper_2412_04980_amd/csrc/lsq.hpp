// Host side of the Arnoldi least-squares problems of the (F)GMRES solvers
// (Algorithm 1): the Hessenberg columns are reduced by Givens rotations as they
// arrive, |g_{j+1}| is the residual norm of the least-squares solution after
// column j, and solve() back-substitutes the triangular system.
#pragma once
#include <cmath>
#include <complex>
#include <vector>

#include "cplx.hpp"

namespace hm {

using cd = std::complex<double>;

struct LSQ {
  int cap = 0;
  double beta = 0;
  std::vector<cd> R, cs_s, g;   // R: (cap+1) x cap column-major, rotated
  std::vector<double> cs_c;
  void init(int cap_, double beta_) {
    cap = cap_;
    beta = beta_;
    R.assign((size_t)(cap + 1) * cap, cd(0));
    cs_c.assign(cap, 0.0);
    cs_s.assign(cap, cd(0));
    g.assign(cap + 1, cd(0));
    g[0] = beta;
  }
  // column j from h[0..j+1]; returns |g_{j+1}|
  double add(int j, const c128* h) {
    cd* col = &R[(size_t)j * (cap + 1)];
    for (int i = 0; i <= j + 1; ++i) col[i] = cd(h[i].re, h[i].im);
    for (int i = 0; i < j; ++i) {
      const cd t = cs_c[i] * col[i] + cs_s[i] * col[i + 1];
      col[i + 1] = -std::conj(cs_s[i]) * col[i] + cs_c[i] * col[i + 1];
      col[i] = t;
    }
    const cd a = col[j], b = col[j + 1];
    double c;
    cd s;
    if (b == cd(0)) {
      c = 1.0; s = 0.0;
    } else if (a == cd(0)) {
      c = 0.0; s = 1.0;
    } else {
      const double aa = std::abs(a);
      const double nrm = std::hypot(aa, std::abs(b));
      c = aa / nrm;
      s = (a / aa) * std::conj(b) / nrm;
    }
    cs_c[j] = c;
    cs_s[j] = s;
    col[j] = c * a + s * b;
    col[j + 1] = 0.0;
    g[j + 1] = -std::conj(s) * g[j];
    g[j] = c * g[j];
    return std::abs(g[j + 1]);
  }
  void solve(int m, std::vector<c128>& y) const {
    std::vector<cd> yy(m);
    for (int i = m - 1; i >= 0; --i) {
      cd acc = g[i];
      for (int k = i + 1; k < m; ++k) acc -= R[(size_t)k * (cap + 1) + i] * yy[k];
      yy[i] = acc / R[(size_t)i * (cap + 1) + i];
    }
    y.resize(m);
    for (int i = 0; i < m; ++i) y[i] = mk(yy[i].real(), yy[i].imag());
  }
};

}  // namespace hm
