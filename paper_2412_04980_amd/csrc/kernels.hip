// HIP kernels of the MADP library for gfx950 (wave64).
//
// Stencils (Sec. 2.1 and Sec. 3.3 of the paper), deflation transfers Z^T / Z
// (higher-order deflation vectors), multigrid transfers for the CSLP V-cycle,
// vector updates and reductions of the Krylov methods (Algorithm 1).
// All grid arrays are row-major with x fastest; complex values interleaved.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <type_traits>

#include "kernels.hpp"

#include <mutex>
#include <vector>

// Reduction partials of the entry points that take no workspace
// (hm_residual_noalloc): one copy per device, held until the process ends.
// Host code never passes this name to a kernel (on the host it is only a
// stand-in); it uses the device address from hipGetSymbolAddress.
static __device__ __align__(256) hm::c128 scratch[hm::kMaxChunks];

namespace hm {

namespace {

constexpr int BX = 64;   // one wavefront along x
constexpr int BY = 4;    // four wavefronts per block
constexpr int NT = 256;

inline dim3 grid2d(int nx, int ny) { return dim3((nx + BX - 1) / BX, (ny + BY - 1) / BY); }
inline unsigned blocks1d(size_t n) {
  size_t b = (n + NT - 1) / NT;
  return (unsigned)(b > 0 ? b : 1);
}

// Grid of a batched launch: the members are the z dimension.
inline dim3 zgrid(unsigned x, const Batch& z) { return dim3(x, 1, (unsigned)z.n); }
inline dim3 zgrid(dim3 g, const Batch& z) { return dim3(g.x, g.y, (unsigned)z.n); }

// The member a block works on: block z takes member slot[z], whose buffers lie
// slot * stride bytes after member 0's (dz on the device, hz in pinned host
// memory).  Null pointers (absent operands) stay null.
// The offset is applied as byte-pointer arithmetic on the argument itself (no
// integer round trip), so the compiler still sees a global, non-aliasing
// pointer: global (not flat) memory instructions and scalar loads of uniform data.
template <typename P>
__device__ __forceinline__ P* at_member(P* p, long long stride, const Batch& z) {
  using C = typename std::conditional<std::is_const<P>::value, const char, char>::type;
  const long long off = (long long)z.slot[blockIdx.z] * stride;
  return p ? reinterpret_cast<P*>(reinterpret_cast<C*>(p) + off) : p;
}
#define HM_MEMBER(ptr) ptr = at_member(ptr, z.dz, z)

// Ghost-extended value at grid position (x, y), which may lie outside:
// inside -> u, k^2;  one step out in exactly one direction -> Sommerfeld ghost
// u_m + i (2H) k_b u_b with k^2 = 0;  otherwise 0.
// Dirichlet (d.bc == 1): boundary nodes read as zero; one step outside in
// exactly one direction -> ghost 2 u_b - u_m = -u_m with wavenumber 2 k_b - k_m
// (zero when the mirror u_m is itself a boundary node); otherwise 0.
template <typename T>
__device__ __forceinline__ void ext_val_dirichlet(const OpDesc<T>& d, const cx<T>* __restrict__ u,
                                                  const T* __restrict__ k, int x, int y, cx<T>& uv,
                                                  T& k2) {
  const int nx = d.nx, ny = d.ny;
  const bool xin = (unsigned)x < (unsigned)nx;
  const bool yin = (unsigned)y < (unsigned)ny;
  uv = mk(T(0), T(0));
  k2 = T(0);
  if (xin && yin) {
    const size_t p = (size_t)y * nx + x;
    const T kk = k[p];
    k2 = kk * kk;
    if (x > 0 && y > 0 && x < nx - 1 && y < ny - 1) uv = u[p];
    return;
  }
  if (yin && (x == -1 || x == nx)) {
    const int xb = x < 0 ? 0 : nx - 1;
    const int xm = x < 0 ? 1 : nx - 2;
    const size_t row = (size_t)y * nx;
    const T kg = T(2) * k[row + xb] - k[row + xm];
    k2 = kg * kg;
    if (y > 0 && y < ny - 1) {
      const cx<T> um = u[row + xm];
      uv = mk(-um.re, -um.im);
    }
    return;
  }
  if (xin && (y == -1 || y == ny)) {
    const int yb = y < 0 ? 0 : ny - 1;
    const int ym = y < 0 ? 1 : ny - 2;
    const T kg = T(2) * k[(size_t)yb * nx + x] - k[(size_t)ym * nx + x];
    k2 = kg * kg;
    if (x > 0 && x < nx - 1) {
      const cx<T> um = u[(size_t)ym * nx + x];
      uv = mk(-um.re, -um.im);
    }
  }
}

template <typename T>
__device__ __forceinline__ void ext_val(const OpDesc<T>& d, const cx<T>* __restrict__ u,
                                        const T* __restrict__ k, int x, int y, cx<T>& uv, T& k2) {
  if (d.bc) {
    ext_val_dirichlet(d, u, k, x, y, uv, k2);
    return;
  }
  const int nx = d.nx, ny = d.ny;
  const bool xin = (unsigned)x < (unsigned)nx;
  const bool yin = (unsigned)y < (unsigned)ny;
  if (xin && yin) {
    const size_t p = (size_t)y * nx + x;
    uv = u[p];
    const T kk = k[p];
    k2 = kk * kk;
    return;
  }
  k2 = T(0);
  if (yin && (x == -1 || x == nx)) {
    const int xb = x < 0 ? 0 : nx - 1;
    const int xm = x < 0 ? 1 : nx - 2;
    const size_t row = (size_t)y * nx;
    const cx<T> ub = u[row + xb], um = u[row + xm];
    const T c = d.two_H * k[row + xb];
    uv = mk(um.re - c * ub.im, um.im + c * ub.re);
    return;
  }
  if (xin && (y == -1 || y == ny)) {
    const int yb = y < 0 ? 0 : ny - 1;
    const int ym = y < 0 ? 1 : ny - 2;
    const cx<T> ub = u[(size_t)yb * nx + x], um = u[(size_t)ym * nx + x];
    const T c = d.two_H * k[(size_t)yb * nx + x];
    uv = mk(um.re - c * ub.im, um.im + c * ub.re);
    return;
  }
  uv = mk(T(0), T(0));
}

// Five-point row at (x, y): scale*(inv_H2 (4u - sum nbrs) - sigma k^2 u).
template <typename T>
__device__ __forceinline__ cx<T> five_point_row(const OpDesc<T>& d, const cx<T>* __restrict__ u,
                                                const T* __restrict__ k, int x, int y) {
  cx<T> uc, un;
  T k2, kd;
  ext_val(d, u, k, x, y, uc, k2);
  cx<T> s = mk(T(4) * uc.re, T(4) * uc.im);
  ext_val(d, u, k, x - 1, y, un, kd); s = s - un;
  ext_val(d, u, k, x + 1, y, un, kd); s = s - un;
  ext_val(d, u, k, x, y - 1, un, kd); s = s - un;
  ext_val(d, u, k, x, y + 1, un, kd); s = s - un;
  // sigma k^2 u
  const cx<T> sk = mk(d.sig_re * k2, d.sig_im * k2) * uc;
  return d.scale * (d.inv_H2 * s - sk);
}

template <typename T>
__device__ __forceinline__ cx<T> five_point_diag(const OpDesc<T>& d, const T* __restrict__ k, int x,
                                                 int y) {
  const T kk = k[(size_t)y * d.nx + x];
  const T k2 = kk * kk;
  const int nout = (x == 0) + (x == d.nx - 1) + (y == 0) + (y == d.ny - 1);
  if (d.bc && nout) return mk(d.scale * T(4) * d.inv_H2, T(0));   // Dirichlet boundary row
  // scale*(4/H^2 - sigma k^2) - i scale/H^2 * 2H k * nout
  return mk(d.scale * (T(4) * d.inv_H2 - d.sig_re * k2),
            d.scale * (-d.sig_im * k2 - d.inv_H2 * d.two_H * kk * T(nout)));
}

template <typename T, int R>
__device__ __forceinline__ cx<T> wide_diag(const OpDesc<T>& d, const T* __restrict__ k, int x, int y) {
  constexpr int W = 2 * R + 1;
  const T kk = k[(size_t)y * d.nx + x];
  const T k2 = kk * kk;
  // centre entry plus the ghost reflections that land on the node itself:
  // offset +-2 along x at x == 1 / nx-2 and along y at y == 1 / ny-2
  const T lx2 = d.L[R * W + (R + 2)];
  const T ly2 = d.L[(R + 2) * W + R];
  T re = d.L[R * W + R] - d.sig_re * d.K[R * W + R] * k2;
  T im = -d.sig_im * d.K[R * W + R] * k2;
  if (d.bc) {
    // Dirichlet ghost -u_m with wavenumber k_g = 2 k_b - k_m: the tap lands on
    // the node with coefficient -(L - sigma K k_g^2)
    const T kx2 = d.K[R * W + (R + 2)], ky2 = d.K[(R + 2) * W + R];
    const size_t row = (size_t)y * d.nx;
    auto refl = [&](T lc, T kc, T kb, T km) {
      const T kg = T(2) * kb - km;
      re -= lc - d.sig_re * kc * kg * kg;
      im += d.sig_im * kc * kg * kg;
    };
    if (x == 1) refl(lx2, kx2, k[row], k[row + 1]);
    if (x == d.nx - 2) refl(lx2, kx2, k[row + d.nx - 1], k[row + d.nx - 2]);
    if (y == 1) refl(ly2, ky2, k[x], k[(size_t)d.nx + x]);
    if (y == d.ny - 2)
      refl(ly2, ky2, k[(size_t)(d.ny - 1) * d.nx + x], k[(size_t)(d.ny - 2) * d.nx + x]);
    return mk(re, im);
  }
  re += lx2 * T((x == 1) + (x == d.nx - 2)) + ly2 * T((y == 1) + (y == d.ny - 2));
  return mk(re, im);
}

// XCD-aware order of tiles for a 1-D grid of 8 * ceil(tiles / 8) blocks.
// Blocks are dispatched round-robin over the 8 XCDs (block b on XCD b % 8);
// XCD j takes the j-th contiguous range of tiles in row-major order, so the
// tiles above and below a tile run on the same XCD close in time and the halo
// rows they share are read from that XCD's L2 rather than again from HBM.
__device__ __forceinline__ bool xcd_tile(int ntx, int nty, int& tx, int& ty) {
  const int nt = ntx * nty;
  const int per = (nt + 7) / 8;
  const int tile = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (tile >= nt) return false;
  ty = tile / ntx;
  tx = tile - ty * ntx;
  return true;
}

template <typename T, int R>
__device__ __forceinline__ bool is_boundary(const OpDesc<T>& d, int x, int y) {
  return x == 0 || y == 0 || x == d.nx - 1 || y == d.ny - 1;
}

constexpr int ST_SCALED = 3;   // out = Op(s u), vout = s u, s = 1 / scal[0].re

// Output of one 5-point row for the stencil modes (Dirichlet boundary rows
// are d_b u_b; everything else goes through the ghost-extended values).
template <typename T, int MODE>
__device__ __forceinline__ void five_point_emit(const OpDesc<T>& d, const cx<T>* __restrict__ u,
                                                const T* __restrict__ k,
                                                const cx<T>* __restrict__ b,
                                                cx<T>* __restrict__ out, T omega, T sc,
                                                cx<T>* __restrict__ vout, int x, int y, cx<T> au) {
  const size_t p = (size_t)y * d.nx + x;
  if constexpr (MODE == ST_APPLY) {
    out[p] = au;
  } else if constexpr (MODE == ST_SCALED) {
    out[p] = sc * au;
    vout[p] = sc * u[p];
  } else if constexpr (MODE == ST_RESID) {
    out[p] = b[p] - au;
  } else {
    const cx<T> r = b[p] - au;
    out[p] = u[p] + omega * cdiv(r, five_point_diag(d, k, x, y));
  }
}

template <typename T>
__device__ __forceinline__ cx<T> five_point_any(const OpDesc<T>& d, const cx<T>* __restrict__ u,
                                                const T* __restrict__ k, int x, int y) {
  if (d.bc && (x == 0 || y == 0 || x == d.nx - 1 || y == d.ny - 1))
    return (d.scale * T(4) * d.inv_H2) * u[(size_t)y * d.nx + x];   // Dirichlet d_b u_b
  return five_point_row(d, u, k, x, y);
}

// 5-point operator in all stencil modes.  Block = 64 x 4 threads, tile = 64 x 8
// nodes in the XCD-aware order; each thread takes two vertically adjacent nodes,
// which share their middle neighbours (four vertical loads for two outputs) and
// give every thread twice the independent loads in flight.  Nodes whose
// neighbours are all plain grid values take the direct path; the others (the
// boundary band) go through the ghost-extended values.
constexpr int FP_ROWS = 2;

template <typename T, int MODE>
__global__ void __launch_bounds__(NT) k_five_point(OpDesc<T> d, const cx<T>* __restrict__ u,
                                                   const T* __restrict__ k,
                                                   const cx<T>* __restrict__ b,
                                                   cx<T>* __restrict__ out, T omega,
                                                   const c128* __restrict__ scal,
                                                   cx<T>* __restrict__ vout, Batch z) {
  int tx, ty;
  if (!xcd_tile((d.nx + BX - 1) / BX, (d.ny + BY * FP_ROWS - 1) / (BY * FP_ROWS), tx, ty)) return;
  HM_MEMBER(u); HM_MEMBER(k); HM_MEMBER(b); HM_MEMBER(out); HM_MEMBER(scal); HM_MEMBER(vout);
  if (z.use_omega) omega = (T)z.omega[blockIdx.z];
  const int nx = d.nx, ny = d.ny;
  const int x = tx * BX + threadIdx.x;
  const int y = ty * BY * FP_ROWS + threadIdx.y * FP_ROWS;
  if (x >= nx || y >= ny) return;
  T sc = T(1);
  if constexpr (MODE == ST_SCALED) sc = (T)(1.0 / scal[0].re);
  const int e = d.bc ? 2 : 1;        // Dirichlet: neighbours on the boundary read as zero
  if (x >= e && x <= nx - 1 - e && y >= e && y + 1 <= ny - 1 - e) {
    const size_t p0 = (size_t)y * nx + x, p1 = p0 + nx;
    const cx<T> us = u[p0 - nx], u0 = u[p0], u1 = u[p1], un = u[p1 + nx];
    const cx<T> w0 = u[p0 - 1], e0 = u[p0 + 1], w1 = u[p1 - 1], e1 = u[p1 + 1];
    const T k0 = k[p0], k1 = k[p1];
    cx<T> s0 = mk(T(4) * u0.re, T(4) * u0.im);
    s0 = s0 - w0; s0 = s0 - e0; s0 = s0 - us; s0 = s0 - u1;
    cx<T> s1 = mk(T(4) * u1.re, T(4) * u1.im);
    s1 = s1 - w1; s1 = s1 - e1; s1 = s1 - u0; s1 = s1 - un;
    const T q0 = k0 * k0, q1 = k1 * k1;
    const cx<T> a0 = d.scale * (d.inv_H2 * s0 - mk(d.sig_re * q0, d.sig_im * q0) * u0);
    const cx<T> a1 = d.scale * (d.inv_H2 * s1 - mk(d.sig_re * q1, d.sig_im * q1) * u1);
    five_point_emit<T, MODE>(d, u, k, b, out, omega, sc, vout, x, y, a0);
    five_point_emit<T, MODE>(d, u, k, b, out, omega, sc, vout, x, y + 1, a1);
    return;
  }
#pragma unroll
  for (int r = 0; r < FP_ROWS; ++r) {
    if (y + r >= ny) break;
    five_point_emit<T, MODE>(d, u, k, b, out, omega, sc, vout, x, y + r,
                             five_point_any(d, u, k, x, y + r));
  }
}

inline unsigned five_point_blocks(int nx, int ny) {
  const size_t nt = (size_t)((nx + BX - 1) / BX) * ((ny + BY * FP_ROWS - 1) / (BY * FP_ROWS));
  return (unsigned)(8 * ((nt + 7) / 8));
}

// Wide (5x5 / 7x7) stencil with the ghost-extended input tile staged in LDS.
// Block = 64 x 4 threads, tile = 64 x 8 outputs; each thread produces WT_R = 2
// vertically adjacent outputs and keeps one stencil row in registers while it
// is reused by the outputs that need it (fewer LDS reads per output).
constexpr int WT_X = 64;
constexpr int WT_R = 2;
constexpr int WT_Y = BY * WT_R;

template <typename T, int R, int MODE>
__global__ void __launch_bounds__(NT) k_wide_tiled(OpDesc<T> d, const cx<T>* __restrict__ u,
                                                   const T* __restrict__ k,
                                                   const cx<T>* __restrict__ b,
                                                   cx<T>* __restrict__ out, T omega,
                                                   const c128* __restrict__ scal,
                                                   cx<T>* __restrict__ vout, Batch z) {
  constexpr int W = 2 * R + 1;
  constexpr int SX = WT_X + 2 * R;
  constexpr int SY = WT_Y + 2 * R;
  __shared__ cx<T> su[SY][SX];
  __shared__ T sk[SY][SX];
  // XCD-aware tile order: the 8 XCDs (round-robin dispatch) each take one
  // contiguous range of tiles in row-major order, so the tile above a tile ran
  // shortly before on the same XCD and its halo rows are still in that L2
  const int ntx = (d.nx + WT_X - 1) / WT_X, nty = (d.ny + WT_Y - 1) / WT_Y;
  const int per = (ntx * nty + 7) / 8;
  const int tile = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (tile >= ntx * nty) return;
  HM_MEMBER(u); HM_MEMBER(k); HM_MEMBER(b); HM_MEMBER(out); HM_MEMBER(scal); HM_MEMBER(vout);
  if (z.use_omega) omega = (T)z.omega[blockIdx.z];
  const int x0 = (tile % ntx) * WT_X, y0 = (tile / ntx) * WT_Y;
  const int tid = threadIdx.y * BX + threadIdx.x;
  T sc = T(1);
  if constexpr (MODE == ST_SCALED) sc = (T)(1.0 / scal[0].re);
  for (int idx = tid; idx < SX * SY; idx += NT) {
    const int r = idx / SX, c = idx - r * SX;
    cx<T> uv;
    T k2;
    ext_val(d, u, k, x0 - R + c, y0 - R + r, uv, k2);
    // the ghost values are linear in u, so scaling the extended tile scales u
    if constexpr (MODE == ST_SCALED) uv = sc * uv;
    su[r][c] = uv;
    sk[r][c] = k2;
  }
  __syncthreads();
  const int tx = threadIdx.x;
  const int x = x0 + tx;
  const int ly0 = threadIdx.y * WT_R;          // local row of this thread's first output
  // separable evaluation on the extended tile:
  //   L u = sum_b m_b (t * u)_row + t_b (m * u)_row,  K (k^2 u) = sum_b m_b (m * k^2 u)_row
  T lre[WT_R], lim[WT_R], kre[WT_R], kim[WT_R];
#pragma unroll
  for (int o = 0; o < WT_R; ++o) { lre[o] = lim[o] = kre[o] = kim[o] = T(0); }
  // vertical weights without run-time indexing: a queue of m1/t1 shifted one
  // row per pass and, per output o, the weights m1[rr - o], t1[rr - o] of the
  // current pass (zero outside the stencil).  An index into the kernel
  // arguments inside the loop made scalar loads whose waits also drained the
  // tile's LDS reads.
  T qm[W], qt[W], mo[WT_R], to[WT_R];
#pragma unroll
  for (int a = 0; a < W; ++a) { qm[a] = d.m1[a]; qt[a] = d.t1[a]; }
#pragma unroll
  for (int o = 0; o < WT_R; ++o) { mo[o] = T(0); to[o] = T(0); }
#pragma unroll 1
  for (int rr = 0; rr < WT_R + 2 * R; ++rr) {
    // this pass's weights: output o takes m1[rr - o]
#pragma unroll
    for (int o = WT_R - 1; o > 0; --o) { mo[o] = mo[o - 1]; to[o] = to[o - 1]; }
    mo[0] = qm[0];
    to[0] = qt[0];
#pragma unroll
    for (int a = 0; a + 1 < W; ++a) { qm[a] = qm[a + 1]; qt[a] = qt[a + 1]; }
    qm[W - 1] = T(0);
    qt[W - 1] = T(0);
    T tur = 0, tui = 0, mur = 0, mui = 0, mwr = 0, mwi = 0;
#pragma unroll
    for (int a = 0; a < W; ++a) {
      const cx<T> uv = su[ly0 + rr][tx + a];
      const T k2 = sk[ly0 + rr][tx + a];
      const T ta = d.t1[a], ma = d.m1[a];
      tur += ta * uv.re; tui += ta * uv.im;
      mur += ma * uv.re; mui += ma * uv.im;
      const T mk2 = ma * k2;
      mwr += mk2 * uv.re; mwi += mk2 * uv.im;
    }
#pragma unroll
    for (int o = 0; o < WT_R; ++o) {           // tap row (b + R) = rr - o
      lre[o] += mo[o] * tur + to[o] * mur;
      lim[o] += mo[o] * tui + to[o] * mui;
      kre[o] += mo[o] * mwr;
      kim[o] += mo[o] * mwi;
    }
  }
  T are[WT_R], aim[WT_R];
#pragma unroll
  for (int o = 0; o < WT_R; ++o) {
    // L u - sigma K w
    are[o] = lre[o] - (d.sig_re * kre[o] - d.sig_im * kim[o]);
    aim[o] = lim[o] - (d.sig_re * kim[o] + d.sig_im * kre[o]);
  }
  if (x >= d.nx) return;
#pragma unroll
  for (int o = 0; o < WT_R; ++o) {
    const int y = y0 + ly0 + o;
    if (y >= d.ny) break;
    const size_t p = (size_t)y * d.nx + x;
    const int cy = ly0 + o + R, cxl = tx + R;
    cx<T> uc = su[cy][cxl];
    cx<T> au;
    const bool bnd = x == 0 || y == 0 || x == d.nx - 1 || y == d.ny - 1;
    if (bnd && d.bc) {
      // Dirichlet boundary row d_b u_b; the tile holds zero there, so read u
      uc = u[p];
      if constexpr (MODE == ST_SCALED) uc = sc * uc;
      au = (d.scale * T(4) * d.inv_H2) * uc;
    } else if (bnd) {
      const T k2 = sk[cy][cxl];
      cx<T> s = mk(T(4) * uc.re, T(4) * uc.im);
      s = s - su[cy][cxl - 1];
      s = s - su[cy][cxl + 1];
      s = s - su[cy - 1][cxl];
      s = s - su[cy + 1][cxl];
      const cx<T> sk2 = mk(d.sig_re * k2, d.sig_im * k2) * uc;
      au = d.scale * (d.inv_H2 * s - sk2);
    } else {
      au = mk(are[o], aim[o]);
    }
    if constexpr (MODE == ST_APPLY) {
      out[p] = au;
    } else if constexpr (MODE == ST_SCALED) {
      out[p] = au;
      vout[p] = uc;
    } else if constexpr (MODE == ST_RESID) {
      out[p] = b[p] - au;
    } else {
      const cx<T> dg = bnd ? five_point_diag(d, k, x, y) : wide_diag<T, R>(d, k, x, y);
      out[p] = uc + omega * cdiv(b[p] - au, dg);
    }
  }
}

// Persistent form of the wide stencil for Sommerfeld boundaries.  A grid of
// resident blocks walks the tiles (each XCD a contiguous range of them, as in
// k_wide_tiled), and each block loads the next tile's grid values into
// registers while it evaluates the current tile from LDS: the halo loads
// overlap the arithmetic, and no partial second round of blocks is left at
// the end.  Tile values are read at clamped positions, so a point one step
// outside the grid in exactly one direction holds its boundary node's u_b and
// k_b; its Sommerfeld ghost u_m + i 2H k_b u_b is completed once the mirror
// u_m is in LDS.  The arithmetic of an output is that of k_wide_tiled.
template <typename T, int R, int MODE>
__global__ void __launch_bounds__(NT) k_wide_persist(OpDesc<T> d, const cx<T>* __restrict__ u,
                                                     const T* __restrict__ k,
                                                     const cx<T>* __restrict__ b,
                                                     cx<T>* __restrict__ out, T omega,
                                                     const c128* __restrict__ scal,
                                                     cx<T>* __restrict__ vout, Batch z) {
  constexpr int W = 2 * R + 1;
  constexpr int SX = WT_X + 2 * R;
  constexpr int SY = WT_Y + 2 * R;
  constexpr int NP = SX * SY;
  constexpr int PTS = (NP + NT - 1) / NT;      // tile points per thread
  __shared__ cx<T> su[SY][SX];
  __shared__ T sk[SY][SX];
  HM_MEMBER(u); HM_MEMBER(k); HM_MEMBER(b); HM_MEMBER(out); HM_MEMBER(scal); HM_MEMBER(vout);
  if (z.use_omega) omega = (T)z.omega[blockIdx.z];
  const int nx = d.nx, ny = d.ny;
  const int ntx = (nx + WT_X - 1) / WT_X, nty = (ny + WT_Y - 1) / WT_Y;
  const int nt = ntx * nty;
  const int per = (nt + 7) / 8;
  const int nloc = (int)(gridDim.x >> 3);      // blocks per XCD
  const int t_lo = (int)(blockIdx.x & 7) * per;
  const int t_hi = min(t_lo + per, nt);
  int tile = t_lo + (int)(blockIdx.x >> 3);
  if (tile >= t_hi) return;
  const int tid = threadIdx.y * BX + threadIdx.x;
  T sc = T(1);
  if constexpr (MODE == ST_SCALED) sc = (T)(1.0 / scal[0].re);
  cx<T> ru[PTS];
  T rk[PTS];
  auto fetch = [&](int t) {
    const int x0 = (t % ntx) * WT_X - R, y0 = (t / ntx) * WT_Y - R;
#pragma unroll
    for (int q = 0; q < PTS; ++q) {
      const int idx = min(tid + q * NT, NP - 1);
      const int r = idx / SX, c = idx - r * SX;
      const int xc = min(max(x0 + c, 0), nx - 1), yc = min(max(y0 + r, 0), ny - 1);
      const size_t p = (size_t)yc * nx + xc;
      ru[q] = u[p];
      rk[q] = k[p];
    }
  };
  fetch(tile);
  for (;;) {
    const int x0 = (tile % ntx) * WT_X, y0 = (tile / ntx) * WT_Y;
    const bool edge = x0 < R || y0 < R || x0 + WT_X + R > nx || y0 + WT_Y + R > ny;
    __syncthreads();                             // the previous tile is no longer read
#pragma unroll
    for (int q = 0; q < PTS; ++q) {
      const int idx = tid + q * NT;
      if (idx < NP) {
        const int r = idx / SX, c = idx - r * SX;
        const int x = x0 - R + c, y = y0 - R + r;
        const bool xin = (unsigned)x < (unsigned)nx, yin = (unsigned)y < (unsigned)ny;
        cx<T> uv = mk(T(0), T(0));
        T k2 = T(0);
        if (xin && yin) {
          uv = ru[q];
          k2 = rk[q] * rk[q];
        } else if ((yin && (x == -1 || x == nx)) || (xin && (y == -1 || y == ny))) {
          const T c2 = d.two_H * rk[q];          // i 2H k_b u_b; the mirror is added below
          uv = mk(-c2 * ru[q].im, c2 * ru[q].re);
        }
        // the ghost values are linear in u, so scaling the extended tile scales u
        if constexpr (MODE == ST_SCALED) uv = sc * uv;
        su[r][c] = uv;
        sk[r][c] = k2;
      }
    }
    if (edge) {                                  // uniform over the block
      __syncthreads();
#pragma unroll
      for (int q = 0; q < PTS; ++q) {
        const int idx = tid + q * NT;
        if (idx < NP) {
          const int r = idx / SX, c = idx - r * SX;
          const int x = x0 - R + c, y = y0 - R + r;
          const bool xin = (unsigned)x < (unsigned)nx, yin = (unsigned)y < (unsigned)ny;
          if (yin && (x == -1 || x == nx)) su[r][c] = su[r][x < 0 ? c + 2 : c - 2] + su[r][c];
          else if (xin && (y == -1 || y == ny)) su[r][c] = su[y < 0 ? r + 2 : r - 2][c] + su[r][c];
        }
      }
    }
    // the next tile's loads (this tile again for the last one: cached) are
    // in flight during the arithmetic below
    const int next = tile + nloc < t_hi ? tile + nloc : tile;
    fetch(next);
    __syncthreads();
    const int tx = threadIdx.x;
    const int x = x0 + tx;
    const int ly0 = threadIdx.y * WT_R;
    T lre[WT_R], lim[WT_R], kre[WT_R], kim[WT_R];
#pragma unroll
    for (int o = 0; o < WT_R; ++o) { lre[o] = lim[o] = kre[o] = kim[o] = T(0); }
    // vertical weights without run-time indexing: a queue of m1/t1 shifted one
    // row per pass and, per output o, the weights m1[rr - o], t1[rr - o] of the
    // current pass (zero outside the stencil).  An index into the kernel
    // arguments inside the loop made scalar loads whose waits also drained the
    // tile's LDS reads.
    T qm[W], qt[W], mo[WT_R], to[WT_R];
#pragma unroll
    for (int a = 0; a < W; ++a) { qm[a] = d.m1[a]; qt[a] = d.t1[a]; }
#pragma unroll
    for (int o = 0; o < WT_R; ++o) { mo[o] = T(0); to[o] = T(0); }
#pragma unroll 1
    for (int rr = 0; rr < WT_R + 2 * R; ++rr) {
#pragma unroll
      for (int o = WT_R - 1; o > 0; --o) { mo[o] = mo[o - 1]; to[o] = to[o - 1]; }
      mo[0] = qm[0];
      to[0] = qt[0];
#pragma unroll
      for (int a = 0; a + 1 < W; ++a) { qm[a] = qm[a + 1]; qt[a] = qt[a + 1]; }
      qm[W - 1] = T(0);
      qt[W - 1] = T(0);
      T tur = 0, tui = 0, mur = 0, mui = 0, mwr = 0, mwi = 0;
#pragma unroll
      for (int a = 0; a < W; ++a) {
        const cx<T> uv = su[ly0 + rr][tx + a];
        const T k2 = sk[ly0 + rr][tx + a];
        const T ta = d.t1[a], ma = d.m1[a];
        tur += ta * uv.re; tui += ta * uv.im;
        mur += ma * uv.re; mui += ma * uv.im;
        const T mk2 = ma * k2;
        mwr += mk2 * uv.re; mwi += mk2 * uv.im;
      }
#pragma unroll
      for (int o = 0; o < WT_R; ++o) {         // tap row (b + R) = rr - o
        lre[o] += mo[o] * tur + to[o] * mur;
        lim[o] += mo[o] * tui + to[o] * mui;
        kre[o] += mo[o] * mwr;
        kim[o] += mo[o] * mwi;
      }
    }
    if (x < nx) {
#pragma unroll
      for (int o = 0; o < WT_R; ++o) {
        const int y = y0 + ly0 + o;
        if (y >= ny) break;
        const size_t p = (size_t)y * nx + x;
        const int cy = ly0 + o + R, cxl = tx + R;
        const cx<T> uc = su[cy][cxl];
        cx<T> au;
        const bool bnd = x == 0 || y == 0 || x == nx - 1 || y == ny - 1;
        if (bnd) {
          const T k2 = sk[cy][cxl];
          cx<T> s = mk(T(4) * uc.re, T(4) * uc.im);
          s = s - su[cy][cxl - 1];
          s = s - su[cy][cxl + 1];
          s = s - su[cy - 1][cxl];
          s = s - su[cy + 1][cxl];
          const cx<T> sk2 = mk(d.sig_re * k2, d.sig_im * k2) * uc;
          au = d.scale * (d.inv_H2 * s - sk2);
        } else {
          au = mk(lre[o] - (d.sig_re * kre[o] - d.sig_im * kim[o]),
                  lim[o] - (d.sig_re * kim[o] + d.sig_im * kre[o]));
        }
        if constexpr (MODE == ST_APPLY) {
          out[p] = au;
        } else if constexpr (MODE == ST_SCALED) {
          out[p] = au;
          vout[p] = uc;
        } else if constexpr (MODE == ST_RESID) {
          out[p] = b[p] - au;
        } else {
          const cx<T> dg = bnd ? five_point_diag(d, k, x, y) : wide_diag<T, R>(d, k, x, y);
          out[p] = uc + omega * cdiv(b[p] - au, dg);
        }
      }
    }
    if (next == tile) break;
    tile = next;
  }
}

template <typename T, int R>
__global__ void __launch_bounds__(NT) k_jacobi0(OpDesc<T> d, const T* __restrict__ k,
                                                const cx<T>* __restrict__ b, cx<T>* __restrict__ x_out,
                                                T omega, Batch z) {
  const int x = blockIdx.x * BX + threadIdx.x;
  const int y = blockIdx.y * BY + threadIdx.y;
  if (x >= d.nx || y >= d.ny) return;
  HM_MEMBER(k); HM_MEMBER(b); HM_MEMBER(x_out);
  if (z.use_omega) omega = (T)z.omega[blockIdx.z];
  const size_t p = (size_t)y * d.nx + x;
  cx<T> dg;
  if constexpr (R == 1) {
    dg = five_point_diag(d, k, x, y);
  } else {
    dg = is_boundary<T, R>(d, x, y) ? five_point_diag(d, k, x, y) : wide_diag<T, R>(d, k, x, y);
  }
  x_out[p] = omega * cdiv(b[p], dg);
}

// ---- transfers -------------------------------------------------------------

// With dir != 0 (Dirichlet boundaries) every transfer is masked to the
// interior: boundary values of the input count as zero and boundary values of
// the output are zero, so boundary-free vectors stay boundary-free.
__device__ __forceinline__ bool on_bnd(int x, int y, int nx, int ny) {
  return x == 0 || y == 0 || x == nx - 1 || y == ny - 1;
}

// ---- row-streaming transfers ------------------------------------------------
// One-thread-per-output transfers read their 3x3 / 5x5 neighbourhoods with
// stride-2 loads and stay far below the HBM rate.  These versions stream rows:
// a block is four waves side by side walking down TR coarse rows.  Lane l of a
// wave stands for coarse column I = I0 + l - 1; it loads its own fine pair
// (2I, 2I+1) (restriction) or coarse value I (prolongation) with coalesced
// loads and takes its neighbours' values across lanes.  Lanes 0 and 63 carry
// only the halo, so a wave produces the TW = 62 columns of lanes 1..62.  Every
// load reads a clamped address inside the grid and is masked afterwards (zero
// outside the grid, and on the boundary for Dirichlet transfers): with no
// branch around a load, the next rows' loads stay in flight while the current
// rows are filtered.  Summation order (horizontal, then vertical) is that of
// the separable weights.  Blocks go in the XCD-aware tile order.
constexpr int TW = 62;              // coarse columns per wave (lanes 1..62)
constexpr int TCOLS = 4 * TW;       // coarse columns per block

// blocks of a transfer with TRB coarse rows per block (8 per XCD turn)
inline unsigned sep_blocks(int nxc, int nyc, int trb) {
  const size_t nt = (size_t)((nxc + TCOLS - 1) / TCOLS) * ((nyc + trb - 1) / trb);
  return (unsigned)(8 * ((nt + 7) / 8));
}
// coarse rows per block: 8, or fewer on small grids so that the launch still
// has about four blocks per compute unit
inline int sep_rows(int nxc, int nyc) {
  int trb = 8;
  while (trb > 2 && sep_blocks(nxc, nyc, trb) < 1024) trb /= 2;
  return trb;
}

template <typename T>
__device__ __forceinline__ cx<T> lane_val(const cx<T>& v, int src) {
  return mk(__shfl(v.re, src, 64), __shfl(v.im, src, 64));
}

// Value at (x, y) of an nx x ny field, zero unless lo <= x < nx - lo and
// lo <= y < ny - lo; the load itself always reads a node of the grid.
template <typename T>
__device__ __forceinline__ cx<T> clamped_load(const cx<T>* __restrict__ f, int x, int y, int nx,
                                              int ny, int lo) {
  const int xc = min(max(x, 0), nx - 1), yc = min(max(y, 0), ny - 1);
  const cx<T> v = f[(size_t)yc * nx + xc];
  const bool in = x >= lo && x < nx - lo && y >= lo && y < ny - lo;
  return in ? v : mk(T(0), T(0));
}

// fine row values owned by one lane: its pair (2I, 2I+1)
template <typename T>
struct FinePair {
  cx<T> a, b;
};

template <typename T>
__device__ __forceinline__ FinePair<T> load_fine_pair(const cx<T>* __restrict__ f, int I, int y,
                                                      int nxf, int nyf, int lo) {
  FinePair<T> r;
  r.a = clamped_load(f, 2 * I, y, nxf, nyf, lo);
  r.b = clamped_load(f, 2 * I + 1, y, nxf, nyf, lo);
  return r;
}

// horizontal filter of one fine row at coarse column I (valid on lanes 1..62):
//   H = 2: (f[2I-2] + 4 f[2I-1] + 6 f[2I] + 4 f[2I+1] + f[2I+2]) / 8
//   H = 1: (f[2I-1] + 2 f[2I] + f[2I+1]) / 4
template <typename Ti, typename To, int H>
__device__ __forceinline__ cx<To> hfilter(const FinePair<Ti>& r, int lane) {
  const cx<Ti> pb = lane_val(r.b, lane - 1);
  if constexpr (H == 2) {
    const cx<Ti> pa = lane_val(r.a, lane - 1), na = lane_val(r.a, lane + 1);
    return mk(To(0.125) * (To)pa.re + To(0.5) * (To)pb.re + To(0.75) * (To)r.a.re +
                  To(0.5) * (To)r.b.re + To(0.125) * (To)na.re,
              To(0.125) * (To)pa.im + To(0.5) * (To)pb.im + To(0.75) * (To)r.a.im +
                  To(0.5) * (To)r.b.im + To(0.125) * (To)na.im);
  } else {
    return mk(To(0.25) * (To)pb.re + To(0.5) * (To)r.a.re + To(0.25) * (To)r.b.re,
              To(0.25) * (To)pb.im + To(0.5) * (To)r.a.im + To(0.25) * (To)r.b.im);
  }
}

// Restriction fine -> coarse: H = 2 is Z^T (p = [1 4 6 4 1]/8 per dimension),
// H = 1 full weighting ([1 2 1]/4 per dimension).
template <typename Ti, typename To, int H, int TR>
__global__ void __launch_bounds__(NT) k_restrict_rows(const cx<Ti>* __restrict__ f, int nxf, int nyf,
                                                      cx<To>* __restrict__ c, int nxc, int nyc,
                                                      int dir, Batch z) {
  int tx, ty;
  if (!xcd_tile((nxc + TCOLS - 1) / TCOLS, (nyc + TR - 1) / TR, tx, ty)) return;
  HM_MEMBER(f); HM_MEMBER(c);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int I = tx * TCOLS + w * TW + lane - 1;
  const bool owner = lane >= 1 && lane <= TW && I < nxc;
  const int J0 = ty * TR;
  const int lo = dir ? 1 : 0;
  const To vw[5] = {To(0.125), To(0.5), To(0.75), To(0.5), To(0.125)};
  const To fw[3] = {To(0.25), To(0.5), To(0.25)};
  // window of horizontally filtered fine rows 2J - H .. 2J + H
  cx<To> win[2 * H + 1];
#pragma unroll
  for (int t = 0; t < 2 * H - 1; ++t)            // rows 2 J0 - H .. 2 J0 + H - 2
    win[t + 2] = hfilter<Ti, To, H>(load_fine_pair(f, I, 2 * J0 - H + t, nxf, nyf, lo), lane);
  FinePair<Ti> cur0 = load_fine_pair(f, I, 2 * J0 + H - 1, nxf, nyf, lo);
  FinePair<Ti> cur1 = load_fine_pair(f, I, 2 * J0 + H, nxf, nyf, lo);
#pragma unroll
  for (int q = 0; q < TR; ++q) {
    const int J = J0 + q;
    if (J >= nyc) break;                         // uniform over the block
    FinePair<Ti> nxt0 = cur0, nxt1 = cur1;
    if (q + 1 < TR) {                            // next rows in flight
      nxt0 = load_fine_pair(f, I, 2 * J + H + 1, nxf, nyf, lo);
      nxt1 = load_fine_pair(f, I, 2 * J + H + 2, nxf, nyf, lo);
    }
#pragma unroll
    for (int t = 0; t < 2 * H - 1; ++t) win[t] = win[t + 2];
    win[2 * H - 1] = hfilter<Ti, To, H>(cur0, lane);
    win[2 * H] = hfilter<Ti, To, H>(cur1, lane);
    To re = To(0), im = To(0);
#pragma unroll
    for (int t = 0; t <= 2 * H; ++t) {
      const To wt = H == 2 ? vw[t] : fw[t];
      re += wt * win[t].re;
      im += wt * win[t].im;
    }
    if (owner) {
      cx<To> out = mk(re, im);
      if (dir && on_bnd(I, J, nxc, nyc)) out = mk(To(0), To(0));
      c[(size_t)J * nxc + I] = out;
    }
    cur0 = nxt0;
    cur1 = nxt1;
  }
}

// Prolongation coarse -> fine.  ZDEF: deflation interpolation Z written to f
// (fine 2I: (c[I-1] + 6 c[I] + c[I+1]) / 8, fine 2I+1: (c[I] + c[I+1]) / 2 per
// dimension); otherwise bilinear interpolation added to f.  Lanes 1..62
// produce the fine pair (2I, 2I+1) of their coarse column I.
template <typename Ti, typename To, bool ZDEF>
__device__ __forceinline__ void hinterp(const cx<Ti>& own, int lane, cx<To>& ev, cx<To>& od) {
  const cx<Ti> nv = lane_val(own, lane + 1);
  if constexpr (ZDEF) {
    const cx<Ti> pv = lane_val(own, lane - 1);
    ev = mk(To(0.125) * (To)pv.re + To(0.75) * (To)own.re + To(0.125) * (To)nv.re,
            To(0.125) * (To)pv.im + To(0.75) * (To)own.im + To(0.125) * (To)nv.im);
  } else {
    ev = mk((To)own.re, (To)own.im);
  }
  od = mk(To(0.5) * (To)own.re + To(0.5) * (To)nv.re, To(0.5) * (To)own.im + To(0.5) * (To)nv.im);
}

// the four fine values (rows 2J, 2J+1; columns 2I, 2I+1) a lane updates, read
// ahead of the bilinear correction (addresses clamped into the grid; values
// off the grid are never stored back)
template <typename T>
__device__ __forceinline__ void load_fine_quad(const cx<T>* __restrict__ f, int I, int J, int nxf,
                                               int nyf, cx<T> (&q)[2][2]) {
#pragma unroll
  for (int par = 0; par < 2; ++par)
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int x = min(max(2 * I + side, 0), nxf - 1);
      const int y = min(2 * J + par, nyf - 1);
      q[par][side] = f[(size_t)y * nxf + x];
    }
}

template <typename Ti, typename To, bool ZDEF, int TR>
__global__ void __launch_bounds__(NT) k_prolong_rows(const cx<Ti>* __restrict__ c, int nxc, int nyc,
                                                     cx<To>* __restrict__ f, int nxf, int nyf,
                                                     int dir, Batch z) {
  int tx, ty;
  if (!xcd_tile((nxc + TCOLS - 1) / TCOLS, (nyc + TR - 1) / TR, tx, ty)) return;
  HM_MEMBER(c); HM_MEMBER(f);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int I = tx * TCOLS + w * TW + lane - 1;
  const bool owner = lane >= 1 && lane <= TW && I < nxc;
  const int J0 = ty * TR;
  const int lo = dir ? 1 : 0;
  // Z: every coarse row of the block (J0 - 1 .. J0 + TR) is loaded before the
  // first store, so no wait in the row loop is held up by the stores; the
  // bilinear correction reads fine values too and streams rows instead
  constexpr int NPRE = ZDEF ? TR + 2 : 3;
  cx<Ti> crow[NPRE];
#pragma unroll
  for (int r = 0; r < NPRE; ++r) crow[r] = clamped_load(c, I, J0 - 1 + r, nxc, nyc, lo);
  // horizontal interpolants of coarse rows J-1, J, J+1: [row][even / odd]
  cx<To> hv[3][2];
  hinterp<Ti, To, ZDEF>(crow[0], lane, hv[1][0], hv[1][1]);
  hinterp<Ti, To, ZDEF>(crow[1], lane, hv[2][0], hv[2][1]);
  cx<Ti> cur = crow[2];
  cx<To> fcur[2][2];
  if constexpr (!ZDEF) load_fine_quad(f, I, J0, nxf, nyf, fcur);
#pragma unroll
  for (int q = 0; q < TR; ++q) {
    const int J = J0 + q;
    if (J >= nyc) break;                         // uniform over the block
    cx<Ti> nxt = cur;
    cx<To> fnxt[2][2];
    if (q + 1 < TR) {
      if constexpr (ZDEF) {
        nxt = crow[q + 3 < NPRE ? q + 3 : NPRE - 1];
      } else {                                   // next rows in flight
        nxt = clamped_load(c, I, J + 2, nxc, nyc, lo);
        load_fine_quad(f, I, J + 1, nxf, nyf, fnxt);
      }
    }
    hv[0][0] = hv[1][0]; hv[0][1] = hv[1][1];
    hv[1][0] = hv[2][0]; hv[1][1] = hv[2][1];
    hinterp<Ti, To, ZDEF>(cur, lane, hv[2][0], hv[2][1]);
#pragma unroll
    for (int par = 0; par < 2; ++par) {          // fine rows 2J, 2J+1
      const int y = 2 * J + par;
#pragma unroll
      for (int side = 0; side < 2; ++side) {     // fine columns 2I, 2I+1
        const int x = 2 * I + side;
        cx<To> v;
        if (par == 0) {
          if constexpr (ZDEF) {
            v = mk(To(0.125) * hv[0][side].re + To(0.75) * hv[1][side].re +
                       To(0.125) * hv[2][side].re,
                   To(0.125) * hv[0][side].im + To(0.75) * hv[1][side].im +
                       To(0.125) * hv[2][side].im);
          } else {
            v = hv[1][side];
          }
        } else {
          v = mk(To(0.5) * hv[1][side].re + To(0.5) * hv[2][side].re,
                 To(0.5) * hv[1][side].im + To(0.5) * hv[2][side].im);
        }
        if (!owner || x >= nxf || y >= nyf) continue;
        const size_t p = (size_t)y * nxf + x;
        const bool fb = dir && on_bnd(x, y, nxf, nyf);
        if constexpr (ZDEF) {
          f[p] = fb ? mk(To(0), To(0)) : v;
        } else {
          if (!fb) f[p] = fcur[par][side] + v;
        }
      }
    }
    cur = nxt;
    if constexpr (!ZDEF) {
#pragma unroll
      for (int par = 0; par < 2; ++par)
#pragma unroll
        for (int side = 0; side < 2; ++side) fcur[par][side] = fnxt[par][side];
    }
  }
}

template <typename Ti, typename To>
__global__ void __launch_bounds__(NT) k_inject(const Ti* __restrict__ f, int nxf, To* __restrict__ c,
                                               int nxc, int nyc) {
  const int I = blockIdx.x * BX + threadIdx.x;
  const int J = blockIdx.y * BY + threadIdx.y;
  if (I >= nxc || J >= nyc) return;
  c[(size_t)J * nxc + I] = (To)f[(size_t)(2 * J) * nxf + 2 * I];
}

template <typename Ti, typename To>
__global__ void __launch_bounds__(NT) k_convert_real(const Ti* __restrict__ a, To* __restrict__ b,
                                                     size_t n) {
  const size_t i = (size_t)blockIdx.x * NT + threadIdx.x;
  if (i < n) b[i] = (To)a[i];
}

// ---- vector kernels ----------------------------------------------------------

template <typename Ti, typename To>
__global__ void __launch_bounds__(NT) k_convert(const cx<Ti>* __restrict__ a, cx<To>* __restrict__ b,
                                                size_t n, Batch z) {
  const size_t i = (size_t)blockIdx.x * NT + threadIdx.x;
  HM_MEMBER(a); HM_MEMBER(b);
  if (i < n) b[i] = cvt<To>(a[i]);
}

template <typename T>
__global__ void __launch_bounds__(NT) k_add(const cx<T>* __restrict__ a, const cx<T>* __restrict__ b,
                                            cx<T>* __restrict__ out, size_t n, Batch z) {
  const size_t i = (size_t)blockIdx.x * NT + threadIdx.x;
  HM_MEMBER(a); HM_MEMBER(b); HM_MEMBER(out);
  if (i < n) out[i] = a[i] + b[i];
}

template <typename T>
__global__ void __launch_bounds__(NT) k_scale_dev(const cx<T>* __restrict__ x, cx<T>* __restrict__ y,
                                                  const c128* __restrict__ scal, int inv, size_t n,
                                                  Batch z) {
  const size_t i = (size_t)blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  HM_MEMBER(x); HM_MEMBER(y); HM_MEMBER(scal);
  const c128 sc = scal[0];
  if (inv) {
    const T s = (T)(1.0 / sc.re);
    y[i] = s * x[i];
  } else {
    y[i] = cvt<T>(sc) * x[i];
  }
}

template <typename T>
__global__ void __launch_bounds__(NT) k_zero(cx<T>* __restrict__ x, size_t n, Batch z) {
  const size_t i = (size_t)blockIdx.x * NT + threadIdx.x;
  HM_MEMBER(x);
  if (i < n) x[i] = mk(T(0), T(0));
}

template <typename T>
__global__ void __launch_bounds__(NT) k_combine(const cx<T>* __restrict__ V, size_t ldv, int m,
                                                const c128* __restrict__ coef, size_t coef_ld,
                                                double sign, cx<T>* __restrict__ out,
                                                int accumulate, size_t n, Batch z) {
  const size_t i = (size_t)blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  HM_MEMBER(V); HM_MEMBER(out);
  coef += (size_t)z.slot[blockIdx.z] * coef_ld;
  if (m < 0) m = z.cnt[blockIdx.z];
  double re = 0, im = 0;
#pragma unroll 8
  for (int j = 0; j < m; ++j) {
    const c128 c = coef[j];
    const cx<T> v = V[(size_t)j * ldv + i];
    re += c.re * (double)v.re - c.im * (double)v.im;
    im += c.re * (double)v.im + c.im * (double)v.re;
  }
  re *= sign;
  im *= sign;
  if (accumulate) {
    const cx<T> o = out[i];
    re += (double)o.re;
    im += (double)o.im;
  }
  out[i] = mk((T)re, (T)im);
}

// y = A x with A in complex128 in every precision (the coarsest multigrid
// solve stays FP64); x is widened exactly, y rounded to the level's type.
template <typename T>
__global__ void __launch_bounds__(NT) k_dense_matvec(const c128* __restrict__ A, int n,
                                                     const cx<T>* __restrict__ x, cx<T>* __restrict__ y,
                                                     Batch z) {
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  HM_MEMBER(A); HM_MEMBER(x); HM_MEMBER(y);
  double re = 0, im = 0;
  for (int j = 0; j < n; ++j) {
    const c128 a = A[(size_t)i * n + j];
    const cx<T> v = x[j];
    re += a.re * (double)v.re - a.im * (double)v.im;
    im += a.re * (double)v.im + a.im * (double)v.re;
  }
  y[i] = mk((T)re, (T)im);
}

__global__ void __launch_bounds__(NT) k_identity(c128* __restrict__ out, int n) {
  const size_t idx = (size_t)blockIdx.x * NT + threadIdx.x;
  if (idx >= (size_t)n * n) return;
  const size_t i = idx % n, j = idx / n;
  out[idx] = mk(i == j ? 1.0 : 0.0, 0.0);
}

// ---- reductions ----------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum of (re, im) over a 256-thread block; valid in thread 0.
__device__ __forceinline__ c128 block_sum(double re, double im, double* sh) {
  re = wave_sum(re);
  im = wave_sum(im);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
    sh[2 * wid] = re;
    sh[2 * wid + 1] = im;
  }
  __syncthreads();
  c128 r = mk(0.0, 0.0);
  if (threadIdx.x == 0) {
    for (int w = 0; w < NT / 64; ++w) {
      r.re += sh[2 * w];
      r.im += sh[2 * w + 1];
    }
  }
  return r;
}

inline size_t chunk_len(size_t n, int nchunks) { return (n + nchunks - 1) / nchunks; }

constexpr int G = 4;   // dot products per block in the multi-dot

// Streaming load of a basis element with the non-temporal hint (the caches
// need not keep it).
template <typename T>
__device__ __forceinline__ cx<T> load_stream(const cx<T>* p) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  const v2 t = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
  return mk(t.x, t.y);
}

// (re, im) += conj(v) w in FP64 with explicitly fused multiply-adds, so that
// every instantiation (plain or non-temporal loads) rounds the same way
template <typename T>
__device__ __forceinline__ void dot_acc(double& re, double& im, const cx<T>& v, const cx<T>& w) {
  re = fma((double)v.re, (double)w.re, re);
  re = fma((double)v.im, (double)w.im, re);
  im = fma((double)v.re, (double)w.im, im);
  im = fma(-(double)v.im, (double)w.re, im);
}

// One chunk of the partial dots of w with NG consecutive basis vectors (NG and
// the load kind fixed at compile time, so that the NG + 1 loads of a row are
// all in flight together); re/im accumulate over the rows in order.
template <typename T, int NG, bool NTL>
__device__ __forceinline__ void dot_rows(const cx<T>* __restrict__ V, size_t ldv,
                                         const cx<T>* __restrict__ w, size_t lo, size_t hi,
                                         double* re, double* im) {
  size_t i = lo + threadIdx.x;
  for (; i + NT < hi; i += 2 * NT) {
    const cx<T> wa = w[i], wb = w[i + NT];
    cx<T> va[NG], vb[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      va[g] = NTL ? load_stream(V + (size_t)g * ldv + i) : V[(size_t)g * ldv + i];
      vb[g] = NTL ? load_stream(V + (size_t)g * ldv + i + NT) : V[(size_t)g * ldv + i + NT];
    }
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      dot_acc(re[g], im[g], va[g], wa);
      dot_acc(re[g], im[g], vb[g], wb);
    }
  }
  if (i < hi) {
    const cx<T> wv = w[i];
    cx<T> v[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) v[g] = NTL ? load_stream(V + (size_t)g * ldv + i) : V[(size_t)g * ldv + i];
#pragma unroll
    for (int g = 0; g < NG; ++g) dot_acc(re[g], im[g], v[g], wv);
  }
}

template <typename T, int NG>
__device__ __forceinline__ void dot_rows_kind(const cx<T>* __restrict__ V, size_t ldv,
                                              const cx<T>* __restrict__ w, size_t lo, size_t hi,
                                              bool ntl, double* re, double* im) {
  if (ntl) dot_rows<T, NG, true>(V, ldv, w, lo, hi, re, im);
  else dot_rows<T, NG, false>(V, ldv, w, lo, hi, re, im);
}

// Partial dots of w with V_{i0}..V_{i0+G-1} over one chunk of the vector
// (block = (chunk, group)); partials[i * nchunks + chunk].  Few accumulators
// per thread keep occupancy high; the re-reads of w by the groups of a chunk
// are served by the caches.  STREAM (bases larger than the Infinity Cache):
// groups whose vectors are all older than the `recent` most recent ones are
// loaded with the non-temporal hint, the others with plain loads; otherwise
// every vector with plain loads, so that the update pass and the next step
// find them in the cache.
template <typename T, bool STREAM>
__global__ void __launch_bounds__(NT) k_multidot(const cx<T>* __restrict__ V, size_t ldv, int m,
                                                 const cx<T>* __restrict__ w, size_t n, size_t clen,
                                                 c128* __restrict__ partials, int nchunks,
                                                 int recent, Batch z) {
  __shared__ double sh[NT / 64][2 * G];
  HM_MEMBER(V); HM_MEMBER(w); HM_MEMBER(partials);
  // XCD-aware block order: workgroups are dispatched round-robin over the 8
  // XCDs, so blocks b, b + 8, b + 16, ... share an L2.  All groups of one chunk
  // go to the same XCD in consecutive order: the chunk of w comes from HBM once
  // and from that L2 for the other groups.  nchunks is a multiple of 8.
  const int ngroups = (m + G - 1) / G;
  const int xcd = blockIdx.x & 7, local = blockIdx.x >> 3;
  const int chunk = (local / ngroups) * 8 + xcd;
  const int i0 = (local % ngroups) * G;
  const size_t lo = (size_t)chunk * clen;
  const size_t hi = lo + clen < n ? lo + clen : n;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double re[G], im[G];
#pragma unroll
  for (int g = 0; g < G; ++g) { re[g] = 0; im[g] = 0; }
  const int gm = m - i0 < G ? m - i0 : G;           // vectors of this group
  const bool ntl = STREAM && i0 + gm <= m - recent;
  const cx<T>* Vg = V + (size_t)i0 * ldv;
  static_assert(G == 4, "the group tails below cover G = 4");
  if (gm == 4) dot_rows_kind<T, 4>(Vg, ldv, w, lo, hi, ntl, re, im);
  else if (gm == 3) dot_rows_kind<T, 3>(Vg, ldv, w, lo, hi, ntl, re, im);
  else if (gm == 2) dot_rows_kind<T, 2>(Vg, ldv, w, lo, hi, ntl, re, im);
  else dot_rows_kind<T, 1>(Vg, ldv, w, lo, hi, ntl, re, im);
#pragma unroll
  for (int g = 0; g < G; ++g) {
    re[g] = wave_sum(re[g]);
    im[g] = wave_sum(im[g]);
  }
  if (lane == 0) {
#pragma unroll
    for (int g = 0; g < G; ++g) {
      sh[wid][2 * g] = re[g];
      sh[wid][2 * g + 1] = im[g];
    }
  }
  __syncthreads();
  if (threadIdx.x < G && i0 + (int)threadIdx.x < m) {
    const int g = threadIdx.x;
    double sr = 0, si = 0;
    for (int w2 = 0; w2 < NT / 64; ++w2) {
      sr += sh[w2][2 * g];
      si += sh[w2][2 * g + 1];
    }
    partials[(size_t)(i0 + g) * nchunks + chunk] = mk(sr, si);
  }
}

// ---- S Arnoldi steps per pair of sweeps over the basis (S = 1, 2, 3) ----------
// Pass A reads the basis vectors GP per block.
constexpr int GP = 2;
// Pass A rows: the partial dots of the S right vectors Y_0..Y_{S-1} with NG left
// vectors vp[0..NG-1] over one chunk, each thread two rows per pass.
template <typename T, int NG, bool NTL, int S>
__device__ __forceinline__ void dots_rows(const cx<T>* const* vp, const cx<T>* const* yp,
                                          size_t lo, size_t hi, double (*re)[GP],
                                          double (*im)[GP]) {
  size_t i = lo + threadIdx.x;
  for (; i + NT < hi; i += 2 * NT) {
    cx<T> ya[S], yb[S], va[NG], vb[NG];
#pragma unroll
    for (int r = 0; r < S; ++r) { ya[r] = yp[r][i]; yb[r] = yp[r][i + NT]; }
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      va[g] = NTL ? load_stream(vp[g] + i) : vp[g][i];
      vb[g] = NTL ? load_stream(vp[g] + i + NT) : vp[g][i + NT];
    }
#pragma unroll
    for (int r = 0; r < S; ++r)
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        dot_acc(re[r][g], im[r][g], va[g], ya[r]);
        dot_acc(re[r][g], im[r][g], vb[g], yb[r]);
      }
  }
  if (i < hi) {
    cx<T> y[S], v[NG];
#pragma unroll
    for (int r = 0; r < S; ++r) y[r] = yp[r][i];
#pragma unroll
    for (int g = 0; g < NG; ++g) v[g] = NTL ? load_stream(vp[g] + i) : vp[g][i];
#pragma unroll
    for (int r = 0; r < S; ++r)
#pragma unroll
      for (int g = 0; g < NG; ++g) dot_acc(re[r][g], im[r][g], v[g], y[r]);
  }
}

// Pass A of S Arnoldi steps (Y_0 = z = M v_j, Y_{k+1} = M Y_k): the dots of
// Y_0..Y_{S-1} with V_0..V_{m-1} and with the Y themselves, in one read of the
// basis.  Block = (chunk, group): group gi < ngv holds V_{GP gi}..V_{GP gi + 1},
// the groups after it hold the Y, GP at a time.  Value r (m + S) + i for right
// vector Y_r and left vector i (V_i for i < m, then Y_{i-m}):
// partials[value * nchunks + chunk].  Chunks, block order and load policy as
// k_multidot.
template <typename T, bool STREAM, int S>
__global__ void __launch_bounds__(NT) k_multidots(const cx<T>* __restrict__ V, size_t ldv, int m,
                                                  const cx<T>* __restrict__ y0,
                                                  const cx<T>* __restrict__ y1,
                                                  const cx<T>* __restrict__ y2, size_t n,
                                                  size_t clen, c128* __restrict__ partials,
                                                  int nchunks, int recent, Batch z) {
  __shared__ double sh[NT / 64][2 * S * GP];
  HM_MEMBER(V); HM_MEMBER(y0); HM_MEMBER(y1); HM_MEMBER(y2); HM_MEMBER(partials);
  const cx<T>* yp[3] = {y0, y1, y2};
  constexpr int ngy = (S + GP - 1) / GP;
  const int ngv = (m + GP - 1) / GP, ngroups = ngv + ngy;
  const int xcd = blockIdx.x & 7, local = blockIdx.x >> 3;
  const int chunk = (local / ngroups) * 8 + xcd;
  const int gi = local % ngroups;
  const size_t lo = (size_t)chunk * clen;
  const size_t hi = lo + clen < n ? lo + clen : n;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double re[S][GP], im[S][GP];
#pragma unroll
  for (int r = 0; r < S; ++r)
#pragma unroll
    for (int g = 0; g < GP; ++g) re[r][g] = im[r][g] = 0;
  int first, gm;                                 // first left index, left vectors
  const cx<T>* vp[GP];
  bool ntl = false;
  if (gi < ngv) {
    first = gi * GP;
    gm = m - first < GP ? m - first : GP;
    ntl = STREAM && first + gm <= m - recent;
#pragma unroll
    for (int g = 0; g < GP; ++g) vp[g] = V + (size_t)(first + (g < gm ? g : 0)) * ldv;
  } else {
    const int k0 = (gi - ngv) * GP;
    first = m + k0;
    gm = S - k0 < GP ? S - k0 : GP;
#pragma unroll
    for (int g = 0; g < GP; ++g) vp[g] = yp[k0 + (g < gm ? g : 0)];
  }
  static_assert(GP == 2, "the group tails below cover GP = 2");
  if (gm == 2) {
    if (ntl) dots_rows<T, 2, true, S>(vp, yp, lo, hi, re, im);
    else dots_rows<T, 2, false, S>(vp, yp, lo, hi, re, im);
  } else {
    if (ntl) dots_rows<T, 1, true, S>(vp, yp, lo, hi, re, im);
    else dots_rows<T, 1, false, S>(vp, yp, lo, hi, re, im);
  }
#pragma unroll
  for (int r = 0; r < S; ++r)
#pragma unroll
    for (int g = 0; g < GP; ++g) {
      re[r][g] = wave_sum(re[r][g]);
      im[r][g] = wave_sum(im[r][g]);
    }
  if (lane == 0) {
#pragma unroll
    for (int r = 0; r < S; ++r)
#pragma unroll
      for (int g = 0; g < GP; ++g) {
        sh[wid][2 * (r * GP + g)] = re[r][g];
        sh[wid][2 * (r * GP + g) + 1] = im[r][g];
      }
  }
  __syncthreads();
  if (threadIdx.x < S * GP) {
    const int r = threadIdx.x / GP, g = threadIdx.x - r * GP;
    if (g < gm) {
      double sr = 0, si = 0;
      for (int w2 = 0; w2 < NT / 64; ++w2) {
        sr += sh[w2][2 * (r * GP + g)];
        si += sh[w2][2 * (r * GP + g) + 1];
      }
      partials[(size_t)(r * (m + S) + first + g) * nchunks + chunk] = mk(sr, si);
    }
  }
}

// out[i] = sum_c partials[i*nchunks + c]; sqrt_re: out = sqrt(re)
__global__ void __launch_bounds__(NT) k_final(const c128* __restrict__ partials, int nchunks,
                                              c128* __restrict__ out, int sqrt_re,
                                              c128* __restrict__ host_out, Batch z) {
  __shared__ double sh[2 * NT / 64];
  HM_MEMBER(partials); HM_MEMBER(out);
  host_out = at_member(host_out, z.hz, z);
  const int i = blockIdx.x;
  double re = 0, im = 0;
  for (int c = threadIdx.x; c < nchunks; c += NT) {
    const c128 v = partials[(size_t)i * nchunks + c];
    re += v.re;
    im += v.im;
  }
  const c128 s = block_sum(re, im, sh);
  if (threadIdx.x == 0) {
    const c128 v = sqrt_re ? mk(sqrt(s.re), 0.0) : s;
    out[i] = v;
    if (host_out) host_out[i] = v;      // pinned host mirror, read after an event
  }
}

// Partial of next^H w (NEXT) or of ||w||^2 for one row.
template <typename T, bool NEXT>
__device__ __forceinline__ void mgs_acc(double& re, double& im, const cx<T>& wv, const cx<T>& v) {
  if (NEXT) {
    re += (double)v.re * (double)wv.re + (double)v.im * (double)wv.im;
    im += (double)v.re * (double)wv.im - (double)v.im * (double)wv.re;
  } else {
    re += (double)wv.re * (double)wv.re + (double)wv.im * (double)wv.im;
  }
}

// One modified Gram-Schmidt step fused with the next dot: w -= hprev * prev
// (PREV), then the chunk's partial of next^H w (NEXT) or of ||w||^2.  Which of
// prev and next are present is fixed at compile time, and each thread takes
// two rows per pass, so that the loads of both rows are in flight together;
// the partial sums its rows in order.
template <typename T, bool PREV, bool NEXT>
__global__ void __launch_bounds__(NT) k_mgs_step(cx<T>* __restrict__ w, const cx<T>* __restrict__ prev,
                                                 const c128* __restrict__ hprev,
                                                 const cx<T>* __restrict__ next, size_t n, size_t clen,
                                                 c128* __restrict__ partials, Batch z) {
  __shared__ double sh[2 * NT / 64];
  HM_MEMBER(w); HM_MEMBER(prev); HM_MEMBER(hprev); HM_MEMBER(next); HM_MEMBER(partials);
  const size_t lo = (size_t)blockIdx.x * clen;
  const size_t hi = lo + clen < n ? lo + clen : n;
  double re = 0, im = 0;
  cx<T> h = mk(T(0), T(0));
  if (PREV) h = cvt<T>(hprev[0]);
  const cx<T> zero = mk(T(0), T(0));
  size_t i = lo + threadIdx.x;
  for (; i + NT < hi; i += 2 * NT) {
    cx<T> wa = w[i], wb = w[i + NT];
    const cx<T> pa = PREV ? prev[i] : zero, pb = PREV ? prev[i + NT] : zero;
    const cx<T> na = NEXT ? next[i] : zero, nb = NEXT ? next[i + NT] : zero;
    if (PREV) {
      wa = wa - h * pa;
      wb = wb - h * pb;
      w[i] = wa;
      w[i + NT] = wb;
    }
    mgs_acc<T, NEXT>(re, im, wa, na);
    mgs_acc<T, NEXT>(re, im, wb, nb);
  }
  if (i < hi) {
    cx<T> wa = w[i];
    if (PREV) {
      wa = wa - h * prev[i];
      w[i] = wa;
    }
    mgs_acc<T, NEXT>(re, im, wa, NEXT ? next[i] : zero);
  }
  const c128 s = block_sum(re, im, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// (re, im) += c v in FP64 with explicitly fused multiply-adds (the same
// rounding in every instantiation)
template <typename T>
__device__ __forceinline__ void upd_acc(double& re, double& im, const c128& c, const cx<T>& v) {
  re = fma(c.re, (double)v.re, re);
  re = fma(-c.im, (double)v.im, re);
  im = fma(c.re, (double)v.im, im);
  im = fma(c.im, (double)v.re, im);
}

// w -= sum_j h_j V_j with the partial ||w||^2 of one chunk; every thread
// updates two elements (i, i + NT) per pass for more loads in flight.
template <typename T, bool STREAM>
__global__ void __launch_bounds__(NT) k_cgs_update_norm(cx<T>* __restrict__ w, const cx<T>* __restrict__ V,
                                                        size_t ldv, int m, const c128* __restrict__ h,
                                                        size_t n, size_t clen,
                                                        c128* __restrict__ partials, int recent,
                                                        Batch z) {
  __shared__ double sh[2 * NT / 64];
  HM_MEMBER(w); HM_MEMBER(V); HM_MEMBER(h); HM_MEMBER(partials);
  const int chunk = (int)blockIdx.x;
  const size_t lo = (size_t)chunk * clen;
  const size_t hi = lo + clen < n ? lo + clen : n;
  double acc = 0;
  for (size_t i = lo + threadIdx.x; i < hi; i += 2 * NT) {
    const size_t i2 = i + NT;
    const bool two = i2 < hi;
    const cx<T> w0 = w[i];
    const cx<T> w1 = two ? w[i2] : mk(T(0), T(0));
    double re0 = 0, im0 = 0, re1 = 0, im1 = 0;
#pragma unroll 8
    for (int j = 0; j < m; ++j) {
      const c128 c = h[j];
      const bool old = STREAM && j < m - recent;   // see k_multidot
      const cx<T> v0 = old ? load_stream(V + (size_t)j * ldv + i) : V[(size_t)j * ldv + i];
      upd_acc(re0, im0, c, v0);
      if (two) {
        const cx<T> v1 = old ? load_stream(V + (size_t)j * ldv + i2) : V[(size_t)j * ldv + i2];
        upd_acc(re1, im1, c, v1);
      }
    }
    const cx<T> n0 = mk((T)((double)w0.re - re0), (T)((double)w0.im - im0));
    w[i] = n0;
    acc = fma((double)n0.re, (double)n0.re, acc);
    acc = fma((double)n0.im, (double)n0.im, acc);
    if (two) {
      const cx<T> n1 = mk((T)((double)w1.re - re1), (T)((double)w1.im - im1));
      w[i2] = n1;
      acc = fma((double)n1.re, (double)n1.re, acc);
      acc = fma((double)n1.im, (double)n1.im, acc);
    }
  }
  const c128 s = block_sum(acc, 0.0, sh);
  if (threadIdx.x == 0) partials[chunk] = s;
}

// Pass B of S Arnoldi steps, one read of the basis: with coefficient rows
// C_t = coef + t cld (V_i at C_t[i], Y_k at C_t[m + k]),
//   V_{m+t} = sum_i C_t[i] V_i + sum_k C_t[m+k] Y_k   (t = 0..S-2, new basis vectors)
//   Y_0    <- sum_i C_{S-1}[i] V_i + sum_k C_{S-1}[m+k] Y_k   (the next unnormalised vector)
// with the partial ||Y_0||^2 of one chunk; two elements per thread per pass.
// Chunks and load policy as k_cgs_update_norm.
template <typename T, bool STREAM, int S>
__global__ void __launch_bounds__(NT) k_updates(cx<T>* __restrict__ y0,
                                                const cx<T>* __restrict__ y1,
                                                const cx<T>* __restrict__ y2,
                                                cx<T>* __restrict__ V, size_t ldv, int m,
                                                const c128* __restrict__ coef, int cld, size_t n,
                                                size_t clen, c128* __restrict__ partials,
                                                int recent, Batch z) {
  __shared__ double sh[2 * NT / 64];
  HM_MEMBER(y0); HM_MEMBER(y1); HM_MEMBER(y2); HM_MEMBER(V); HM_MEMBER(coef);
  HM_MEMBER(partials);
  const cx<T>* yp[3] = {y0, y1, y2};
  const int chunk = (int)blockIdx.x;
  const size_t lo = (size_t)chunk * clen;
  const size_t hi = lo + clen < n ? lo + clen : n;
  double acc = 0;
  for (size_t i = lo + threadIdx.x; i < hi; i += 2 * NT) {
    const size_t i2 = i + NT;
    const bool two = i2 < hi;
    double r0[S], q0[S], r1[S], q1[S];
#pragma unroll
    for (int t = 0; t < S; ++t) r0[t] = q0[t] = r1[t] = q1[t] = 0;
#pragma unroll 2
    for (int j = 0; j < m; ++j) {
      const bool old = STREAM && j < m - recent;
      const cx<T> v0 = old ? load_stream(V + (size_t)j * ldv + i) : V[(size_t)j * ldv + i];
      const cx<T> v1 = two ? (old ? load_stream(V + (size_t)j * ldv + i2)
                                  : V[(size_t)j * ldv + i2])
                           : mk(T(0), T(0));
#pragma unroll
      for (int t = 0; t < S; ++t) {
        const c128 c = coef[(size_t)t * cld + j];
        upd_acc(r0[t], q0[t], c, v0);
        upd_acc(r1[t], q1[t], c, v1);
      }
    }
#pragma unroll
    for (int k = 0; k < S; ++k) {
      const cx<T> a = yp[k][i];
      const cx<T> b = two ? yp[k][i2] : mk(T(0), T(0));
#pragma unroll
      for (int t = 0; t < S; ++t) {
        const c128 c = coef[(size_t)t * cld + m + k];
        upd_acc(r0[t], q0[t], c, a);
        upd_acc(r1[t], q1[t], c, b);
      }
    }
#pragma unroll
    for (int t = 0; t + 1 < S; ++t) {
      V[(size_t)(m + t) * ldv + i] = mk((T)r0[t], (T)q0[t]);
      if (two) V[(size_t)(m + t) * ldv + i2] = mk((T)r1[t], (T)q1[t]);
    }
    const cx<T> n0 = mk((T)r0[S - 1], (T)q0[S - 1]);
    y0[i] = n0;
    acc = fma((double)n0.re, (double)n0.re, acc);
    acc = fma((double)n0.im, (double)n0.im, acc);
    if (two) {
      const cx<T> n1 = mk((T)r1[S - 1], (T)q1[S - 1]);
      y0[i2] = n1;
      acc = fma((double)n1.re, (double)n1.re, acc);
      acc = fma((double)n1.im, (double)n1.im, acc);
    }
  }
  const c128 s = block_sum(acc, 0.0, sh);
  if (threadIdx.x == 0) partials[chunk] = s;
}

template <typename T>
__global__ void __launch_bounds__(NT) k_norm2(const cx<T>* __restrict__ x, size_t n, size_t clen,
                                              c128* __restrict__ partials, Batch z) {
  __shared__ double sh[2 * NT / 64];
  HM_MEMBER(x); HM_MEMBER(partials);
  const size_t lo = (size_t)blockIdx.x * clen;
  const size_t hi = lo + clen < n ? lo + clen : n;
  double acc = 0;
  for (size_t i = lo + threadIdx.x; i < hi; i += NT) {
    const cx<T> v = x[i];
    acc += (double)v.re * (double)v.re + (double)v.im * (double)v.im;
  }
  const c128 s = block_sum(acc, 0.0, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// True residual r = b - A u of the five-point operator d (FP64) over one chunk
// of the nodes, with the chunk's partial sums of |r|^2 (re) and |b|^2 (im);
// r is written when it is not null.
__global__ void __launch_bounds__(NT) k_residual_norm(OpDesc<double> d, const c128* __restrict__ u,
                                                      const double* __restrict__ k,
                                                      const c128* __restrict__ b,
                                                      c128* __restrict__ r, size_t n, size_t clen,
                                                      c128* __restrict__ partials) {
  __shared__ double sh[2 * NT / 64];
  const size_t lo = (size_t)blockIdx.x * clen;
  const size_t hi = lo + clen < n ? lo + clen : n;
  double rr = 0, bb = 0;
  for (size_t p = lo + threadIdx.x; p < hi; p += NT) {
    const int y = (int)(p / (size_t)d.nx);
    const int x = (int)(p - (size_t)y * d.nx);
    const c128 bv = b[p];
    const c128 rv = bv - five_point_any(d, u, k, x, y);
    if (r) r[p] = rv;
    rr += rv.re * rv.re + rv.im * rv.im;
    bb += bv.re * bv.re + bv.im * bv.im;
  }
  const c128 s = block_sum(rr, bb, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// norms[0] = sqrt(sum of re), norms[1] = sqrt(sum of im) over the partials,
// summed in a fixed order
__global__ void __launch_bounds__(NT) k_residual_final(const c128* __restrict__ partials,
                                                       int nchunks, double* __restrict__ norms) {
  __shared__ double sh[2 * NT / 64];
  double re = 0, im = 0;
  for (int c = threadIdx.x; c < nchunks; c += NT) {
    re += partials[c].re;
    im += partials[c].im;
  }
  const c128 s = block_sum(re, im, sh);
  if (threadIdx.x == 0) {
    norms[0] = sqrt(s.re);
    norms[1] = sqrt(s.im);
  }
}

__global__ void __launch_bounds__(NT) k_check_k(const double* __restrict__ k, size_t n, size_t clen,
                                                c128* __restrict__ partials) {
  __shared__ double sh[2 * NT / 64];
  const size_t lo = (size_t)blockIdx.x * clen;
  const size_t hi = lo + clen < n ? lo + clen : n;
  double bad = 0;
  for (size_t i = lo + threadIdx.x; i < hi; i += NT) {
    const double v = k[i];
    if (!(v >= 0.0) || !isfinite(v)) bad += 1.0;
  }
  const c128 s = block_sum(bad, 0.0, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ void __launch_bounds__(NT) k_max_partial(const double* __restrict__ a, size_t n, size_t clen,
                                                    c128* __restrict__ partials) {
  __shared__ double sh[NT / 64];
  const size_t lo = (size_t)blockIdx.x * clen;
  const size_t hi = lo + clen < n ? lo + clen : n;
  double m = -INFINITY;
  for (size_t i = lo + threadIdx.x; i < hi; i += NT) m = fmax(m, a[i]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < NT / 64; ++w) m = fmax(m, sh[w]);
    partials[blockIdx.x] = mk(m, 0.0);
  }
}

__global__ void __launch_bounds__(NT) k_max_final(const c128* __restrict__ partials, int nchunks,
                                                  c128* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double m = -INFINITY;
  for (int c = 0; c < nchunks; ++c) m = fmax(m, partials[c].re);
  out[0] = mk(m, 0.0);
}

// CSR of the five-point operator: row p = y*nx + x, entries at rowptr[p] = 5p.
// A neighbour outside the grid is the Sommerfeld ghost mirror + 2iHk u_centre:
// its coupling moves onto the mirrored inside neighbour (doubling it) and the
// 2iHk part is already in the diagonal; the freed slot keeps a zero.
__global__ void __launch_bounds__(NT) k_csr5_assemble(OpDesc<double> d, const double* __restrict__ k,
                                                      int* __restrict__ rowptr,
                                                      int* __restrict__ colidx,
                                                      c128* __restrict__ vals) {
  const size_t p = (size_t)blockIdx.x * NT + threadIdx.x;
  const size_t n = (size_t)d.nx * d.ny;
  if (p > n) return;
  rowptr[p] = (int)(5 * p);
  if (p == n) return;
  const int x = (int)(p % d.nx), y = (int)(p / d.nx);
  const double off = -d.scale * d.inv_H2;
  // slots: centre, west, east, south, north
  const int col[5] = {(int)p, (int)p - 1, (int)p + 1, (int)p - d.nx, (int)p + d.nx};
  const bool in[5] = {true, x > 0, x < d.nx - 1, y > 0, y < d.ny - 1};
  const int mirror[5] = {0, 2, 1, 4, 3};
  double c[5] = {0, 0, 0, 0, 0};
  for (int q = 1; q < 5; ++q) c[in[q] ? q : mirror[q]] += off;
  const size_t base = 5 * p;
  vals[base] = five_point_diag(d, k, x, y);
  colidx[base] = col[0];
  for (int q = 1; q < 5; ++q) {
    colidx[base + q] = in[q] ? col[q] : (int)p;
    vals[base + q] = mk(c[q], 0.0);
  }
}

// CSR SpMV in the "CSR-stream" form: when the NT rows of a block hold at most
// kCsrStage entries, the block forms the products vals[q] * x[col[q]] for its
// contiguous entry range with coalesced loads into LDS, and each thread then
// sums its row from LDS; a block with more entries falls back to one thread
// per row reading its entries directly.
constexpr int kCsrStage = 2048;

// x[c] for a column index inside [0, ncols), NaN otherwise (an index outside
// makes its row's result NaN instead of reading outside x)
__device__ __forceinline__ c128 csr_x(const c128* __restrict__ x, int c, int ncols) {
  return (unsigned)c < (unsigned)ncols ? x[c] : mk(__builtin_nan(""), __builtin_nan(""));
}

__global__ void __launch_bounds__(NT) k_csr_spmv(int nrows, int ncols, const int* __restrict__ rowptr,
                                                 const int* __restrict__ colidx,
                                                 const c128* __restrict__ vals,
                                                 const c128* __restrict__ x, c128* __restrict__ y) {
  __shared__ c128 prod[kCsrStage];
  const int r0 = blockIdx.x * NT;
  const int r1 = min(r0 + NT, nrows);
  const int r = r0 + (int)threadIdx.x;
  const int q0 = rowptr[r0], q1 = rowptr[r1];
  int a = 0, b = 0;
  if (r < nrows) {
    a = rowptr[r];
    b = rowptr[r + 1];
  }
  double re = 0, im = 0;
  if (q1 - q0 <= kCsrStage) {          // uniform over the block
#pragma unroll 4
    for (int i = threadIdx.x; i < q1 - q0; i += NT) {
      const c128 v = vals[q0 + i];
      const c128 xv = csr_x(x, colidx[q0 + i], ncols);
      prod[i] = mk(v.re * xv.re - v.im * xv.im, v.re * xv.im + v.im * xv.re);
    }
    __syncthreads();
    for (int q = a; q < b; ++q) {
      re += prod[q - q0].re;
      im += prod[q - q0].im;
    }
  } else {
    for (int q = a; q < b; ++q) {
      const c128 v = vals[q];
      const c128 xv = csr_x(x, colidx[q], ncols);
      re += v.re * xv.re - v.im * xv.im;
      im += v.re * xv.im + v.im * xv.re;
    }
  }
  if (r < nrows) y[r] = mk(re, im);
}

// ---- small coarse levels: one Krylov solve per workgroup ----------------------
// GMRES from x = 0 on the level's operator (the Krylov CSLP of Sec. 4.2, or a
// multigrid coarsest solve), run to its stopping test by one workgroup of 1024
// threads per member, with no host round trip per step: the operator applied
// from a ghost-extended copy of the whole level in LDS, classical (or
// modified) Gram-Schmidt with block reductions, the Givens rotations and the
// stopping test of reading R11 on the device, back substitution and x = V y.
// Used when the level fits in LDS; one launch replaces about five launches and
// one host wait per step.  For the operator a thread takes tasks of SG_RB
// vertically adjacent nodes of one column (rows reuse the stencil's row sums);
// a wave's lanes take
// consecutive columns; the Gram-Schmidt sweeps take nodes in row-major order
// with the work vector w in global memory (both stay in the caches on these
// sizes).
constexpr int SG_NT = 512;
constexpr int SG_WAVES = SG_NT / 64;
constexpr int SG_RB = 3;           // nodes of a task (one column)
constexpr int SG_G = 8;            // dots per block reduction (classical Gram-Schmidt)

// Sum over the block of NV complex values per thread; every thread gets the
// sums (fixed order: lanes by the wave reduction, then waves in order).  The
// first 2 NV threads add the wave partials and publish the sums, which every
// thread then reads once.
template <int NV>
__device__ __forceinline__ void sg_block_sum(double (&re)[NV], double (&im)[NV],
                                             double* __restrict__ red) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  // the wave sums of every value, level by level (the shuffles of one level
  // are independent and go out together; per value the order of wave_sum)
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      re[v] += __shfl_xor(re[v], off, 64);
      im[v] += __shfl_xor(im[v], off, 64);
    }
  }
  double* part = red;                       // [2 NV][SG_WAVES]
  double* sum = red + 2 * NV * SG_WAVES;    // [2 NV]
  __syncthreads();                          // the previous sums have been read
  if (lane == 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      part[(2 * v) * SG_WAVES + wid] = re[v];
      part[(2 * v + 1) * SG_WAVES + wid] = im[v];
    }
  }
  __syncthreads();
  if (threadIdx.x < 2 * NV) {
    double acc = 0;
    for (int w = 0; w < SG_WAVES; ++w) acc += part[threadIdx.x * SG_WAVES + w];
    sum[threadIdx.x] = acc;
  }
  __syncthreads();
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    re[v] = sum[2 * v];
    im[v] = sum[2 * v + 1];
  }
}

// Operator of the level at column x, rows y0 .. y0 + SG_RB - 1 (those inside the
// grid), from the ghost-extended level in LDS (row stride sx, offset R).
template <typename T, int R>
__device__ __forceinline__ void sg_apply(const OpDesc<T>& d, const cx<T>* __restrict__ su,
                                         const T* __restrict__ sk, int sx,
                                         const cx<T>* __restrict__ ug, int x, int y0,
                                         cx<T> (&out)[SG_RB]) {
  constexpr int W = 2 * R + 1;
  auto U = [&](int xx, int yy) { return su[(yy + R) * sx + xx + R]; };
  auto K2 = [&](int xx, int yy) { return sk[(yy + R) * sx + xx + R]; };
  T lre[SG_RB], lim[SG_RB], kre[SG_RB], kim[SG_RB];
#pragma unroll
  for (int o = 0; o < SG_RB; ++o) { lre[o] = lim[o] = kre[o] = kim[o] = T(0); }
  if constexpr (R >= 2) {
    // vertical weights without run-time indexing: a queue of m1/t1 shifted one
    // row per pass and, per output o, the weights m1[rr - o], t1[rr - o] of the
    // current pass (zero outside the stencil).  An index into the kernel
    // arguments inside the loop made scalar loads whose waits also drained the
    // tile's LDS reads.
    T qm[W], qt[W], mo[SG_RB], to[SG_RB];
#pragma unroll
    for (int a = 0; a < W; ++a) { qm[a] = d.m1[a]; qt[a] = d.t1[a]; }
#pragma unroll
    for (int o = 0; o < SG_RB; ++o) { mo[o] = T(0); to[o] = T(0); }
#pragma unroll 1
    for (int rr = 0; rr < SG_RB + 2 * R; ++rr) {
#pragma unroll
      for (int o = SG_RB - 1; o > 0; --o) { mo[o] = mo[o - 1]; to[o] = to[o - 1]; }
      mo[0] = qm[0];
      to[0] = qt[0];
#pragma unroll
      for (int a = 0; a + 1 < W; ++a) { qm[a] = qm[a + 1]; qt[a] = qt[a + 1]; }
      qm[W - 1] = T(0);
      qt[W - 1] = T(0);
      const int yy = y0 - R + rr;
      if (yy < -R || yy >= d.ny + R) continue;
      T tur = 0, tui = 0, mur = 0, mui = 0, mwr = 0, mwi = 0;
#pragma unroll
      for (int a = 0; a < W; ++a) {
        const cx<T> uv = U(x - R + a, yy);
        const T k2 = K2(x - R + a, yy);
        const T ta = d.t1[a], ma = d.m1[a];
        tur += ta * uv.re; tui += ta * uv.im;
        mur += ma * uv.re; mui += ma * uv.im;
        const T mk2 = ma * k2;
        mwr += mk2 * uv.re; mwi += mk2 * uv.im;
      }
#pragma unroll
      for (int o = 0; o < SG_RB; ++o) {        // tap row (b + R) = rr - o
        lre[o] += mo[o] * tur + to[o] * mur;
        lim[o] += mo[o] * tui + to[o] * mui;
        kre[o] += mo[o] * mwr;
        kim[o] += mo[o] * mwi;
      }
    }
  }
#pragma unroll
  for (int o = 0; o < SG_RB; ++o) {
    const int y = y0 + o;
    if (y >= d.ny) break;
    const cx<T> uc = U(x, y);
    const bool bnd = x == 0 || y == 0 || x == d.nx - 1 || y == d.ny - 1;
    if (bnd && d.bc) {
      // Dirichlet boundary row d_b u_b; the ghost-extended copy holds zero there
      out[o] = (d.scale * T(4) * d.inv_H2) * ug[(size_t)y * d.nx + x];
    } else if (bnd || R == 1) {
      const T k2 = K2(x, y);
      cx<T> s = mk(T(4) * uc.re, T(4) * uc.im);
      s = s - U(x - 1, y);
      s = s - U(x + 1, y);
      s = s - U(x, y - 1);
      s = s - U(x, y + 1);
      const cx<T> sk2 = mk(d.sig_re * k2, d.sig_im * k2) * uc;
      out[o] = d.scale * (d.inv_H2 * s - sk2);
    } else {
      out[o] = mk(lre[o] - (d.sig_re * kre[o] - d.sig_im * kim[o]),
                  lim[o] - (d.sig_re * kim[o] + d.sig_im * kre[o]));
    }
  }
}

// (ar, ai) += sum_{i < m} c_i V_i[p] in order, four basis loads in flight
template <typename T>
__device__ __forceinline__ void sg_combine(const cx<T>* __restrict__ V, int n, int p,
                                           const c128* __restrict__ c, int m, double& ar,
                                           double& ai) {
  int i = 0;
  for (; i + 4 <= m; i += 4) {
    cx<T> v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = V[(size_t)(i + q) * n + p];
#pragma unroll
    for (int q = 0; q < 4; ++q) upd_acc(ar, ai, c[i + q], v[q]);
  }
  for (; i < m; ++i) upd_acc(ar, ai, c[i], V[(size_t)i * n + p]);
}

template <typename T, int R>
__global__ void __launch_bounds__(SG_NT) k_gmres_small(OpDesc<T> d, const T* __restrict__ k,
                                                       const cx<T>* __restrict__ b,
                                                       cx<T>* __restrict__ x,
                                                       cx<T>* __restrict__ V,
                                                       cx<T>* __restrict__ w,
                                                       c128* __restrict__ H, SmallGmresArgs ga,
                                                       c128* __restrict__ info, Batch z) {
  extern __shared__ double smem[];
  HM_MEMBER(k); HM_MEMBER(b); HM_MEMBER(x); HM_MEMBER(V); HM_MEMBER(w); HM_MEMBER(H);
  info = at_member(info, z.hz, z);
  const int nx = d.nx, ny = d.ny;
  const int n = nx * ny;
  const int sx = nx + 2 * R, sy = ny + 2 * R;
  const int ldh = ga.ldh;
  const int maxit = ga.maxit[blockIdx.z];
  const double tol = ga.tol[blockIdx.z];
  const int tid = threadIdx.x;
  // LDS: reduction scratch, control slots, Givens state, the ghost-extended
  // level and its k^2
  double* red = smem;                                    // 2 SG_G (SG_WAVES + 1)
  double* ctl = red + 2 * SG_G * (SG_WAVES + 1);         // 4: stop, breakdown, estimate
  c128* hc = (c128*)(ctl + 4);                           // ldh: the current column / y
  c128* gs = hc + ldh;                                   // ldh: g
  c128* sn = gs + ldh;                                   // ldh: rotation sines
  double* cn = (double*)(sn + ldh);                      // ldh (even): rotation cosines
  cx<T>* su = (cx<T>*)(cn + ((ldh + 1) & ~1));
  T* sk = (T*)(su + (size_t)sx * sy);
  const int ntask = nx * ((ny + SG_RB - 1) / SG_RB);
  // k^2 of the level, ghost-extended once (the ghost wavenumber is zero)
  for (int idx = tid; idx < sx * sy; idx += SG_NT) {
    const int r = idx / sx, c = idx - r * sx;
    cx<T> uv;
    T k2;
    ext_val(d, b, k, c - R, r - R, uv, k2);
    sk[idx] = k2;
  }
  // beta = ||b||
  double bre[1] = {0}, bim[1] = {0};
  for (int p = tid; p < n; p += SG_NT) {
    const cx<T> v = b[p];
    bre[0] = fma((double)v.re, (double)v.re, bre[0]);
    bre[0] = fma((double)v.im, (double)v.im, bre[0]);
  }
  sg_block_sum<1>(bre, bim, red);
  const double beta = sqrt(bre[0]);
  if (beta == 0.0 || maxit <= 0) {
    for (int p = tid; p < n; p += SG_NT) x[p] = mk(T(0), T(0));
    if (tid == 0) info[0] = mk(0.0, beta);
    return;
  }
  {
    const T s = (T)(1.0 / beta);
    for (int p = tid; p < n; p += SG_NT) V[p] = s * b[p];
  }
  if (tid == 0) gs[0] = mk(beta, 0.0);
  int m = 0;
  for (int j = 0;; ++j) {
    const cx<T>* vj = V + (size_t)j * n;
    __syncthreads();                 // V_j written by every thread; LDS copy free
    for (int idx = tid; idx < sx * sy; idx += SG_NT) {
      const int r = idx / sx, c = idx - r * sx;
      cx<T> uv;
      T k2;
      ext_val(d, vj, k, c - R, r - R, uv, k2);
      su[idx] = uv;
    }
    __syncthreads();
    // w = Op V_j, SG_RB nodes of one column per task
    for (int task = tid; task < ntask; task += SG_NT) {
      const int x0 = task % nx, y0 = (task / nx) * SG_RB;
      cx<T> out[SG_RB];
      sg_apply<T, R>(d, su, sk, sx, vj, x0, y0, out);
#pragma unroll
      for (int o = 0; o < SG_RB; ++o)
        if (y0 + o < ny) w[(size_t)(y0 + o) * nx + x0] = out[o];
    }
    __syncthreads();                 // w complete
    // orthogonalise against V_0 .. V_j
    if (ga.mgs) {
      for (int i = 0; i <= j; ++i) {
        const cx<T>* vi = V + (size_t)i * n;
        double re[1] = {0}, im[1] = {0};
        for (int p = tid; p < n; p += SG_NT) dot_acc(re[0], im[0], vi[p], w[p]);
        sg_block_sum<1>(re, im, red);
        const c128 h = mk(re[0], im[0]);
        if (tid == 0) hc[i] = h;
        const cx<T> ht = cvt<T>(h);
        for (int p = tid; p < n; p += SG_NT) w[p] = w[p] - ht * vi[p];
        __syncthreads();
      }
    } else {
      for (int i0 = 0; i0 <= j; i0 += SG_G) {
        const int gm = j + 1 - i0 < SG_G ? j + 1 - i0 : SG_G;
        double re[SG_G], im[SG_G];
#pragma unroll
        for (int g = 0; g < SG_G; ++g) { re[g] = 0; im[g] = 0; }
        for (int p = tid; p < n; p += SG_NT) {
          const cx<T> wv = w[p];
          cx<T> vv[SG_G];
#pragma unroll
          for (int g = 0; g < SG_G; ++g)       // every load of the node in flight together
            vv[g] = V[(size_t)(i0 + (g < gm ? g : 0)) * n + p];
#pragma unroll
          for (int g = 0; g < SG_G; ++g)
            if (g < gm) dot_acc(re[g], im[g], vv[g], wv);
        }
        sg_block_sum<SG_G>(re, im, red);
        if (tid == 0)
          for (int g = 0; g < gm; ++g) hc[i0 + g] = mk(re[g], im[g]);
      }
      __syncthreads();               // hc complete
      for (int p = tid; p < n; p += SG_NT) {
        double ar = 0, ai = 0;
        sg_combine(V, n, p, hc, j + 1, ar, ai);
        const cx<T> wv = w[p];
        w[p] = mk((T)((double)wv.re - ar), (T)((double)wv.im - ai));
      }
    }
    double nre[1] = {0}, nim[1] = {0};
    for (int p = tid; p < n; p += SG_NT) {
      const cx<T> wv = w[p];
      nre[0] = fma((double)wv.re, (double)wv.re, nre[0]);
      nre[0] = fma((double)wv.im, (double)wv.im, nre[0]);
    }
    sg_block_sum<1>(nre, nim, red);
    const double hn = sqrt(nre[0]);
    // Givens rotations of the column (thread 0), the estimate |g_{j+1}|
    if (tid == 0) {
      c128* col = hc;                  // rotated in LDS, then stored as column j of H
      col[j + 1] = mk(hn, 0.0);
      for (int i = 0; i < j; ++i) {
        const c128 a = col[i], bb = col[i + 1];
        const c128 s = sn[i];
        const double c = cn[i];
        col[i] = mk(c * a.re, c * a.im) + s * bb;
        col[i + 1] = mk(c * bb.re, c * bb.im) - cmulc(s, a);
      }
      const c128 a = col[j], bb = col[j + 1];
      double c;
      c128 s;
      if (bb.re == 0.0 && bb.im == 0.0) {
        c = 1.0; s = mk(0.0, 0.0);
      } else if (a.re == 0.0 && a.im == 0.0) {
        c = 0.0; s = mk(1.0, 0.0);
      } else {
        const double aa = hypot(a.re, a.im);
        const double nrm = hypot(aa, hypot(bb.re, bb.im));
        c = aa / nrm;
        // s = (a / |a|) conj(b) / nrm
        const c128 t = cmulc(bb, mk(a.re / aa, a.im / aa));
        s = mk(t.re / nrm, t.im / nrm);
      }
      cn[j] = c;
      sn[j] = s;
      col[j] = mk(c * a.re, c * a.im) + s * bb;
      col[j + 1] = mk(0.0, 0.0);
      const c128 gj = gs[j];
      gs[j + 1] = mk(0.0, 0.0) - cmulc(s, gj);  // -conj(s) g_j
      gs[j] = mk(c * gj.re, c * gj.im);
      for (int i = 0; i <= j; ++i) H[(size_t)j * ldh + i] = col[i];
      const double est = hypot(gs[j + 1].re, gs[j + 1].im);
      const bool broke = hn <= 1e-14 * beta;
      ctl[0] = (broke || (tol >= 0.0 && est <= tol * beta) || j + 1 >= maxit) ? 1.0 : 0.0;
      ctl[1] = broke ? 1.0 : 0.0;
      ctl[2] = est;
    }
    __syncthreads();
    const bool stop = ctl[0] != 0.0, broke = ctl[1] != 0.0;
    if (!broke) {
      const T s = (T)(1.0 / hn);
      cx<T>* vn = V + (size_t)(j + 1) * n;
      for (int p = tid; p < n; p += SG_NT) vn[p] = s * w[p];
    }
    if (stop) {
      m = j + 1;
      break;
    }
  }
  // y from the rotated triangle (copied into the LDS the level used; thread 0
  // back-substitutes, y overwrites hc), then x = V y
  c128* tri = (c128*)su;                                 // m x m, column-major
  for (int e = tid; e < m * m; e += SG_NT) {
    const int col = e / m, row = e - col * m;
    if (row <= col) tri[e] = H[(size_t)col * ldh + row];
  }
  __syncthreads();
  if (tid == 0) {
    for (int i = m - 1; i >= 0; --i) {
      c128 acc = gs[i];
      for (int kk = i + 1; kk < m; ++kk) acc = acc - tri[kk * m + i] * hc[kk];
      hc[i] = cdiv(acc, tri[i * m + i]);
    }
    info[0] = mk((double)m, ctl[2] / beta);
  }
  __syncthreads();
  for (int p = tid; p < n; p += SG_NT) {
    double ar = 0, ai = 0;
    sg_combine(V, n, p, hc, m, ar, ai);
    x[p] = mk((T)ar, (T)ai);
  }
}

}  // namespace

// ============================ launchers ======================================

hipError_t launch_csr5_assemble(const OpDesc<double>& d, const double* k, int* rowptr, int* colidx,
                                c128* vals, hipStream_t s) {
  const size_t n = (size_t)d.nx * d.ny;
  k_csr5_assemble<<<blocks1d(n + 1), NT, 0, s>>>(d, k, rowptr, colidx, vals);
  return hipGetLastError();
}

hipError_t launch_csr_spmv(int nrows, int ncols, const int* rowptr, const int* colidx,
                           const c128* vals, const c128* x, c128* y, hipStream_t s) {
  k_csr_spmv<<<blocks1d((size_t)nrows), NT, 0, s>>>(nrows, ncols, rowptr, colidx, vals, x, y);
  return hipGetLastError();
}

// blocks of the tiled wide stencil: 8 equal ranges of tiles (one per XCD)
static unsigned wide_blocks(int nx, int ny) {
  const int nt = ((nx + WT_X - 1) / WT_X) * ((ny + WT_Y - 1) / WT_Y);
  return (unsigned)(8 * ((nt + 7) / 8));
}

// blocks of the persistent wide stencil: the blocks that fit on the device at
// once (shared by the members of a batch), 8 per round-robin turn over the
// XCDs, and no more per XCD than its range has tiles
template <typename T, int R, int MODE>
static unsigned persist_blocks(int nx, int ny, const Batch& z) {
  static int resident = 0;                     // per kernel instance; same value on every call
  if (resident == 0) {
    int dev = 0, ncu = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_wide_persist<T, R, MODE>, NT, 0) !=
            hipSuccess)
      return 0;
    resident = std::max(8, per_cu * ncu);
  }
  const int nt = ((nx + WT_X - 1) / WT_X) * ((ny + WT_Y - 1) / WT_Y);
  const int per = (nt + 7) / 8;
  const int nloc = std::max(1, std::min(per, resident / 8 / std::max(1, z.n)));
  return (unsigned)(8 * nloc);
}

// The persistent form serves the Sommerfeld grids, except the 5x5 Jacobi sweep:
// its persistent instance needs 144 VGPRs (3 waves per SIMD) and measured
// 75 us per launch at 2049^2 against 67 us for the one-tile-per-block form.
template <typename T>
hipError_t launch_stencil(const OpDesc<T>& d, int mode, const cx<T>* u, const T* k, const cx<T>* b,
                          cx<T>* out, T omega, hipStream_t s, const Batch& z) {
  const dim3 g = zgrid(five_point_blocks(d.nx, d.ny), z), blk(BX, BY);
  const dim3 gw = zgrid(wide_blocks(d.nx, d.ny), z);
#define HM_ST(R, M)                                                                           \
  if constexpr (R == 1) k_five_point<T, M><<<g, blk, 0, s>>>(d, u, k, b, out, omega, nullptr,    \
                                                             nullptr, z);                      \
  else if (d.bc == 0 && !(R == 2 && M == ST_JACOBI)) {                                         \
    const unsigned nb = persist_blocks<T, R, M>(d.nx, d.ny, z);                                 \
    if (nb == 0) return hipErrorInvalidValue;                                                   \
    k_wide_persist<T, R, M><<<zgrid(nb, z), blk, 0, s>>>(d, u, k, b, out, omega, nullptr,       \
                                                         nullptr, z);                           \
  } else k_wide_tiled<T, R, M><<<gw, blk, 0, s>>>(d, u, k, b, out, omega, nullptr, nullptr, z)
#define HM_STR(R)                              \
  if (mode == ST_APPLY) HM_ST(R, ST_APPLY);    \
  else if (mode == ST_RESID) HM_ST(R, ST_RESID); \
  else HM_ST(R, ST_JACOBI);
  if (d.R == 1) { HM_STR(1) }
  else if (d.R == 2) { HM_STR(2) }
  else if (d.R == 3) { HM_STR(3) }
  else return hipErrorInvalidValue;
#undef HM_STR
#undef HM_ST
  return hipGetLastError();
}

template <typename T>
hipError_t launch_stencil_scaled(const OpDesc<T>& d, const cx<T>* u, const T* k, const c128* scal,
                                 cx<T>* vout, cx<T>* out, hipStream_t s, const Batch& z) {
  const dim3 g = zgrid(five_point_blocks(d.nx, d.ny), z), blk(BX, BY);
  const dim3 gw = zgrid(wide_blocks(d.nx, d.ny), z);
  if (d.R == 1)
    k_five_point<T, ST_SCALED><<<g, blk, 0, s>>>(d, u, k, nullptr, out, T(0), scal, vout, z);
  else if (d.R == 2 && d.bc == 0)
    k_wide_persist<T, 2, ST_SCALED><<<zgrid(persist_blocks<T, 2, ST_SCALED>(d.nx, d.ny, z), z),
                                      blk, 0, s>>>(d, u, k, nullptr, out, T(0), scal, vout, z);
  else if (d.R == 3 && d.bc == 0)
    k_wide_persist<T, 3, ST_SCALED><<<zgrid(persist_blocks<T, 3, ST_SCALED>(d.nx, d.ny, z), z),
                                      blk, 0, s>>>(d, u, k, nullptr, out, T(0), scal, vout, z);
  else if (d.R == 2)
    k_wide_tiled<T, 2, ST_SCALED><<<gw, blk, 0, s>>>(d, u, k, nullptr, out, T(0), scal, vout, z);
  else if (d.R == 3)
    k_wide_tiled<T, 3, ST_SCALED><<<gw, blk, 0, s>>>(d, u, k, nullptr, out, T(0), scal, vout, z);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename T>
hipError_t launch_jacobi0(const OpDesc<T>& d, const T* k, const cx<T>* b, cx<T>* x, T omega,
                          hipStream_t s, const Batch& z) {
  const dim3 g = zgrid(grid2d(d.nx, d.ny), z), blk(BX, BY);
  if (d.R == 1) k_jacobi0<T, 1><<<g, blk, 0, s>>>(d, k, b, x, omega, z);
  else if (d.R == 2) k_jacobi0<T, 2><<<g, blk, 0, s>>>(d, k, b, x, omega, z);
  else if (d.R == 3) k_jacobi0<T, 3><<<g, blk, 0, s>>>(d, k, b, x, omega, z);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

// a transfer kernel K<ARGS..., TRB> with the rows per block chosen for the grid
#define HM_SEP_UNPACK(...) __VA_ARGS__
#define HM_SEP_LAUNCH(K, TARGS, ...)                                                           \
  do {                                                                                          \
    const int trb_ = sep_rows(nxc, nyc);                                                        \
    const dim3 g_ = zgrid(sep_blocks(nxc, nyc, trb_), z);                                       \
    if (trb_ == 8) K<HM_SEP_UNPACK TARGS, 8><<<g_, NT, 0, s>>>(__VA_ARGS__);                    \
    else if (trb_ == 4) K<HM_SEP_UNPACK TARGS, 4><<<g_, NT, 0, s>>>(__VA_ARGS__);               \
    else K<HM_SEP_UNPACK TARGS, 2><<<g_, NT, 0, s>>>(__VA_ARGS__);                              \
  } while (0)

template <typename Ti, typename To>
hipError_t launch_restrict_z(const cx<Ti>* f, int nxf, int nyf, cx<To>* c, int dir,
                             hipStream_t s, const Batch& z) {
  const int nxc = (nxf - 1) / 2 + 1, nyc = (nyf - 1) / 2 + 1;
  HM_SEP_LAUNCH(k_restrict_rows, (Ti, To, 2), f, nxf, nyf, c, nxc, nyc, dir, z);
  return hipGetLastError();
}

template <typename Ti, typename To>
hipError_t launch_prolong_z(const cx<Ti>* c, int nxf, int nyf, cx<To>* f, int dir,
                            hipStream_t s, const Batch& z) {
  const int nxc = (nxf - 1) / 2 + 1, nyc = (nyf - 1) / 2 + 1;
  HM_SEP_LAUNCH(k_prolong_rows, (Ti, To, true), c, nxc, nyc, f, nxf, nyf, dir, z);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_restrict_fw(const cx<T>* f, int nxf, int nyf, cx<T>* c, int dir, hipStream_t s,
                              const Batch& z) {
  const int nxc = (nxf - 1) / 2 + 1, nyc = (nyf - 1) / 2 + 1;
  HM_SEP_LAUNCH(k_restrict_rows, (T, T, 1), f, nxf, nyf, c, nxc, nyc, dir, z);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong_bilinear_add(const cx<T>* c, int nxf, int nyf, cx<T>* f, int dir,
                                       hipStream_t s, const Batch& z) {
  const int nxc = (nxf - 1) / 2 + 1, nyc = (nyf - 1) / 2 + 1;
  HM_SEP_LAUNCH(k_prolong_rows, (T, T, false), c, nxc, nyc, f, nxf, nyf, dir, z);
  return hipGetLastError();
}

template <typename Ti, typename To>
hipError_t launch_inject(const Ti* f, int nxf, int nyf, To* c, hipStream_t s) {
  const int nxc = (nxf - 1) / 2 + 1, nyc = (nyf - 1) / 2 + 1;
  k_inject<Ti, To><<<grid2d(nxc, nyc), dim3(BX, BY), 0, s>>>(f, nxf, c, nxc, nyc);
  return hipGetLastError();
}

template <typename Ti, typename To>
hipError_t launch_convert_real(const Ti* a, To* b, size_t n, hipStream_t s) {
  k_convert_real<Ti, To><<<blocks1d(n), NT, 0, s>>>(a, b, n);
  return hipGetLastError();
}

template <typename Ti, typename To>
hipError_t launch_convert(const cx<Ti>* a, cx<To>* b, size_t n, hipStream_t s, const Batch& z) {
  k_convert<Ti, To><<<zgrid(blocks1d(n), z), NT, 0, s>>>(a, b, n, z);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_add(const cx<T>* a, const cx<T>* b, cx<T>* out, size_t n, hipStream_t s,
                      const Batch& z) {
  k_add<T><<<zgrid(blocks1d(n), z), NT, 0, s>>>(a, b, out, n, z);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_scale_dev(const cx<T>* x, cx<T>* y, const c128* scal, int inv, size_t n,
                            hipStream_t s, const Batch& z) {
  k_scale_dev<T><<<zgrid(blocks1d(n), z), NT, 0, s>>>(x, y, scal, inv, n, z);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_zero(cx<T>* x, size_t n, hipStream_t s, const Batch& z) {
  k_zero<T><<<zgrid(blocks1d(n), z), NT, 0, s>>>(x, n, z);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_combine(const cx<T>* V, size_t ldv, int m, const c128* coef, size_t coef_ld,
                          double sign, cx<T>* out, int accumulate, size_t n, hipStream_t s,
                          const Batch& z) {
  k_combine<T><<<zgrid(blocks1d(n), z), NT, 0, s>>>(V, ldv, m, coef, coef_ld, sign, out, accumulate,
                                                    n, z);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dense_matvec(const c128* A, int n, const cx<T>* x, cx<T>* y, hipStream_t s,
                               const Batch& z) {
  k_dense_matvec<T><<<zgrid(blocks1d((size_t)n), z), NT, 0, s>>>(A, n, x, y, z);
  return hipGetLastError();
}

hipError_t launch_identity(c128* out, int n, hipStream_t s) {
  k_identity<<<blocks1d((size_t)n * n), NT, 0, s>>>(out, n);
  return hipGetLastError();
}

int reduction_chunks(size_t n) {
  size_t c = (n + NT * 2 - 1) / (NT * 2);
  if (c < 1) c = 1;
  if (c > (size_t)kMaxChunks) c = kMaxChunks;
  return (int)c;
}

// chunks of the multi-dot: long chunks (fewer partials per dot) for short
// bases, shorter ones for long bases; at least ~2048 blocks in flight when the
// vector allows one element per thread.  The chunk length is a whole number of
// 256-element passes and the chunk count a multiple of 8 (one slot per XCD;
// trailing chunks may be empty).
static size_t multidot_chunk_len(size_t n, int m) {
  const size_t per = m >= 40 ? NT * 4 : NT * 16;
  const int ngroups = (m + G - 1) / G;
  size_t nch = (n + per - 1) / per;
  const size_t want = (2048 + ngroups - 1) / ngroups;
  const size_t most = (n + NT - 1) / NT;
  if (nch < want) nch = want < most ? want : most;
  if (nch < 1) nch = 1;
  size_t clen = (n + nch - 1) / nch;
  clen = (clen + NT - 1) / NT * NT;
  while ((n + clen - 1) / clen > (size_t)kMaxChunks) clen += NT;
  return clen;
}
static int multidot_chunks(size_t n, int m, const RedBuf& rb) {
  (void)rb;
  const size_t clen = multidot_chunk_len(n, m);
  const size_t nch = (n + clen - 1) / clen;
  return (int)((nch + 7) & ~(size_t)7);
}

template <typename T>
hipError_t launch_multidot_partial(const cx<T>* V, size_t ldv, int m, const cx<T>* w, size_t n,
                                   RedBuf rb, hipStream_t s, const Batch& z,
                                   const CachePolicy& cp) {
  if (m <= 0) return hipSuccess;
  const int nch = multidot_chunks(n, m, rb);
  const size_t clen = multidot_chunk_len(n, m);
  // load policy (default kCacheBasisBytes, kCacheRecentBytes): measured on the
  // coarsest-level solves of 1025^2 .. 4097^2 and 4597 x 1453 problems
  const dim3 g = zgrid(((m + G - 1) / G) * nch, z);
  const int recent = (int)(cp.recent / ((double)n * sizeof(cx<T>)));
  if ((double)(m + 1) * (double)n * sizeof(cx<T>) > cp.basis)
    k_multidot<T, true><<<g, NT, 0, s>>>(V, ldv, m, w, n, clen, rb.partials, nch, recent, z);
  else
    k_multidot<T, false><<<g, NT, 0, s>>>(V, ldv, m, w, n, clen, rb.partials, nch, recent, z);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_multidot_final(int m, size_t n, RedBuf rb, c128* out, hipStream_t s,
                                 c128* host_out, const Batch& z) {
  if (m <= 0) return hipSuccess;
  k_final<<<zgrid(m, z), NT, 0, s>>>(rb.partials, multidot_chunks(n, m, rb), out, 0, host_out, z);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_multidot(const cx<T>* V, size_t ldv, int m, const cx<T>* w, size_t n, RedBuf rb,
                           c128* out, hipStream_t s) {
  const hipError_t e = launch_multidot_partial<T>(V, ldv, m, w, n, rb, s);
  if (e != hipSuccess) return e;
  return launch_multidot_final<T>(m, n, rb, out, s);
}

template <typename T>
hipError_t launch_mgs_step(cx<T>* w, const cx<T>* prev, const c128* hprev, const cx<T>* next,
                           size_t n, RedBuf rb, c128* out, hipStream_t s, c128* host_out,
                           const Batch& z) {
  const size_t clen = chunk_len(n, rb.nchunks);
  const dim3 g = zgrid(rb.nchunks, z);
  if (prev && next)
    k_mgs_step<T, true, true><<<g, NT, 0, s>>>(w, prev, hprev, next, n, clen, rb.partials, z);
  else if (prev)
    k_mgs_step<T, true, false><<<g, NT, 0, s>>>(w, prev, hprev, next, n, clen, rb.partials, z);
  else if (next)
    k_mgs_step<T, false, true><<<g, NT, 0, s>>>(w, prev, hprev, next, n, clen, rb.partials, z);
  else
    k_mgs_step<T, false, false><<<g, NT, 0, s>>>(w, prev, hprev, next, n, clen, rb.partials, z);
  k_final<<<zgrid(1, z), NT, 0, s>>>(rb.partials, rb.nchunks, out, next ? 0 : 1, host_out, z);
  return hipGetLastError();
}

// chunk length of the update: whole passes of the two-element loop, with
// e = 1, 2, 4, ... elements per thread growing like sqrt(n) / 256 (so the
// block count also grows like sqrt(n)); a partial last pass would make one
// thread of each block re-read all m basis vectors
static size_t update_chunk_len(size_t n) {
  size_t e = 1;
  while ((double)(2 * e) * NT <= std::sqrt((double)n) * 1.5) e *= 2;
  size_t clen = (size_t)NT * e;
  while ((n + clen - 1) / clen > (size_t)kMaxChunks) clen += 2 * NT;
  return clen;
}
static int update_chunks(size_t n, const RedBuf& rb) {
  (void)rb;
  return (int)((n + update_chunk_len(n) - 1) / update_chunk_len(n));
}

template <typename T>
hipError_t launch_cgs_update_partial(cx<T>* w, const cx<T>* V, size_t ldv, int m, const c128* h,
                                     size_t n, RedBuf rb, hipStream_t s,
                                     const Batch& z, const CachePolicy& cp) {
  const int nch = update_chunks(n, rb);
  const size_t clen = update_chunk_len(n);
  const int recent = (int)(cp.recent / ((double)n * sizeof(cx<T>)));
  const dim3 g = zgrid(nch, z);
  if ((double)(m + 1) * (double)n * sizeof(cx<T>) > cp.basis)
    k_cgs_update_norm<T, true><<<g, NT, 0, s>>>(w, V, ldv, m, h, n, clen, rb.partials, recent, z);
  else
    k_cgs_update_norm<T, false><<<g, NT, 0, s>>>(w, V, ldv, m, h, n, clen, rb.partials, recent, z);
  return hipGetLastError();
}

hipError_t launch_update_norm_final(size_t n, RedBuf rb, c128* out, hipStream_t s,
                                    c128* host_out, const Batch& z) {
  k_final<<<zgrid(1, z), NT, 0, s>>>(rb.partials, update_chunks(n, rb), out, 1, host_out, z);
  return hipGetLastError();
}

// Between the passes of S Arnoldi steps (one block per member): Arnoldi in the
// coordinates of B = [V_0..V_j, Y_0..Y_{S-1}] (m = j + 1 basis vectors, taken
// as orthonormal) with the inner products of pass A (d[r (m + S) + i] =
// (left i)^H Y_r), G = B^H B.  M acts on coordinates through the Hessenberg
// columns 0..j-1 in H (M V_i = V H_{., i}), M v_j = Y_0 and M Y_k = Y_{k+1}.
// Step j + t (t < S) takes w = M q_{j+t}, h = <q_l, w>_G for every earlier
// vector (classical Gram-Schmidt, one pass), w -= sum h_l q_l and, for
// t < S - 1, q_{j+t+1} = w / <w, w>_G^(1/2); the last step's subdiagonal entry
// is the explicit norm that pass B takes.  Columns j..j+S-1 go to H and the
// pinned mirror Hh; pass B's coefficient rows (the coordinates of
// q_{j+1}..q_{j+S-1} and of the last w) to coef, cld apart.  Coordinates in
// LDS: nb = m + S <= kCoefMax.
// The kernel is one workgroup whose time is latency.  The coordinate work
// (O(m S) per step) runs in wave 0 alone, lane l holding rows l, l + 64, ...,
// so its sums are wave reductions without barriers; the products with H
// (t >= 1, O(m^2)) are split evenly over every wave.
constexpr int kCoefMax = 512;
constexpr int NC = 512;
constexpr int NWC = NC / 64;

// Sums over one wave of NV complex values (valid in every lane); the
// butterfly steps of all values interleaved.
template <int NV>
__device__ __forceinline__ void wave_sums(c128 (&v)[NV]) {
  double r[2 * NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    r[2 * q] = v[q].re;
    r[2 * q + 1] = v[q].im;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int q = 0; q < 2 * NV; ++q) r[q] += __shfl_xor(r[q], off, 64);
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = mk(r[2 * q], r[2 * q + 1]);
}

// Orders the LDS accesses of one wave (its lanes run in lockstep and its LDS
// operations complete in order; this keeps the compiler from moving them).
__device__ __forceinline__ void wave_lds_order() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int S>
__global__ void __launch_bounds__(NC) k_coefs(const c128* __restrict__ d, c128* __restrict__ H,
                                              int ld, int j, c128* __restrict__ coef, int cld,
                                              c128* __restrict__ Hh, Batch z) {
  __shared__ c128 Dl[S * kCoefMax];             // pass A's dots
  __shared__ c128 Q[S][kCoefMax];               // q_{j+1}.. (t < S - 1) and the last w
  __shared__ c128 Gw[kCoefMax];                 // G w (rows < m)
  __shared__ c128 part[NWC][kCoefMax];          // per-wave partial rows of H p
  HM_MEMBER(d); HM_MEMBER(H); HM_MEMBER(coef);
  Hh = at_member(Hh, z.hz, z);
  const int m = j + 1, nb = m + S, tid = threadIdx.x, lane = tid & 63;
  const bool w0 = tid < 64;
  for (int i = tid; i < S * nb; i += NC) Dl[i] = d[i];
  __syncthreads();
  auto VY = [&](int i, int k) { return Dl[k * nb + i]; };        // V_i^H Y_k
  auto YY = [&](int k, int l) { return Dl[l * nb + m + k]; };    // Y_k^H Y_l
  // (wave 0) G P into Gw (rows < m, lane-owned) and gy (rows m.., every lane),
  // with out[s] = <L_s, P>_G for the NL coordinate rows L_s
  auto gram_dots = [&](const c128* P, auto& out, const c128* const* L, c128 (&gy)[S]) {
    constexpr int NL = sizeof(out) / sizeof(c128);
    c128 v[S + NL];
#pragma unroll
    for (int q = 0; q < S + NL; ++q) v[q] = mk(0.0, 0.0);
    for (int i = lane; i < m; i += 64) {
      c128 g = P[i];
      const c128 pi = P[i];
#pragma unroll
      for (int k = 0; k < S; ++k) {
        const c128 vy = VY(i, k);
        g = g + vy * P[m + k];
        v[k] = v[k] + cmulc(vy, pi);
      }
      Gw[i] = g;
#pragma unroll
      for (int s2 = 0; s2 < NL; ++s2) v[S + s2] = v[S + s2] + cmulc(L[s2][i], g);
    }
    wave_sums<S + NL>(v);
#pragma unroll
    for (int k = 0; k < S; ++k) {
      c128 g = v[k];
#pragma unroll
      for (int l = 0; l < S; ++l) g = g + YY(k, l) * P[m + l];
      gy[k] = g;
    }
#pragma unroll
    for (int s2 = 0; s2 < NL; ++s2) {
      c128 o = v[S + s2];
#pragma unroll
      for (int k = 0; k < S; ++k) o = o + cmulc(L[s2][m + k], gy[k]);
      out[s2] = o;
    }
  };
  // (every wave) rows < m of M P, sum_{i = max(0, r-1)}^{j-1} H[r, i] P_i, into
  // out.  The work is the (row band of 64, column) pairs whose column reaches
  // the band, in band-major order, split evenly over the waves; a wave reads
  // one column of a band per load (coalesced), sixteen loads in flight, and
  // stores its sum for a band into its own partial row; the partials are
  // added in wave order (the result does not depend on timing).
  auto h_product = [&](const c128* P, c128* out) {
    const int nbands = (m + 63) >> 6;
    auto lo = [&](int bb) { return bb > 0 ? 64 * bb - 1 : 0; };
    int T = 0;
    for (int bb = 0; bb < nbands; ++bb) T += j > lo(bb) ? j - lo(bb) : 0;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    c128* mine = part[wv];
    for (int r = lane; r < m; r += 64) mine[r] = mk(0.0, 0.0);
    const int beg = (int)((long long)T * wv / NWC), end = (int)((long long)T * (wv + 1) / NWC);
    int b = 0, i = 0, rem = beg;
    for (; b < nbands; ++b) {
      const int len = j > lo(b) ? j - lo(b) : 0;
      if (rem < len) {
        i = lo(b) + rem;
        break;
      }
      rem -= len;
    }
    int bcur = b;
    c128 acc = mk(0.0, 0.0);
    auto flush = [&](int bb) {
      const int r = 64 * bb + lane;
      if (r < m) mine[r] = acc;                // each band once per wave
    };
    for (int cnt = end - beg; cnt > 0; cnt -= 16) {
      c128 hv[16];
      int bq[16], iq[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        bq[q] = b;
        iq[q] = i;
        const int r = 64 * b + lane;
        hv[q] = (q < cnt && r < m && i + 1 >= r) ? H[(size_t)i * ld + r] : mk(0.0, 0.0);
        if (q < cnt && ++i == j) {
          ++b;
          i = lo(b);
        }
      }
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        if (q < cnt) {
          if (bq[q] != bcur) {
            flush(bcur);
            acc = mk(0.0, 0.0);
            bcur = bq[q];
          }
          acc = acc + hv[q] * P[iq[q]];
        }
      }
    }
    if (end > beg) flush(bcur);
    __syncthreads();
    if (w0)
      for (int r = lane; r < m; r += 64) {
        c128 g = part[0][r];
        for (int w = 1; w < NWC; ++w) g = g + part[w][r];
        out[r] = g;
      }
  };
  c128* W = Q[S - 1];                           // w of the current step (last row reused)
#pragma unroll 1
  for (int t = 0; t < S; ++t) {
    // w = M q_{j+t}
    if (t > 0) {
      __syncthreads();                          // q_{j+t} (wave 0) for every wave
      h_product(Q[t - 1], W);                   // W is not Q[t - 1] (t - 1 < S - 1)
    }
    if (!w0) continue;
    if (t == 0) {
      for (int i = lane; i < nb; i += 64) W[i] = mk(i == m ? 1.0 : 0.0, 0.0);
    } else {
      const c128* P = Q[t - 1];                 // its last Y coordinate is 0
      for (int i = lane; i < nb; i += 64)
        if (i >= m) W[i] = i == m ? P[j] : P[i - 1];
    }
    wave_lds_order();
    // h: <e_l, w>_G = (G w)_l for l <= j; <q_{j+1+s}, w>_G for s < t
    c128 gy[S];
    c128 hs[S > 1 ? S - 1 : 1];
    const c128* L[S > 1 ? S - 1 : 1];
#pragma unroll
    for (int s2 = 0; s2 < (S > 1 ? S - 1 : 1); ++s2) {
      L[s2] = Q[s2];
      hs[s2] = mk(0.0, 0.0);
    }
    if (t == 0) {
      c128 none[1];
      const c128* L0[1] = {W};
      gram_dots(W, none, L0, gy);               // (the dot is not used)
    } else if (S >= 2 && t == 1) {
      c128 h1[1];
      gram_dots(W, h1, L, gy);
      hs[0] = h1[0];
    } else if (S >= 3 && t == 2) {
      c128 h2[2];
      gram_dots(W, h2, L, gy);
      hs[0] = h2[0];
      hs[1] = h2[1];
    }
    c128* col = H + (size_t)(j + t) * ld;
    c128* hcol = Hh + (size_t)(j + t) * ld;
    for (int l = lane; l <= j; l += 64) {
      col[l] = Gw[l];
      hcol[l] = Gw[l];
    }
    if (lane == 0) {
#pragma unroll
      for (int s2 = 0; s2 < t; ++s2) {
        col[j + 1 + s2] = hs[s2];
        hcol[j + 1 + s2] = hs[s2];
      }
    }
    wave_lds_order();                           // w's Y part read by every lane
    // w -= sum_l h_l q_l (the e_l part first, then the earlier q's)
    for (int i = lane; i < nb; i += 64) {
      c128 v = W[i];
      if (i <= j) v = v - Gw[i];
#pragma unroll
      for (int s2 = 0; s2 < t; ++s2) v = v - hs[s2] * Q[s2][i];
      W[i] = v;
    }
    wave_lds_order();
    if (t + 1 < S) {
      c128 ww[1];
      const c128* LW[1] = {W};
      gram_dots(W, ww, LW, gy);
      const double bt = ww[0].re > 0 ? sqrt(ww[0].re) : 0.0, ib = 1.0 / bt;
      if (lane == 0) {
        col[j + t + 1] = mk(bt, 0.0);
        hcol[j + t + 1] = mk(bt, 0.0);
      }
      for (int i = lane; i < nb; i += 64) Q[t][i] = ib * W[i];
      wave_lds_order();
    }
  }
  // pass B's rows (wave 0): q_{j+1}..q_{j+S-1}, then the last w
  if (w0)
    for (int t = 0; t < S; ++t)
      for (int i = lane; i < nb; i += 64) coef[(size_t)t * cld + i] = Q[t][i];
}

// Pass A of S Arnoldi steps and its final sums: out[r (m + S) + i].
template <typename T>
hipError_t launch_multidots(int S, const cx<T>* V, size_t ldv, int m, const cx<T>* y0,
                            const cx<T>* y1, const cx<T>* y2, size_t n, RedBuf rb, c128* out,
                            hipStream_t s, const Batch& z, const CachePolicy& cp) {
  if (m <= 0 || S < 1 || S > 3) return hipErrorInvalidValue;
  const int ngroups = (m + GP - 1) / GP + (S + GP - 1) / GP;
  const bool st = (double)(m + 1) * (double)n * sizeof(cx<T>) > cp.basis;
  // resident blocks of the plain-load instance for both load forms, so the
  // chunks (and the sums) do not depend on the load form
  static int resident[4] = {};
  int& res = resident[S];
  if (res == 0) {
    int dev = 0, ncu = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    const void* fn = S == 1   ? (const void*)k_multidots<T, false, 1>
                     : S == 2 ? (const void*)k_multidots<T, false, 2>
                              : (const void*)k_multidots<T, false, 3>;
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, NT, 0);
    if (e != hipSuccess) return e;
    res = std::max(8, per_cu * ncu);
  }
  // chunks: whole rounds of the resident blocks (a partial last round leaves
  // most of the device idle while it runs), as few rounds as keep the Y chunks
  // of the blocks resident on one XCD within about 3 MB of its 4 MB L2 (every
  // group of a chunk re-reads them).  On the 1150 x 364 coarsest level of the
  // 4597 x 1453 layered problem 1.8 rounds became one (967 -> 918 ms per
  // solve); the 4097^2 problem is unchanged.  The chunks do not depend on the
  // number of batch members, so a member's sums are those of its solve alone.
  const int slots = res;
  const double ybytes = (double)S * sizeof(cx<T>);
  const double nmin = (double)n * ybytes * slots / (8.0 * ngroups * 3.0e6);
  const int rounds = std::max(1, (int)std::ceil(ngroups * nmin / slots));
  int target = std::max(8, (int)((long long)rounds * slots / ngroups) / 8 * 8);
  size_t clen = (n + target - 1) / target;
  clen = (clen + 63) / 64 * 64;
  while ((n + clen - 1) / clen > (size_t)kMaxChunks) clen += 64;
  const int nch = (int)(((n + clen - 1) / clen + 7) & ~(size_t)7);
  const dim3 g = zgrid(ngroups * nch, z);
  const int recent = (int)(cp.recent / ((double)n * sizeof(cx<T>)));
#define HM_MD(SS)                                                                                 \
  if (st) k_multidots<T, true, SS><<<g, NT, 0, s>>>(V, ldv, m, y0, y1, y2, n, clen, rb.partials, \
                                                    nch, recent, z);                           \
  else k_multidots<T, false, SS><<<g, NT, 0, s>>>(V, ldv, m, y0, y1, y2, n, clen, rb.partials,  \
                                                  nch, recent, z);
  if (S == 1) { HM_MD(1) } else if (S == 2) { HM_MD(2) } else { HM_MD(3) }
#undef HM_MD
  k_final<<<zgrid(S * (m + S), z), NT, 0, s>>>(rb.partials, nch, out, 0, nullptr, z);
  return hipGetLastError();
}

// Pass B of S Arnoldi steps and the norm of the new Y_0 (sqrt to norm_out and
// the pinned host_out).
template <typename T>
hipError_t launch_updates(int S, cx<T>* y0, const cx<T>* y1, const cx<T>* y2, cx<T>* V,
                          size_t ldv, int m, const c128* coef, int cld, size_t n, RedBuf rb,
                          c128* norm_out, c128* host_out, hipStream_t s, const Batch& z,
                          const CachePolicy& cp) {
  if (S < 1 || S > 3) return hipErrorInvalidValue;
  const int nch = update_chunks(n, rb);
  const size_t clen = update_chunk_len(n);
  const int recent = (int)(cp.recent / ((double)n * sizeof(cx<T>)));
  const dim3 g = zgrid(nch, z);
  const bool st = (double)(m + 1) * (double)n * sizeof(cx<T>) > cp.basis;
#define HM_UP(SS)                                                                                \
  if (st) k_updates<T, true, SS><<<g, NT, 0, s>>>(y0, y1, y2, V, ldv, m, coef, cld, n, clen,    \
                                                  rb.partials, recent, z);                     \
  else k_updates<T, false, SS><<<g, NT, 0, s>>>(y0, y1, y2, V, ldv, m, coef, cld, n, clen,      \
                                                rb.partials, recent, z);
  if (S == 1) { HM_UP(1) } else if (S == 2) { HM_UP(2) } else { HM_UP(3) }
#undef HM_UP
  k_final<<<zgrid(1, z), NT, 0, s>>>(rb.partials, nch, norm_out, 1, host_out, z);
  return hipGetLastError();
}

int coefs_max_basis() { return kCoefMax; }

hipError_t launch_coefs(int S, const c128* dots, c128* H, int ld, int j, c128* coef, int cld,
                        c128* host_H, hipStream_t s, const Batch& z) {
  if (j + 1 + S > kCoefMax) return hipErrorInvalidValue;
  if (S == 1) k_coefs<1><<<zgrid(1, z), NC, 0, s>>>(dots, H, ld, j, coef, cld, host_H, z);
  else if (S == 2) k_coefs<2><<<zgrid(1, z), NC, 0, s>>>(dots, H, ld, j, coef, cld, host_H, z);
  else if (S == 3) k_coefs<3><<<zgrid(1, z), NC, 0, s>>>(dots, H, ld, j, coef, cld, host_H, z);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cgs_update_norm(cx<T>* w, const cx<T>* V, size_t ldv, int m, const c128* h,
                                  size_t n, RedBuf rb, c128* out, hipStream_t s) {
  const hipError_t e = launch_cgs_update_partial<T>(w, V, ldv, m, h, n, rb, s);
  if (e != hipSuccess) return e;
  return launch_update_norm_final(n, rb, out, s);
}

template <typename T>
hipError_t launch_norm(const cx<T>* x, size_t n, RedBuf rb, c128* out, hipStream_t s,
                       c128* host_out, const Batch& z) {
  const size_t clen = chunk_len(n, rb.nchunks);
  k_norm2<T><<<zgrid(rb.nchunks, z), NT, 0, s>>>(x, n, clen, rb.partials, z);
  k_final<<<zgrid(1, z), NT, 0, s>>>(rb.partials, rb.nchunks, out, 1, host_out, z);
  return hipGetLastError();
}

hipError_t launch_max_real(const double* a, size_t n, RedBuf rb, c128* out, hipStream_t s) {
  const size_t clen = chunk_len(n, rb.nchunks);
  k_max_partial<<<rb.nchunks, NT, 0, s>>>(a, n, clen, rb.partials);
  k_max_final<<<1, 64, 0, s>>>(rb.partials, rb.nchunks, out);
  return hipGetLastError();
}

size_t small_gmres_lds(int nx, int ny, int R, size_t es, size_t ks, int cap) {
  const size_t ldh = (size_t)cap + 2;
  const size_t level = (size_t)(nx + 2 * R) * (ny + 2 * R) * (es + ks);
  const size_t tri = (size_t)cap * cap * sizeof(c128);   // reuses the level's area at the end
  return sizeof(double) * (2 * SG_G * (SG_WAVES + 1) + 4) + 3 * ldh * sizeof(c128) +
         ((ldh + 1) & ~(size_t)1) * sizeof(double) + (level > tri ? level : tri);
}

template <typename T>
bool small_gmres_fits(const OpDesc<T>& d, int cap) {
  static int lds_max = -1;                     // per device type; the same on every call
  if (lds_max < 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      v = 0;
    lds_max = v;
  }
  return d.R >= 1 && d.R <= 3 && cap + 2 <= SmallGmresArgs::kMaxLdh &&
         (long)d.nx * d.ny <= SmallGmresArgs::kMaxNodes &&
         small_gmres_lds(d.nx, d.ny, d.R, sizeof(cx<T>), sizeof(T), cap) <= (size_t)lds_max;
}

template <typename T, int R>
static hipError_t launch_gmres_small_r(const OpDesc<T>& d, const T* k, const cx<T>* b, cx<T>* x,
                                       cx<T>* V, cx<T>* w, c128* H, const SmallGmresArgs& ga,
                                       c128* info, hipStream_t s, const Batch& z) {
  const size_t lds = small_gmres_lds(d.nx, d.ny, R, sizeof(cx<T>), sizeof(T), ga.ldh - 2);
  static size_t granted = 0;                   // dynamic LDS limit raised for this kernel
  if (lds > granted) {
    const hipError_t e = hipFuncSetAttribute((const void*)k_gmres_small<T, R>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    granted = lds;
  }
  k_gmres_small<T, R><<<zgrid(1, z), SG_NT, lds, s>>>(d, k, b, x, V, w, H, ga, info, z);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gmres_small(const OpDesc<T>& d, const T* k, const cx<T>* b, cx<T>* x, cx<T>* V,
                              cx<T>* w, c128* H, const SmallGmresArgs& ga, c128* info,
                              hipStream_t s, const Batch& z) {
  if (d.R == 1) return launch_gmres_small_r<T, 1>(d, k, b, x, V, w, H, ga, info, s, z);
  if (d.R == 2) return launch_gmres_small_r<T, 2>(d, k, b, x, V, w, H, ga, info, s, z);
  if (d.R == 3) return launch_gmres_small_r<T, 3>(d, k, b, x, V, w, H, ga, info, s, z);
  return hipErrorInvalidValue;
}

hipError_t launch_residual_norm(const OpDesc<double>& d, const c128* u, const double* k,
                                const c128* b, c128* r, c128* partials, double* norms,
                                hipStream_t s) {
  const size_t n = (size_t)d.nx * d.ny;
  const int nch = reduction_chunks(n);
  const size_t clen = chunk_len(n, nch);
  k_residual_norm<<<nch, NT, 0, s>>>(d, u, k, b, r, n, clen, partials);
  k_residual_final<<<1, NT, 0, s>>>(partials, nch, norms);
  return hipGetLastError();
}

hipError_t scratch_address(c128** ptr, size_t* bytes) {
  static std::mutex mu;
  static std::vector<c128*> addr;                // by device ordinal
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(mu);
  if ((size_t)dev >= addr.size()) addr.resize((size_t)dev + 1, nullptr);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = (c128*)p;
  }
  *ptr = addr[dev];
  *bytes = sizeof(scratch);
  return hipSuccess;
}

hipError_t launch_check_k(const double* k, size_t n, RedBuf rb, c128* out, hipStream_t s) {
  const size_t clen = chunk_len(n, rb.nchunks);
  k_check_k<<<rb.nchunks, NT, 0, s>>>(k, n, clen, rb.partials);
  k_final<<<1, NT, 0, s>>>(rb.partials, rb.nchunks, out, 0, nullptr, Batch());
  return hipGetLastError();
}

// ---- explicit instantiations ----------------------------------------------------
#define HM_INST_T(T)                                                                              \
  template hipError_t launch_stencil<T>(const OpDesc<T>&, int, const cx<T>*, const T*,              \
                                        const cx<T>*, cx<T>*, T, hipStream_t, const Batch&);         \
  template hipError_t launch_jacobi0<T>(const OpDesc<T>&, const T*, const cx<T>*, cx<T>*, T,         \
                                        hipStream_t, const Batch&);                                 \
  template hipError_t launch_restrict_fw<T>(const cx<T>*, int, int, cx<T>*, int, hipStream_t,      \
                                            const Batch&);                                          \
  template hipError_t launch_prolong_bilinear_add<T>(const cx<T>*, int, int, cx<T>*, int,         \
                                                     hipStream_t, const Batch&);                    \
  template hipError_t launch_add<T>(const cx<T>*, const cx<T>*, cx<T>*, size_t, hipStream_t,       \
                                    const Batch&);                                                  \
  template hipError_t launch_scale_dev<T>(const cx<T>*, cx<T>*, const c128*, int, size_t,          \
                                          hipStream_t, const Batch&);                               \
  template hipError_t launch_zero<T>(cx<T>*, size_t, hipStream_t, const Batch&);                   \
  template hipError_t launch_dense_matvec<T>(const c128*, int, const cx<T>*, cx<T>*, hipStream_t,  \
                                             const Batch&);                                         \
  template hipError_t launch_combine<T>(const cx<T>*, size_t, int, const c128*, size_t, double,    \
                                        cx<T>*, int, size_t, hipStream_t, const Batch&);            \
  template hipError_t launch_multidot<T>(const cx<T>*, size_t, int, const cx<T>*, size_t, RedBuf,  \
                                         c128*, hipStream_t);                                       \
  template hipError_t launch_multidot_partial<T>(const cx<T>*, size_t, int, const cx<T>*, size_t,  \
                                                 RedBuf, hipStream_t, const Batch&,                 \
                                                 const CachePolicy&);                               \
  template hipError_t launch_multidot_final<T>(int, size_t, RedBuf, c128*, hipStream_t, c128*,     \
                                               const Batch&);                                       \
  template hipError_t launch_cgs_update_partial<T>(cx<T>*, const cx<T>*, size_t, int, const c128*, \
                                                   size_t, RedBuf, hipStream_t, const Batch&,       \
                                                   const CachePolicy&);                             \
  template hipError_t launch_multidots<T>(int, const cx<T>*, size_t, int, const cx<T>*,            \
                                          const cx<T>*, const cx<T>*, size_t, RedBuf, c128*,        \
                                          hipStream_t, const Batch&, const CachePolicy&);          \
  template hipError_t launch_updates<T>(int, cx<T>*, const cx<T>*, const cx<T>*, cx<T>*, size_t,   \
                                        int, const c128*, int, size_t, RedBuf, c128*, c128*,        \
                                        hipStream_t, const Batch&, const CachePolicy&);            \
  template hipError_t launch_stencil_scaled<T>(const OpDesc<T>&, const cx<T>*, const T*,            \
                                               const c128*, cx<T>*, cx<T>*, hipStream_t,            \
                                               const Batch&);                                       \
  template hipError_t launch_mgs_step<T>(cx<T>*, const cx<T>*, const c128*, const cx<T>*, size_t,  \
                                         RedBuf, c128*, hipStream_t, c128*, const Batch&);          \
  template hipError_t launch_cgs_update_norm<T>(cx<T>*, const cx<T>*, size_t, int, const c128*,    \
                                                size_t, RedBuf, c128*, hipStream_t);                \
  template hipError_t launch_norm<T>(const cx<T>*, size_t, RedBuf, c128*, hipStream_t, c128*,      \
                                     const Batch&);                                                 \
  template bool small_gmres_fits<T>(const OpDesc<T>&, int);                                        \
  template hipError_t launch_gmres_small<T>(const OpDesc<T>&, const T*, const cx<T>*, cx<T>*,       \
                                            cx<T>*, cx<T>*, c128*, const SmallGmresArgs&, c128*,    \
                                            hipStream_t, const Batch&);
HM_INST_T(float)
HM_INST_T(double)
#undef HM_INST_T

#define HM_INST_2(A, B)                                                                          \
  template hipError_t launch_restrict_z<A, B>(const cx<A>*, int, int, cx<B>*, int, hipStream_t,  \
                                              const Batch&);                                     \
  template hipError_t launch_prolong_z<A, B>(const cx<A>*, int, int, cx<B>*, int, hipStream_t,   \
                                             const Batch&);                                      \
  template hipError_t launch_inject<A, B>(const A*, int, int, B*, hipStream_t);                 \
  template hipError_t launch_convert_real<A, B>(const A*, B*, size_t, hipStream_t);             \
  template hipError_t launch_convert<A, B>(const cx<A>*, cx<B>*, size_t, hipStream_t,           \
                                           const Batch&);
HM_INST_2(float, float)
HM_INST_2(double, double)
HM_INST_2(float, double)
HM_INST_2(double, float)
#undef HM_INST_2

}  // namespace hm
