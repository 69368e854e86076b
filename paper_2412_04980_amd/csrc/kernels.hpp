// Host-side launchers of the HIP kernels of the MADP library (gfx950).
// Every launcher enqueues on the given stream and returns hipSuccess or the
// launch error; none synchronises.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>

#include "cplx.hpp"

namespace hm {

// Description of one grid operator (Sec. 2.1 / 3.3):
//   R = 1: five-point rows everywhere:
//          scale * ( inv_H2 (4u - sum of 4 neighbours) - sigma k^2 u )
//   R = 2, 3: re-discretised (2R+1)^2 stencil on non-boundary rows
//          sum_{a,b} ( L[b][a] - sigma K[b][a] k^2_{p} ) u_p
//          and the five-point row above on boundary nodes.
// Points outside the grid take the Sommerfeld ghost value
// u_m + i two_H k_b u_b (one step out in exactly one direction, wavenumber 0)
// or zero (further out, or out in both directions).
template <typename T>
struct OpDesc {
  int nx, ny;
  int R;
  T inv_H2;   // 1 / H^2 of the five-point rows
  T two_H;    // 2 H of the ghost term
  T scale;    // s_l of the five-point rows
  T sig_re, sig_im;
  T L[49];    // (2R+1)^2 Laplace coefficients, already divided by h^2 (finest h)
  T K[49];    // (2R+1)^2 wavenumber coefficients
  // 1-D factors: L[b][a] = t[a] m[b] + m[a] t[b] (t already divided by h^2),
  // K[b][a] = m[a] m[b]
  T t1[7];
  T m1[7];
  int bc;     // 0 Sommerfeld ghosts, 1 homogeneous Dirichlet (boundary rows d_b u_b)
};

enum StencilMode { ST_APPLY = 0, ST_RESID = 1, ST_JACOBI = 2 };

// Members of a lockstep batch: problems with the same layout whose device
// buffers lie dz bytes apart (member i at member 0 + i * dz) and whose pinned
// host staging lies hz bytes apart.  A launch covers the n members listed in
// slot (grid z, block z works on member slot[z]); every pointer a launcher
// takes is member 0's.  The default is the single problem (n = 1, slot 0).
constexpr int kMaxBatch = 16;
struct Batch {
  long long dz = 0;
  long long hz = 0;
  int n = 1;
  unsigned char slot[kMaxBatch] = {};
  int cnt[kMaxBatch] = {};   // per-member counts (launch_combine with m < 0)
  // per-member damping weights of the Jacobi sweeps (they follow each member's
  // wavenumber); used instead of the omega argument when use_omega is set
  int use_omega = 0;
  double omega[kMaxBatch] = {};
};

// out = Op(u)                         (ST_APPLY, b unused)
// out = b - Op(u)                     (ST_RESID)
// out = u + omega D^-1 (b - Op(u))    (ST_JACOBI, D = diagonal of Op)
template <typename T>
hipError_t launch_stencil(const OpDesc<T>& d, int mode, const cx<T>* u, const T* k, const cx<T>* b,
                          cx<T>* out, T omega, hipStream_t s, const Batch& z = Batch());

// Scaled apply for Krylov steps: with s = 1 / scal[0].re,
//   vout = s u   and   out = Op(s u)
// (normalises the new basis vector and applies the operator in one pass).
template <typename T>
hipError_t launch_stencil_scaled(const OpDesc<T>& d, const cx<T>* u, const T* k, const c128* scal,
                                 cx<T>* vout, cx<T>* out, hipStream_t s, const Batch& z = Batch());

// x = omega D^-1 b  (first damped-Jacobi sweep from x = 0)
template <typename T>
hipError_t launch_jacobi0(const OpDesc<T>& d, const T* k, const cx<T>* b, cx<T>* x, T omega,
                          hipStream_t s, const Batch& z = Batch());

// Transfers take dir = 1 for Dirichlet boundaries: boundary values of the input
// count as zero and boundary values of the output are zero (interior masks on
// both sides); dir = 0 for Sommerfeld.
// Deflation restriction Z^T: fine (nxf x nyf) -> coarse; weights p (x) p,
// p = [1 4 6 4 1]/8 at fine offsets -2..2 around 2J; outside values zero.
template <typename Ti, typename To>
hipError_t launch_restrict_z(const cx<Ti>* f, int nxf, int nyf, cx<To>* c, int dir, hipStream_t s,
                             const Batch& z = Batch());
// Deflation interpolation Z: coarse -> fine (transpose of the above).
template <typename Ti, typename To>
hipError_t launch_prolong_z(const cx<Ti>* c, int nxf, int nyf, cx<To>* f, int dir, hipStream_t s,
                            const Batch& z = Batch());

// Full-weighting restriction (1/16)[1 2 1;2 4 2;1 2 1], fine -> coarse.
template <typename T>
hipError_t launch_restrict_fw(const cx<T>* f, int nxf, int nyf, cx<T>* c, int dir, hipStream_t s,
                              const Batch& z = Batch());
// x_fine += bilinear interpolation of e_coarse.
template <typename T>
hipError_t launch_prolong_bilinear_add(const cx<T>* c, int nxf, int nyf, cx<T>* f, int dir,
                                       hipStream_t s, const Batch& z = Batch());
// Injection of a real nodal field: c(J) = f(2J).
template <typename Ti, typename To>
hipError_t launch_inject(const Ti* f, int nxf, int nyf, To* c, hipStream_t s);
// Real-field conversion.
template <typename Ti, typename To>
hipError_t launch_convert_real(const Ti* a, To* b, size_t n, hipStream_t s);

// ---- vector kernels ------------------------------------------------------
template <typename Ti, typename To>
hipError_t launch_convert(const cx<Ti>* a, cx<To>* b, size_t n, hipStream_t s,
                          const Batch& z = Batch());
template <typename T>
hipError_t launch_add(const cx<T>* a, const cx<T>* b, cx<T>* out, size_t n, hipStream_t s,
                      const Batch& z = Batch());  // out = a + b
// y = scal[0] * x  (scal on the device; `inv` = use 1/scal[0].re instead)
template <typename T>
hipError_t launch_scale_dev(const cx<T>* x, cx<T>* y, const c128* scal, int inv, size_t n,
                            hipStream_t s, const Batch& z = Batch());
template <typename T>
hipError_t launch_zero(cx<T>* x, size_t n, hipStream_t s, const Batch& z = Batch());
// out = (accumulate ? out : 0) + sign * sum_{i<m} coef[i] * V_i  (coef on the device).
// In a batch the coefficients of member slot s start at coef + s * coef_ld (they
// are not in the members' workspaces) and m < 0 takes member z's count z.cnt[z].
template <typename T>
hipError_t launch_combine(const cx<T>* V, size_t ldv, int m, const c128* coef, size_t coef_ld,
                          double sign, cx<T>* out, int accumulate, size_t n, hipStream_t s,
                          const Batch& z = Batch());

// y = A x with A a dense n x n row-major complex128 matrix (coarsest multigrid
// solve, FP64 in every precision; x widened, y rounded to T)
template <typename T>
hipError_t launch_dense_matvec(const c128* A, int n, const cx<T>* x, cx<T>* y, hipStream_t s,
                               const Batch& z = Batch());
// out = unit vectors: out[j*n + i] = (i == j)
hipError_t launch_identity(c128* out, int n, hipStream_t s);

// ---- stored-matrix comparison (CSR) ---------------------------------------
// CSR of the five-point operator d (R = 1) with exactly five entries per row in
// the order centre, west, east, south, north; a neighbour outside the grid
// contributes through its mirror (Sommerfeld ghost), its own slot holds a zero
// pointing at the row itself.
hipError_t launch_csr5_assemble(const OpDesc<double>& d, const double* k, int* rowptr, int* colidx,
                                c128* vals, hipStream_t s);
// y = A x for a CSR matrix with nrows rows and ncols columns (x has ncols
// entries; a column index outside [0, ncols) makes its row NaN)
hipError_t launch_csr_spmv(int nrows, int ncols, const int* rowptr, const int* colidx,
                           const c128* vals, const c128* x, c128* y, hipStream_t s);

// ---- small coarse levels: a whole GMRES solve in one workgroup per member ---
// Parameters of one launch: member z (grid z) runs at most maxit[z] steps and
// stops after step j when the Givens estimate |g_{j+1}| <= tol[z] ||b|| (tol < 0:
// exactly maxit steps) or on breakdown; modified Gram-Schmidt if mgs.  ldh is
// the column stride of the device Hessenberg H (cap + 2).
struct SmallGmresArgs {
  static constexpr int kMaxLdh = 512;
  // Largest level (nodes) taken by the one-workgroup solve.  One compute unit
  // streams the basis, so the cost per step grows with the level while the
  // host-driven steps spread over the device: measured per solve, the 33 x 33
  // level of the 129^2 problem gains (12.0 -> 10.6 ms), the 65 x 65 level of a
  // 257^2 problem loses (54 -> 99 ms), and so does a 76 x 126 multigrid coarsest
  // grid in FP32.
  static constexpr int kMaxNodes = 1600;
  int ldh = 0;
  int mgs = 0;
  int maxit[kMaxBatch] = {};
  double tol[kMaxBatch] = {};
};
// True when the level (operator d, basis capacity cap) is taken by the
// one-workgroup solve: at most kMaxNodes nodes, its ghost-extended copy in LDS.
template <typename T>
bool small_gmres_fits(const OpDesc<T>& d, int cap);
// GMRES from x = 0 on d (wavenumber k) for the right-hand side b, basis V of
// (cap+1) x N, work vector w (N), Hessenberg H; writes x and, in info[0] (pinned host memory of
// each member, hz apart), (steps, final estimate / ||b||), or (0, ||b||) when no
// step was taken.
template <typename T>
hipError_t launch_gmres_small(const OpDesc<T>& d, const T* k, const cx<T>* b, cx<T>* x, cx<T>* V,
                              cx<T>* w, c128* H, const SmallGmresArgs& ga, c128* info,
                              hipStream_t s, const Batch& z = Batch());

// ---- reductions (double accumulation; results on the device) --------------
struct RedBuf {
  c128* partials;   // >= kMaxChunks * (max dots) entries
  int nchunks;
};
constexpr int kMaxChunks = 2048;
int reduction_chunks(size_t n);

// out[i] = (V_i, w) = sum conj(V_i) w, i = 0..m-1.  Split in two launches
// (partial sums over chunks of the vector, then the sums of the partials) so
// that the streaming kernel can be timed on its own.  A basis (plus w) up to
// kCacheBasisBytes is read with plain loads in both Gram-Schmidt passes, which
// leave it in the 256 MB Infinity Cache for the other pass and the next step.  A
// larger one keeps only its most recent vectors, kCacheRecentBytes of them,
// cache-resident that way; the older ones are read with the non-temporal hint.
constexpr double kCacheBasisBytes = 256.0 * 1048576.0;
constexpr double kCacheRecentBytes = 200.0 * 1048576.0;
// The two thresholds as a run-time setting (a problem may override them; the
// arithmetic is the same for every setting, only the load hints change).
struct CachePolicy {
  double basis = kCacheBasisBytes;
  double recent = kCacheRecentBytes;
};
template <typename T>
hipError_t launch_multidot_partial(const cx<T>* V, size_t ldv, int m, const cx<T>* w, size_t n,
                                   RedBuf rb, hipStream_t s, const Batch& z = Batch(),
                                   const CachePolicy& cp = CachePolicy());
// host_out (optional): pinned host memory that receives a copy of out
template <typename T>
hipError_t launch_multidot_final(int m, size_t n, RedBuf rb, c128* out, hipStream_t s,
                                 c128* host_out = nullptr, const Batch& z = Batch());
template <typename T>
hipError_t launch_multidot(const cx<T>* V, size_t ldv, int m, const cx<T>* w, size_t n, RedBuf rb,
                           c128* out, hipStream_t s);
// Modified Gram-Schmidt step: if (prev) w -= hprev[0] * prev;  out[0] = (next, w)
// If next == nullptr: out[0] = ||w||_2 (real part).  host_out as for the multi-dot.
template <typename T>
hipError_t launch_mgs_step(cx<T>* w, const cx<T>* prev, const c128* hprev, const cx<T>* next,
                           size_t n, RedBuf rb, c128* out, hipStream_t s,
                           c128* host_out = nullptr, const Batch& z = Batch());
// Classical Gram-Schmidt update fused with the norm: w -= sum_{i<m} h[i] V_i ; out[0] = ||w||
template <typename T>
hipError_t launch_cgs_update_partial(cx<T>* w, const cx<T>* V, size_t ldv, int m, const c128* h,
                                     size_t n, RedBuf rb, hipStream_t s,
                                     const Batch& z = Batch(),
                                     const CachePolicy& cp = CachePolicy());
// S Arnoldi steps per pair of passes over the basis (S = 1, 2, 3; Y_0 = M v_j,
// Y_{k+1} = M Y_k).  Pass A: out[r (m + S) + i] = (left i)^H Y_r for the left
// vectors V_0..V_{m-1}, Y_0..Y_{S-1}; needs S (m + S) kMaxChunks partials.
template <typename T>
hipError_t launch_multidots(int S, const cx<T>* V, size_t ldv, int m, const cx<T>* y0,
                            const cx<T>* y1, const cx<T>* y2, size_t n, RedBuf rb, c128* out,
                            hipStream_t s, const Batch& z = Batch(),
                            const CachePolicy& cp = CachePolicy());
// Between the passes (one block per member): Arnoldi in the coordinates of
// [V_0..V_j, Y] from pass A's dots; columns j..j+S-1 of H (stride ld) and of
// the pinned host_H, except the last subdiagonal entry; pass B's coefficient
// rows at coef, cld apart.  j + 1 + S <= coefs_max_basis().
int coefs_max_basis();
hipError_t launch_coefs(int S, const c128* dots, c128* H, int ld, int j, c128* coef, int cld,
                        c128* host_H, hipStream_t s, const Batch& z = Batch());
// Pass B: V_{m+t} (t < S - 1) and the new Y_0 from the coefficient rows, with
// norm_out[0] = host_out[0] = ||Y_0|| (real part).
template <typename T>
hipError_t launch_updates(int S, cx<T>* y0, const cx<T>* y1, const cx<T>* y2, cx<T>* V,
                          size_t ldv, int m, const c128* coef, int cld, size_t n, RedBuf rb,
                          c128* norm_out, c128* host_out, hipStream_t s,
                          const Batch& z = Batch(), const CachePolicy& cp = CachePolicy());
// sum of the partials written by launch_cgs_update_partial over a vector of length n
hipError_t launch_update_norm_final(size_t n, RedBuf rb, c128* out, hipStream_t s,
                                    c128* host_out = nullptr, const Batch& z = Batch());
template <typename T>
hipError_t launch_cgs_update_norm(cx<T>* w, const cx<T>* V, size_t ldv, int m, const c128* h,
                                  size_t n, RedBuf rb, c128* out, hipStream_t s);
// out[0] = ||x||_2 (real part); host_out as for the multi-dot
template <typename T>
hipError_t launch_norm(const cx<T>* x, size_t n, RedBuf rb, c128* out, hipStream_t s,
                       c128* host_out = nullptr, const Batch& z = Batch());
// out[0].re = max of a real field (reduction over chunks)
hipError_t launch_max_real(const double* a, size_t n, RedBuf rb, c128* out, hipStream_t s);
// True residual of the five-point operator d (FP64): r = b - A u (r may be
// null), norms[0] = ||r||_2, norms[1] = ||b||_2 on the device.  partials: at
// least reduction_chunks(nx * ny) <= kMaxChunks entries.
hipError_t launch_residual_norm(const OpDesc<double>& d, const c128* u, const double* k,
                                const c128* b, c128* r, c128* partials, double* norms,
                                hipStream_t s);
// Device address and size of the library's static scratch array on the
// current device (looked up once per device with hipGetSymbolAddress).
hipError_t scratch_address(c128** ptr, size_t* bytes);
// Validation of the wavenumber field: out[0] = number of entries that are not
// finite or negative (as a double in the real part).
hipError_t launch_check_k(const double* k, size_t n, RedBuf rb, c128* out, hipStream_t s);

}  // namespace hm
