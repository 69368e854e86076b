// Host orchestration of the MADP preconditioner and FGMRES on the GPU.
//
// The paper's method (Algorithm 1 with the MADP configuration of Sec. 4.4):
//   Prec_l(v): v_hat = Z^T v; v_t ~ E^-1 v_hat (level-2 FGMRES to tolerance
//   0.3, or one FGMRES step with Krylov CSLP on the coarsest level);
//   t = Z v_t; r~ = v - A t; r ~ M^-1 r~ (one V-cycle on levels 1-2, GMRES
//   below); return r + t.
// Outer: FGMRES with modified Gram-Schmidt, restart 30, relative residual
// 1e-6, true residual recomputed in FP64.
//
// Every grid step runs in a HIP kernel (kernels.hip); the host holds only the
// control flow and the small Hessenberg least-squares problems.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <stdexcept>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/helmdefl.h"
#include "kernels.hpp"
#include "lsq.hpp"
#include "tables.hpp"

namespace hm {

struct HipError : std::runtime_error {
  using std::runtime_error::runtime_error;
};
struct ArgError : std::runtime_error {
  using std::runtime_error::runtime_error;
};
// a level-2 solve reached the reserved basis (hm_config.level2_basis)
struct BasisError : std::runtime_error {
  using std::runtime_error::runtime_error;
};

#define HM_CHECK(...)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (__VA_ARGS__);                                                         \
    if (e_ != hipSuccess)                                                                  \
      throw HipError(std::string(#__VA_ARGS__) + ": " + hipGetErrorString(e_));            \
  } while (0)

// ---------------------------------------------------------------------------
// Workspace carving: the same walk computes the size (base == nullptr) and
// assigns the pointers.
struct Carver {
  char* base = nullptr;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

// Krylov workspace of one solver instance (type of its vectors given at use).
struct KrylovWS {
  int cap = 0;
  size_t N = 0;
  void* V = nullptr;   // (cap+1) x N
  void* X = nullptr;   // cap x N  (flexible basis; unused by plain GMRES)
  void* w = nullptr;   // N
  void* w2 = nullptr;  // GMRES: second work vector (ping-pong with w)
  c128* h = nullptr;   // device column / scalars, cap + 2
  c128* H = nullptr;   // GMRES: device Hessenberg, cap columns of stride cap + 2
  void* w3 = nullptr;  // S-step GMRES: third work vector
  c128* D = nullptr;   // S-step GMRES: pass A's dots, 3 (cap + 4)
  c128* C = nullptr;   // S-step GMRES: pass B's coefficient rows, 3 (cap + 4)
};

struct MGLevel {
  int nx = 0, ny = 0;
  size_t N = 0;
  double H = 0, omega = 0;
  OpDesc<double> op64{};
  OpDesc<float> op32{};
  double* k = nullptr; // wavenumber, q >= 1 (q = 0 uses the deflation level's)
  float* k32 = nullptr;
  void* x = nullptr;
  void* y = nullptr;
  void* r = nullptr;
  void* b = nullptr;   // q >= 1
};

struct MGHier {
  std::vector<MGLevel> lv;
  bool dense = false;
  void* inv = nullptr;        // dense inverse of the coarsest operator (level type)
  c128* tmpA = nullptr;       // set-up scratch for the dense inverse (n x n each)
  c128* tmpB = nullptr;
  KrylovWS gm;                // coarsest GMRES otherwise
  int maxit = 0;
  // mixed mode (FP32 levels 1-2): the coarsest GMRES in FP64, like the dense
  // inverse, on cast copies of its right-hand side and solution
  bool gm64 = false;
  void* b64 = nullptr;
  void* x64 = nullptr;
  // with a dense coarsest solve the whole cycle is a fixed kernel sequence on
  // fixed buffers: captured as a HIP graph (input = the level's r~ buffer), one
  // per set of batch members (bit mask) that runs it
  std::vector<std::pair<unsigned, hipGraphExec_t>> graphs;
  const void* graph_out = nullptr;
};

struct DefLevel {
  int l = 0, nx = 0, ny = 0;
  size_t N = 0;
  double hl = 0, sl = 0, kmax = 0;
  bool dbl = true;            // precision of the level's work
  OpDesc<double> A64{}, M64{};
  OpDesc<float> A32{}, M32{};
  double* k64 = nullptr;
  float* k32 = nullptr;
  // this level as a coarse problem (l >= 2): FGMRES workspace, rhs / solution
  KrylovWS fg;
  void* rhs = nullptr;
  void* sol = nullptr;
  // preconditioner temporaries
  void* t = nullptr;
  void* rt = nullptr;
  void* xo = nullptr;
  // CSLP approximation
  bool has_mg = false;
  MGHier mg;
  KrylovWS cslp;              // l >= 3: GMRES on M_l
  int cslp_maxit = 0;
};

enum Kind { K_LEVEL2 = 0, K_CSLP = 1, K_MGC = 2, K_OUTER = 3, K_NKIND = 4 };

inline int krylov_maxit(size_t N, double coef) {
  const int m = (int)std::floor(coef * std::pow((double)N, 0.25));
  return m < 1 ? 1 : m;
}

static const int kDenseMax = 512;

template <typename T>
static void set_five_point(OpDesc<T>& d, int nx, int ny, double H, double scale, cd sigma, int bc) {
  std::memset(&d, 0, sizeof(d));
  d.nx = nx; d.ny = ny; d.R = 1;
  d.bc = bc;
  d.inv_H2 = (T)(1.0 / (H * H));
  d.two_H = (T)(2.0 * H);
  d.scale = (T)scale;
  d.sig_re = (T)sigma.real();
  d.sig_im = (T)sigma.imag();
}

template <typename T>
static void set_wide(OpDesc<T>& d, int nx, int ny, double h, int level, cd sigma, int bc) {
  int R = 0;
  std::vector<double> lap, wav;
  coarse_tables(level, &R, lap, wav);
  const double hl = h * std::ldexp(1.0, level - 1);
  const double sl = std::ldexp(1.0, 2 * (level - 1));
  set_five_point(d, nx, ny, hl, sl, sigma, bc);
  d.R = R;
  const double h2 = h * h;
  for (size_t i = 0; i < lap.size(); ++i) {
    d.L[i] = (T)(lap[i] / h2);
    d.K[i] = (T)wav[i];
  }
  int R1 = 0;
  std::vector<double> t1, m1;
  coarse_tables_1d(level, &R1, t1, m1);
  for (size_t i = 0; i < t1.size(); ++i) {
    d.t1[i] = (T)(t1[i] / h2);
    d.m1[i] = (T)m1[i];
  }
}

template <typename T> static inline const OpDesc<T>& opsel(const DefLevel& L, bool cslp);
template <> inline const OpDesc<double>& opsel<double>(const DefLevel& L, bool cslp) { return cslp ? L.M64 : L.A64; }
template <> inline const OpDesc<float>& opsel<float>(const DefLevel& L, bool cslp) { return cslp ? L.M32 : L.A32; }
template <typename T> static inline const OpDesc<T>& mgop(const MGLevel& m);
template <> inline const OpDesc<double>& mgop<double>(const MGLevel& m) { return m.op64; }
template <> inline const OpDesc<float>& mgop<float>(const MGLevel& m) { return m.op32; }
template <typename T> static inline const T* levk(const DefLevel& L);
template <> inline const double* levk<double>(const DefLevel& L) { return L.k64; }
template <> inline const float* levk<float>(const DefLevel& L) { return L.k32; }
template <typename T> static inline const T* mgk(const DefLevel& D, int q);
template <> inline const double* mgk<double>(const DefLevel& D, int q) { return q == 0 ? D.k64 : D.mg.lv[q].k; }
template <> inline const float* mgk<float>(const DefLevel& D, int q) { return q == 0 ? D.k32 : D.mg.lv[q].k32; }

}  // namespace hm

using namespace hm;

struct hm_problem {
  hm_config cfg{};
  std::vector<DefLevel> lev;   // index 1..L
  int L = 0;
  bool mixed = false;
  hipStream_t s = nullptr;
  // outer FGMRES (always FP64)
  KrylovWS outer;
  c128* tmp64 = nullptr;       // N1
  void* pin_v = nullptr;       // precondition input in the level-1 type (mixed)
  void* pin_x = nullptr;
  // reductions / scalars
  RedBuf rb{};
  c128* scal = nullptr;        // small device scratch
  c128* coef = nullptr;        // combination coefficients (device)
  int coef_cap = 0;
  c128* host = nullptr;        // pinned host staging for device results
  c128* host_coef = nullptr;   // pinned host staging for coefficient uploads
  int host_cap = 0;
  c128* host_H = nullptr;      // pinned mirror of a GMRES Hessenberg (lookahead loop)
  size_t host_H_cap = 0;
  bool own_host = true;        // false: the pinned staging belongs to a batch
  // batch members: copies of the caller's right-hand side and solution
  bool batch_io = false;
  c128* ub = nullptr;
  c128* uu = nullptr;
  hipEvent_t col_ev[2] = {nullptr, nullptr};
  hipStream_t cap_stream = nullptr;   // private stream for graph capture
  // counts
  std::vector<int> rec[K_NKIND];
  std::vector<int> rep[K_NKIND];
  size_t rep_pos[K_NKIND] = {0, 0, 0, 0};
  double last_estimate = 0;
  // load hints of the Krylov CSLP's Gram-Schmidt passes (hm_set_basis_cache)
  CachePolicy cache;
  // small coarse levels solved by one workgroup per member (hm_set_small_krylov)
  bool small_krylov = true;
  int krylov_steps = HM_KRYLOV_STEPS_MAX;   // Arnoldi steps per two basis passes
  // optional per-kernel-class timing with HIP events on the problem's stream
  unsigned timing_mask = 0;
  int timing_every = 1;                 // bracket every n-th launch of a class
  long timing_seen[HM_TK_COUNT] = {0};
  struct Pending { hipEvent_t a, b; int cls; double bytes; };
  std::vector<Pending> pending;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
  double t_ms[HM_TK_COUNT] = {0};
  double t_bytes[HM_TK_COUNT] = {0};
  long t_launches[HM_TK_COUNT] = {0};
};

namespace hm {

static thread_local std::string g_last_error;

static int forced_count(hm_problem* p, int kind) {
  if (p->rep[kind].empty()) return -1;
  if (p->rep_pos[kind] >= p->rep[kind].size()) throw ArgError("replay counts exhausted");
  return p->rep[kind][p->rep_pos[kind]++];
}

// Timed launch: brackets the launch with events when its class is enabled.
template <typename F>
static void timed(hm_problem* p, int cls, double bytes, F&& launch) {
  if (!(p->timing_mask & (1u << cls)) || (p->timing_seen[cls]++ % p->timing_every) != 0) {
    HM_CHECK(launch());
    return;
  }
  std::pair<hipEvent_t, hipEvent_t> ev;
  if (p->pool.empty()) {
    HM_CHECK(hipEventCreate(&ev.first));
    HM_CHECK(hipEventCreate(&ev.second));
  } else {
    ev = p->pool.back();
    p->pool.pop_back();
  }
  HM_CHECK(hipEventRecord(ev.first, p->s));
  HM_CHECK(launch());
  HM_CHECK(hipEventRecord(ev.second, p->s));
  p->pending.push_back({ev.first, ev.second, cls, bytes});
}

// Collects finished event pairs (call after a stream synchronisation).
static void harvest(hm_problem* p) {
  for (auto& q : p->pending) {
    float ms = 0;
    HM_CHECK(hipEventElapsedTime(&ms, q.a, q.b));
    p->t_ms[q.cls] += ms;
    p->t_bytes[q.cls] += q.bytes;
    p->t_launches[q.cls] += 1;
    p->pool.push_back({q.a, q.b});
  }
  p->pending.clear();
}

static inline RedBuf rbuf(const hm_problem* p, size_t n) {
  return RedBuf{p->rb.partials, reduction_chunks(n)};
}

static void d2h(hm_problem* p, const c128* dev, int n) {
  HM_CHECK(hipMemcpyAsync(p->host, dev, sizeof(c128) * n, hipMemcpyDeviceToHost, p->s));
  HM_CHECK(hipStreamSynchronize(p->s));
  if (!p->pending.empty()) harvest(p);
}

// ---- members solved in lockstep ------------------------------------------------
// A solve drives one problem, or a batch of problems with the same layout, in
// lockstep: every launch covers the members still active at that point (the
// grid's z dimension), and each member keeps its own stopping decisions,
// Hessenberg least-squares problem and counts on the host, so that its
// arithmetic is exactly that of a solve on its own.  Member i's device buffers
// lie i * dz bytes after member 0's and its pinned staging i * hz bytes after
// member 0's; launches take member 0's pointers and stream.
struct Ctx {
  hm_problem* p;                  // member 0
  std::vector<hm_problem*> mem;   // every member (host state)
  long long dz = 0, hz = 0;
  c128* coef = nullptr;           // batch: coefficient rows on the device, coef_ld apart
  c128* host_coef = nullptr;      // batch: their pinned staging
  size_t coef_ld = 0;
  explicit Ctx(hm_problem* one) : p(one), mem{one} {}
};
using Act = std::vector<int>;     // members of a launch, ascending

static Batch members(const Ctx& c, const Act& a) {
  if (a.empty() || a.size() > (size_t)kMaxBatch) throw std::logic_error("bad member set");
  Batch z;
  z.dz = c.dz;
  z.hz = c.hz;
  z.n = (int)a.size();
  for (size_t t = 0; t < a.size(); ++t) z.slot[t] = (unsigned char)a[t];
  return z;
}

static unsigned mask_of(const Act& a) {
  unsigned m = 0;
  for (int i : a) m |= 1u << i;
  return m;
}

static void wait_stream(Ctx& c) {
  HM_CHECK(hipStreamSynchronize(c.p->s));
  if (!c.p->pending.empty()) harvest(c.p);
}

// ||x|| of every member of a, on the device (dev_out[0]) and in each member's
// pinned host[0].
template <typename T>
static void member_norms(Ctx& c, const Act& a, const cx<T>* x, size_t N, c128* dev_out) {
  HM_CHECK(launch_norm<T>(x, N, rbuf(c.p, N), dev_out, c.p->s, c.p->host, members(c, a)));
  wait_stream(c);
}

// x (+)= sum_i y_i V_i for the members of a (y[t] belongs to a[t]).
template <typename T>
static void combine_members(Ctx& c, const Act& a, const std::vector<std::vector<c128>>& y,
                            const cx<T>* V, size_t N, cx<T>* x, int accumulate) {
  hm_problem* p = c.p;
  // the staging may still feed the previous upload: wait for the stream
  HM_CHECK(hipStreamSynchronize(p->s));
  Batch z = members(c, a);
  if (c.mem.size() == 1) {
    const std::vector<c128>& v = y[0];
    if ((int)v.size() > p->coef_cap) throw ArgError("coefficient buffer too small");
    std::memcpy(p->host_coef, v.data(), sizeof(c128) * v.size());
    HM_CHECK(hipMemcpyAsync(p->coef, p->host_coef, sizeof(c128) * v.size(), hipMemcpyHostToDevice,
                            p->s));
    HM_CHECK(launch_combine<T>(V, N, (int)v.size(), p->coef, 0, 1.0, x, accumulate, N, p->s, z));
    return;
  }
  size_t rows = 0;
  for (size_t t = 0; t < a.size(); ++t) {
    if (y[t].size() > c.coef_ld) throw ArgError("coefficient buffer too small");
    std::memcpy(c.host_coef + (size_t)a[t] * c.coef_ld, y[t].data(), sizeof(c128) * y[t].size());
    z.cnt[t] = (int)y[t].size();
    rows = (size_t)a[t] + 1;
  }
  HM_CHECK(hipMemcpyAsync(c.coef, c.host_coef, sizeof(c128) * rows * c.coef_ld,
                          hipMemcpyHostToDevice, p->s));
  HM_CHECK(launch_combine<T>(V, N, -1, c.coef, c.coef_ld, 1.0, x, accumulate, N, p->s, z));
}

// Host state of one member's Krylov solve.
struct MemberKrylov {
  int i = 0;                 // member index
  double beta = 0, tol = 0;  // initial residual norm; relative tolerance (< 0: none)
  int maxit = 0, steps = 0;
  double est1 = -1, est2 = -1;
  bool ahead = false;
  LSQ lsq;
};

// Members of a0 with a nonzero right-hand side (norm in host[0]) and their
// step limits; replayed counts replace maxit and switch the tolerance off.
// Members with b = 0 get x = 0 and a count of 0 steps.
template <typename T>
static std::vector<MemberKrylov> start_members(Ctx& c, const Act& a0, int kind, int maxit,
                                               double tol, int cap, cx<T>* x, size_t N) {
  std::vector<MemberKrylov> st;
  Act zero;
  for (int i : a0) {
    hm_problem* q = c.mem[i];
    const double beta = q->host[0].re;
    if (beta == 0.0) {
      zero.push_back(i);
      if (kind >= 0) q->rec[kind].push_back(0);
      continue;
    }
    MemberKrylov m;
    m.i = i;
    m.beta = beta;
    m.maxit = maxit;
    m.tol = tol;
    if (kind >= 0) {
      const int forced = forced_count(q, kind);
      if (forced >= 0) {
        m.maxit = forced;
        m.tol = -1;
      }
    }
    if (m.maxit > cap) throw ArgError("Krylov step count exceeds the workspace");
    m.lsq.init(m.maxit, beta);
    st.push_back(std::move(m));
  }
  if (!zero.empty()) HM_CHECK(launch_zero<T>(x, N, c.p->s, members(c, zero)));
  return st;
}

static Act members_of(const std::vector<MemberKrylov>& st, const std::vector<int>& who) {
  Act a;
  for (int t : who) a.push_back(st[t].i);
  return a;
}

// Solutions x (+)= V y of every member from its least-squares problem; records
// the step counts under `kind`.
template <typename T>
static void finish_members(Ctx& c, std::vector<MemberKrylov>& st, int kind, const cx<T>* V,
                           size_t N, cx<T>* x, int accumulate) {
  if (st.empty()) return;
  Act a;
  std::vector<std::vector<c128>> y(st.size());
  for (size_t t = 0; t < st.size(); ++t) {
    st[t].lsq.solve(st[t].steps, y[t]);
    a.push_back(st[t].i);
  }
  combine_members<T>(c, a, y, V, N, x, accumulate);
  if (kind >= 0)
    for (auto& m : st) c.mem[m.i]->rec[kind].push_back(m.steps);
}

// ---- operator application on a level -----------------------------------------
template <typename T>
static void apply_level(Ctx& c, const Act& a, const DefLevel& L, bool cslp, int mode,
                        const cx<T>* u, const cx<T>* b, cx<T>* out) {
  HM_CHECK(launch_stencil<T>(opsel<T>(L, cslp), mode, u, levk<T>(L), b, out, T(0), c.p->s,
                             members(c, a)));
}

// ---- GMRES with classical Gram-Schmidt (Krylov CSLP) ----------------------------
// Unpreconditioned GMRES from x = 0 on the operator `op` with wavenumber `k`.
// The device never waits for the host: step j+1 is enqueued before the host
// reads the Hessenberg columns of step j (written to pinned memory by the
// reduction kernels, waited on with an event), so the host's stopping tests
// overlap the next step.  When a member meets its tolerance at step j, its
// speculative step j+1 has only written w, column j+1 and V_{j+2}, none of
// which its solution uses.
// The same solve when the level fits one workgroup (small_gmres_fits): every
// step, the Givens rotations and the stopping test run on the device, one
// workgroup per member, and the host waits once for the step counts.  A
// member with b = 0 (x = 0, no step) takes no replayed count, as below.
template <typename T>
static void gmres_small(Ctx& c, const Act& a0, const OpDesc<T>& op, const T* k, KrylovWS& ws,
                        int maxit, double tol, int kind, const cx<T>* b, cx<T>* x) {
  hm_problem* p = c.p;
  SmallGmresArgs ga;
  ga.ldh = ws.cap + 2;
  ga.mgs = p->cfg.cslp_orth == HM_ORTH_MODIFIED;
  std::vector<int> forced(a0.size(), -1);
  for (size_t t = 0; t < a0.size(); ++t) {
    forced[t] = kind >= 0 ? forced_count(c.mem[a0[t]], kind) : -1;
    ga.maxit[t] = forced[t] >= 0 ? forced[t] : maxit;
    ga.tol[t] = forced[t] >= 0 ? -1.0 : tol;
    if (ga.maxit[t] > ws.cap) throw ArgError("Krylov step count exceeds the workspace");
  }
  HM_CHECK(launch_gmres_small<T>(op, k, b, x, (cx<T>*)ws.V, (cx<T>*)ws.w, ws.H, ga, p->host_H,
                                 p->s, members(c, a0)));
  wait_stream(c);
  for (size_t t = 0; t < a0.size(); ++t) {
    hm_problem* q = c.mem[a0[t]];
    const c128 info = q->host_H[0];
    if (kind < 0) continue;
    if (info.re == 0.0 && info.im == 0.0 && forced[t] >= 0) --q->rep_pos[kind];
    q->rec[kind].push_back((int)info.re);
  }
}

// The same GMRES with S Arnoldi steps (S = 2, 3; the last block of a solve may
// be shorter) per two reads of the basis.
// For the block of steps j..j+S-1, Y_0 = M v_j and Y_{k+1} = M Y_k.  Pass A
// takes [V_0..V_j, Y]^H Y in one read of the basis; with it, classical
// Gram-Schmidt runs in the coordinates of [V_0..V_j, Y] on the device
// (launch_coefs: M acts on V through the Hessenberg columns already formed),
// giving the columns j..j+S-2 whole and column j+S-1 up to its subdiagonal
// entry; pass B forms v_{j+1}..v_{j+S-1} and the last step's w in one read of
// the basis, with ||w||.  In exact arithmetic these are the iterates of
// one-step classical Gram-Schmidt.  The host reads the columns of a block
// from the pinned mirror while the next block runs; work enqueued past a
// member's last step writes only vectors and columns its solution does not
// use.
template <typename T>
static void gmres_sstep(Ctx& c, const Act& a0, const OpDesc<T>& op, const T* k, KrylovWS& ws,
                        int maxit, double tol, int kind, int S, const cx<T>* b, cx<T>* x) {
  hm_problem* p = c.p;
  const size_t N = ws.N;
  cx<T>* V = (cx<T>*)ws.V;
  cx<T>* wb[3] = {(cx<T>*)ws.w, (cx<T>*)ws.w2, (cx<T>*)ws.w3};
  member_norms<T>(c, a0, b, N, ws.h);
  std::vector<MemberKrylov> st = start_members<T>(c, a0, kind, maxit, tol, ws.cap, x, N);
  if (st.empty()) return;
  const size_t ld = (size_t)ws.cap + 2;
  const int cld = ws.cap + 4;
  for (const auto& m : st)
    if ((size_t)(m.maxit + 2) * ld > p->host_H_cap) throw ArgError("Hessenberg mirror too small");
  const double es = (double)sizeof(cx<T>);
  const int tk_op = op.R == 1 ? HM_TK_FIVE_POINT : HM_TK_WIDE;
  std::vector<int> run;
  for (size_t t = 0; t < st.size(); ++t)
    if (st[t].maxit > 0) run.push_back((int)t);
  // steps of the block at j: S, fewer only where the workspace ends.  The
  // blocks do not depend on a member's step limit (steps past it are not
  // used), so a member's rounding is the same alone and in a batch.
  auto block_len = [&](int j) { return std::min(S, ws.cap - j); };
  // source of the next block: b, then the buffer that holds the last block's w
  // (index si); the block's Y_0 never takes the source's buffer, Y_1 may (the
  // source is consumed by the first apply)
  int si = -1;
  auto enqueue_block = [&](int j, int s, const std::vector<int>& who) {
    const Batch z = members(c, members_of(st, who));
    const double nm = (double)who.size();
    const int m = j + 1;
    const c128* sc = j == 0 ? ws.h : ws.H + (size_t)(j - 1) * ld + j;
    const cx<T>* src = si < 0 ? b : wb[si];
    const int i0 = si < 0 ? 0 : (si + 1) % 3;
    cx<T>* y[3] = {wb[i0], si < 0 ? wb[1] : wb[si], si < 0 ? wb[2] : wb[(si + 2) % 3]};
    timed(p, tk_op, nm * 3.5 * es * N, [&] {
      return launch_stencil_scaled<T>(op, src, k, sc, V + (size_t)j * N, y[0], p->s, z);
    });
    for (int r = 1; r < s; ++r)
      timed(p, tk_op, nm * 2.5 * es * N, [&] {
        return launch_stencil<T>(op, ST_APPLY, y[r - 1], k, nullptr, y[r], T(0), p->s, z);
      });
    timed(p, HM_TK_CGS_DOT, nm * (m + s) * es * N, [&] {
      return launch_multidots<T>(s, V, N, m, y[0], y[1], y[2], N, rbuf(p, N), ws.D, p->s, z,
                                 p->cache);
    });
    HM_CHECK(launch_coefs(s, ws.D, ws.H, (int)ld, j, ws.C, cld, p->host_H, p->s, z));
    timed(p, HM_TK_CGS_UPDATE, nm * (m + 2 * s) * es * N, [&] {
      return launch_updates<T>(s, y[0], y[1], y[2], V, N, m, ws.C, cld, N, rbuf(p, N),
                               ws.H + (size_t)(j + s - 1) * ld + j + s,
                               p->host_H + (size_t)(j + s - 1) * ld + j + s, p->s, z, p->cache);
    });
    si = i0;
  };
  // blocks enqueued one ahead of the host's stopping tests, except for members
  // expected to meet the tolerance within the block (the estimates fall about
  // geometrically)
  auto ahead_of = [&](int j, int s, const std::vector<int>& who) {
    std::vector<int> out;
    for (int t : who) {
      const MemberKrylov& q = st[t];
      double f = q.est1;
      if (q.est1 > 0 && q.est2 > 0)
        for (int r = 0; r < s; ++r) f *= q.est1 / q.est2;
      const bool soon = q.tol >= 0 && q.est1 > 0 && q.est2 > 0 && f <= q.tol * q.beta;
      if (j + s < q.maxit && !soon) out.push_back(t);
    }
    return out;
  };
  int s = 0;
  if (!run.empty()) {
    s = block_len(0);
    enqueue_block(0, s, run);
    HM_CHECK(hipEventRecord(p->col_ev[0], p->s));
  }
  for (int j = 0; !run.empty();) {
    // the next block for the members that will probably go on
    std::vector<int> spec = ahead_of(j, s, run);
    const int si_next = si;                             // holds the w of block j
    const int s_next = block_len(j + s);
    if (!spec.empty()) {
      enqueue_block(j + s, s_next, spec);
      HM_CHECK(hipEventRecord(p->col_ev[1], p->s));
    }
    // the columns of block j: event col_ev[0] follows every launch of block j
    HM_CHECK(hipEventSynchronize(p->col_ev[0]));
    std::vector<int> next;
    for (int t : run) {
      MemberKrylov& q = st[t];
      bool go = true;
      for (int r = 0; r < s && go; ++r) {
        const c128* hc = c.mem[q.i]->host_H + (size_t)(j + r) * ld;
        const double est = q.lsq.add(j + r, hc);
        q.steps = j + r + 1;
        q.est2 = q.est1;
        q.est1 = est;
        const bool broke = hc[j + r + 1].re <= 1e-14 * q.beta;
        if (broke || (q.tol >= 0 && est <= q.tol * q.beta) || j + r + 1 >= q.maxit) go = false;
      }
      if (go) next.push_back(t);
    }
    // members that go on without an enqueued block get it now (from block j's w)
    std::vector<int> late;
    for (int t : next)
      if (std::find(spec.begin(), spec.end(), t) == spec.end()) late.push_back(t);
    if (!late.empty()) {
      si = si_next;                                     // the same buffers as spec's block
      enqueue_block(j + s, s_next, late);
      HM_CHECK(hipEventRecord(p->col_ev[1], p->s));
    }
    std::swap(p->col_ev[0], p->col_ev[1]);
    run.swap(next);
    j += s;
    s = s_next;
  }
  wait_stream(c);                                        // timing events of the blocks
  finish_members<T>(c, st, kind, V, N, x, 0);
}

template <typename T>
static void gmres_cgs(Ctx& c, const Act& a0, const OpDesc<T>& op, const T* k, KrylovWS& ws,
                      int maxit, double tol, int kind, const cx<T>* b, cx<T>* x) {
  hm_problem* p = c.p;
  if (p->small_krylov && small_gmres_fits<T>(op, ws.cap)) {
    gmres_small<T>(c, a0, op, k, ws, maxit, tol, kind, b, x);
    return;
  }
  // the blocks of steps take the later steps' columns from relations that hold
  // to the basis's orthogonality: FP64 levels only (with an FP32 basis the
  // k = 200 solve took one outer step more and moved 2e-5 from the FP64
  // solution)
  if (p->krylov_steps > 1 && p->cfg.cslp_orth == HM_ORTH_CLASSICAL &&
      sizeof(T) == sizeof(double) && ws.cap + 1 + p->krylov_steps <= coefs_max_basis()) {
    gmres_sstep<T>(c, a0, op, k, ws, maxit, tol, kind, p->krylov_steps, b, x);
    return;
  }
  const size_t N = ws.N;
  cx<T>* V = (cx<T>*)ws.V;
  cx<T>* w = (cx<T>*)ws.w;
  member_norms<T>(c, a0, b, N, ws.h);
  std::vector<MemberKrylov> st = start_members<T>(c, a0, kind, maxit, tol, ws.cap, x, N);
  if (st.empty()) return;
  const size_t ld = (size_t)ws.cap + 2;
  for (const auto& m : st)
    if ((size_t)m.maxit * ld > p->host_H_cap) throw ArgError("Hessenberg mirror too small");
  const double es = (double)sizeof(cx<T>);
  const int tk_op = op.R == 1 ? HM_TK_FIVE_POINT : HM_TK_WIDE;
  cx<T>* wb[2] = {w, (cx<T>*)ws.w2};
  const bool mgs = p->cfg.cslp_orth == HM_ORTH_MODIFIED;
  // step j of the members st[t], t in who: v_j = src / s_j (s_0 = ||b||,
  // s_j = h_{j,j-1}) written to the basis in the same pass as w = M v_j;
  // classical Gram-Schmidt: one pass for the dots, one for the update and the
  // new norm; modified Gram-Schmidt: one fused step per basis vector (subtract
  // the previous projection, take the next dot), then the norm
  auto enqueue_step = [&](int j, const std::vector<int>& who) {
    const Batch z = members(c, members_of(st, who));
    const double nm = (double)who.size();
    c128* col = ws.H + (size_t)j * ld;
    const cx<T>* src = j == 0 ? b : wb[(j - 1) & 1];
    const c128* sc = j == 0 ? ws.h : ws.H + (size_t)(j - 1) * ld + j;
    cx<T>* wj = wb[j & 1];
    timed(p, tk_op, nm * 3.5 * es * N, [&] {
      return launch_stencil_scaled<T>(op, src, k, sc, V + (size_t)j * N, wj, p->s, z);
    });
    c128* hcol = p->host_H + (size_t)j * ld;      // pinned mirror of the column
    if (mgs) {
      for (int i = 0; i <= j; ++i)
        timed(p, HM_TK_MGS, nm * (i > 0 ? 4.0 : 2.0) * es * N, [&] {
          return launch_mgs_step<T>(wj, i > 0 ? V + (size_t)(i - 1) * N : nullptr, col + i - 1,
                                    V + (size_t)i * N, N, rbuf(p, N), col + i, p->s, hcol + i, z);
        });
      timed(p, HM_TK_MGS, nm * 3.0 * es * N, [&] {
        return launch_mgs_step<T>(wj, V + (size_t)j * N, col + j, nullptr, N, rbuf(p, N),
                                  col + j + 1, p->s, hcol + j + 1, z);
      });
      HM_CHECK(hipEventRecord(p->col_ev[j & 1], p->s));
      return;
    }
    timed(p, HM_TK_CGS_DOT, nm * (j + 2) * es * N, [&] {
      return launch_multidot_partial<T>(V, N, j + 1, wj, N, rbuf(p, N), p->s, z, p->cache);
    });
    HM_CHECK(launch_multidot_final<T>(j + 1, N, rbuf(p, N), col, p->s, hcol, z));
    timed(p, HM_TK_CGS_UPDATE, nm * (j + 3) * es * N, [&] {
      return launch_cgs_update_partial<T>(wj, V, N, j + 1, col, N, rbuf(p, N), p->s, z,
                                          p->cache);
    });
    HM_CHECK(launch_update_norm_final(N, rbuf(p, N), col + j + 1, p->s, hcol + j + 1, z));
    HM_CHECK(hipEventRecord(p->col_ev[j & 1], p->s));
  };
  std::vector<int> run;              // members at step j
  for (size_t t = 0; t < st.size(); ++t)
    if (st[t].maxit > 0) run.push_back((int)t);
  if (!run.empty()) enqueue_step(0, run);
  for (int j = 0; !run.empty(); ++j) {
    // Step j+1 goes in before step j's columns are read, except for members
    // expected to meet the tolerance at step j: the estimates fall about
    // geometrically, so est_j ~ est_{j-1}^2 / est_{j-2}.  A step enqueued past
    // convergence is wasted work; a wrong guess only costs one wait for the host.
    std::vector<int> ahead;
    for (int t : run) {
      MemberKrylov& m = st[t];
      bool ah = j + 1 < m.maxit;
      if (ah && m.tol >= 0 && m.est1 > 0 && m.est2 > 0 && m.est1 * (m.est1 / m.est2) <= m.tol * m.beta)
        ah = false;
      m.ahead = ah;
      if (ah) ahead.push_back(t);
    }
    if (!ahead.empty()) enqueue_step(j + 1, ahead);
    // the event was last recorded after every member's step j
    HM_CHECK(hipEventSynchronize(p->col_ev[j & 1]));
    std::vector<int> next, late;
    for (int t : run) {
      MemberKrylov& m = st[t];
      const c128* hc = c.mem[m.i]->host_H + (size_t)j * ld;
      const double est = m.lsq.add(j, hc);
      m.steps = j + 1;
      const bool broke = hc[j + 1].re <= 1e-14 * m.beta;
      if (broke || (m.tol >= 0 && est <= m.tol * m.beta) || j + 1 >= m.maxit) continue;
      next.push_back(t);
      if (!m.ahead) late.push_back(t);
      m.est2 = m.est1;
      m.est1 = est;
    }
    if (!late.empty()) enqueue_step(j + 1, late);
    run.swap(next);
  }
  finish_members<T>(c, st, kind, V, N, x, 0);
}

// ---- multigrid V-cycle for the CSLP of level l -----------------------------------
template <typename T>
static const cx<T>* mg_cycle(Ctx& c, const Act& a, DefLevel& D, int q, const cx<T>* b) {
  hm_problem* p = c.p;
  MGHier& H = D.mg;
  MGLevel& m = H.lv[q];
  // the damping weight follows each member's largest wavenumber
  Batch z = members(c, a);
  if (c.mem.size() > 1) {
    z.use_omega = 1;
    for (size_t t = 0; t < a.size(); ++t) z.omega[t] = c.mem[a[t]]->lev[D.l].mg.lv[q].omega;
  }
  const OpDesc<T>& op = mgop<T>(m);
  const T* k = mgk<T>(D, q);
  cx<T>* x = (cx<T>*)m.x;
  cx<T>* y = (cx<T>*)m.y;
  if (q == (int)H.lv.size() - 1) {
    if (H.dense) {
      HM_CHECK(launch_dense_matvec<T>((const c128*)H.inv, (int)m.N, b, x, p->s, z));
      return x;
    }
    if constexpr (std::is_same<T, float>::value) {
      if (H.gm64) {
        c128* b64 = (c128*)H.b64;
        c128* x64 = (c128*)H.x64;
        HM_CHECK(launch_convert<float, double>(b, b64, m.N, p->s, z));
        gmres_cgs<double>(c, a, m.op64, mgk<double>(D, q), H.gm, H.maxit, p->cfg.tol_cslp, K_MGC,
                          b64, x64);
        HM_CHECK(launch_convert<double, float>(x64, x, m.N, p->s, z));
        return x;
      }
    }
    gmres_cgs<T>(c, a, op, k, H.gm, H.maxit, p->cfg.tol_cslp, K_MGC, b, x);
    return x;
  }
  const T om = (T)m.omega;
  HM_CHECK(launch_jacobi0<T>(op, k, b, x, om, p->s, z));
  for (int s = 1; s < p->cfg.mg_nu_pre; ++s) {
    HM_CHECK(launch_stencil<T>(op, ST_JACOBI, x, k, b, y, om, p->s, z));
    std::swap(x, y);
  }
  cx<T>* r = (cx<T>*)m.r;
  HM_CHECK(launch_stencil<T>(op, ST_RESID, x, k, b, r, T(0), p->s, z));
  MGLevel& mc = H.lv[q + 1];
  HM_CHECK(launch_restrict_fw<T>(r, m.nx, m.ny, (cx<T>*)mc.b, p->cfg.bc, p->s, z));
  const cx<T>* e = mg_cycle<T>(c, a, D, q + 1, (const cx<T>*)mc.b);
  HM_CHECK(launch_prolong_bilinear_add<T>(e, m.nx, m.ny, x, p->cfg.bc, p->s, z));
  for (int s = 0; s < p->cfg.mg_nu_post; ++s) {
    HM_CHECK(launch_stencil<T>(op, ST_JACOBI, x, k, b, y, om, p->s, z));
    std::swap(x, y);
  }
  return x;
}

// One V-cycle for the CSLP of level D on b.  When b is the level's r~ buffer
// and the coarsest solve is dense, the cycle runs as a HIP graph captured on
// first use for this set of members (no host decisions inside, no memset
// nodes); otherwise eagerly.
template <typename T>
static const cx<T>* vcycle(Ctx& c, const Act& a, DefLevel& D, const cx<T>* b) {
  hm_problem* p = c.p;
  MGHier& H = D.mg;
  if (!H.dense || (const void*)b != D.rt || !p->cap_stream) return mg_cycle<T>(c, a, D, 0, b);
  const unsigned key = mask_of(a);
  hipGraphExec_t ge = nullptr;
  for (const auto& g : H.graphs)
    if (g.first == key) ge = g.second;
  if (!ge) {
    hipStream_t saved = p->s;
    hipGraph_t g = nullptr;
    HM_CHECK(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
    p->s = p->cap_stream;
    const cx<T>* out = nullptr;
    try {
      out = mg_cycle<T>(c, a, D, 0, b);
    } catch (...) {
      p->s = saved;
      (void)hipStreamEndCapture(p->cap_stream, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    p->s = saved;
    HM_CHECK(hipStreamEndCapture(p->cap_stream, &g));
    const hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HM_CHECK(e);
    H.graphs.push_back({key, ge});
    H.graph_out = out;
  }
  HM_CHECK(hipGraphLaunch(ge, p->s));
  return (const cx<T>*)H.graph_out;
}

}  // namespace hm

namespace hm {

template <typename T>
static void precond(Ctx& c, const Act& a, int l, const cx<T>* v, cx<T>* x);

// CSLP^-1 approximation of level l: one V-cycle (levels 1-2) or GMRES.  Returns
// the buffer holding the result (`out` for GMRES, a multigrid buffer otherwise).
template <typename T>
static const cx<T>* cslp_apply(Ctx& c, const Act& a, int l, const cx<T>* r, cx<T>* out) {
  hm_problem* p = c.p;
  DefLevel& D = p->lev[l];
  if (D.has_mg) return vcycle<T>(c, a, D, r);
  gmres_cgs<T>(c, a, opsel<T>(D, true), levk<T>(D), D.cslp, D.cslp_maxit, p->cfg.tol_cslp, K_CSLP,
               r, out);
  return out;
}

// FGMRES with modified Gram-Schmidt (Algorithm 1) on the operator of level lv,
// zero initial guess.  Preconditioner: Prec_lv (lv < L) or the Krylov CSLP
// (lv == L).
template <typename T>
static void fgmres_level(Ctx& c, const Act& a0, int lv, const cx<T>* b, cx<T>* x, double tol,
                         int maxit, int kind) {
  hm_problem* p = c.p;
  DefLevel& D = p->lev[lv];
  KrylovWS& ws = D.fg;
  const size_t N = D.N;
  cx<T>* V = (cx<T>*)ws.V;
  cx<T>* X = (cx<T>*)ws.X;
  cx<T>* w = (cx<T>*)ws.w;
  member_norms<T>(c, a0, b, N, ws.h);
  // a basis smaller than the step cap (hm_config.level2_basis) limits the steps;
  // a solve that needs more stops the call (BasisError) instead of returning a
  // result the full basis would not give
  const int lim = std::min(maxit, ws.cap);
  std::vector<MemberKrylov> st = start_members<T>(c, a0, kind, lim, tol, ws.cap, x, N);
  if (st.empty()) return;
  std::vector<int> run, every;
  for (size_t t = 0; t < st.size(); ++t) {
    every.push_back((int)t);
    if (st[t].maxit > 0) run.push_back((int)t);
  }
  HM_CHECK(launch_scale_dev<T>(b, V, ws.h, 1, N, p->s, members(c, members_of(st, every))));
  const double es = (double)sizeof(cx<T>);
  for (int j = 0; !run.empty(); ++j) {
    const Act a = members_of(st, run);
    const Batch z = members(c, a);
    const double nm = (double)a.size();
    cx<T>* Vj = V + (size_t)j * N;
    cx<T>* Xj = X + (size_t)j * N;
    if (lv == p->L) {
      // with two levels the coarsest one owns a multigrid hierarchy, whose
      // V-cycle leaves its result in a multigrid buffer: move it into Z_j
      const cx<T>* r = cslp_apply<T>(c, a, lv, Vj, Xj);
      if (r != Xj)
        for (int i : a)
          HM_CHECK(hipMemcpyAsync((char*)Xj + (long long)i * c.dz,
                                  (const char*)r + (long long)i * c.dz, sizeof(cx<T>) * N,
                                  hipMemcpyDeviceToDevice, p->s));
    } else {
      precond<T>(c, a, lv, Vj, Xj);
    }
    timed(p, D.A64.R == 1 ? HM_TK_FIVE_POINT : HM_TK_WIDE, nm * 2.5 * es * N, [&] {
      return launch_stencil<T>(opsel<T>(D, false), ST_APPLY, Xj, levk<T>(D), nullptr, w, T(0),
                               p->s, z);
    });
    for (int i = 0; i <= j; ++i)
      timed(p, HM_TK_MGS, nm * (i > 0 ? 4.0 : 2.0) * es * N, [&] {
        return launch_mgs_step<T>(w, i > 0 ? V + (size_t)(i - 1) * N : nullptr, ws.h + i - 1,
                                  V + (size_t)i * N, N, rbuf(p, N), ws.h + i, p->s, p->host + i, z);
      });
    timed(p, HM_TK_MGS, nm * 3.0 * es * N, [&] {
      return launch_mgs_step<T>(w, Vj, ws.h + j, nullptr, N, rbuf(p, N), ws.h + j + 1, p->s,
                                p->host + j + 1, z);
    });
    wait_stream(c);
    std::vector<int> next, scale;
    for (int t : run) {
      MemberKrylov& m = st[t];
      const c128* hc = c.mem[m.i]->host;
      const double est = m.lsq.add(j, hc);
      m.steps = j + 1;
      const bool broke = hc[j + 1].re <= 1e-14 * m.beta;
      if (!broke) scale.push_back(t);
      const bool met = m.tol >= 0 && est <= m.tol * m.beta;
      if (!broke && !met && m.tol >= 0 && j + 1 >= m.maxit && m.maxit < maxit)
        throw BasisError("a level-2 solve needs more than the " + std::to_string(ws.cap) +
                         " basis vectors reserved (hm_config.level2_basis)");
      if (broke || met || j + 1 >= m.maxit) continue;
      next.push_back(t);
    }
    if (!scale.empty())
      HM_CHECK(launch_scale_dev<T>(w, V + (size_t)(j + 1) * N, ws.h + j + 1, 1, N, p->s,
                                   members(c, members_of(st, scale))));
    run.swap(next);
  }
  finish_members<T>(c, st, kind, X, N, x, 0);
}

// Levels 2..tol_levels above the coarsest iterate to tol_level2; every other
// coarse level takes coarse_steps FGMRES steps (the cycle type, Sec. 3.2).
static bool tol_level(const hm_config& c, int L, int l) {
  return l >= 2 && l < L && l <= c.tol_levels;
}

// Coarse problem E_c x = b of level cl (Algorithm 1, restriction to
// interpolation).  Only level-2 solves are recorded / replayed (kind 0).
template <typename T>
static void coarse_solve(Ctx& c, const Act& a, int cl, const cx<T>* b, cx<T>* x) {
  const hm_problem* p = c.p;
  if (tol_level(p->cfg, p->L, cl))
    fgmres_level<T>(c, a, cl, b, x, p->cfg.tol_level2, p->cfg.level2_maxit, cl == 2 ? K_LEVEL2 : -1);
  else
    fgmres_level<T>(c, a, cl, b, x, -1.0, p->cfg.coarse_steps, -1);
}

template <typename T, typename Tn>
static void coarse_branch(Ctx& c, const Act& a, int l, const cx<T>* v) {
  hm_problem* p = c.p;
  const Batch z = members(c, a);
  DefLevel& D = p->lev[l];
  DefLevel& C = p->lev[l + 1];
  HM_CHECK(launch_restrict_z<T, Tn>(v, D.nx, D.ny, (cx<Tn>*)C.rhs, p->cfg.bc, p->s, z));
  coarse_solve<Tn>(c, a, l + 1, (const cx<Tn>*)C.rhs, (cx<Tn>*)C.sol);
  HM_CHECK(launch_prolong_z<Tn, T>((const cx<Tn>*)C.sol, D.nx, D.ny, (cx<T>*)D.t, p->cfg.bc, p->s,
                                   z));
}

// Prec_l(v) = M_l^-1 (v - A_l t) + t,  t = Z E^-1 Z^T v   (A-DEF1, Sec. 3.1)
template <typename T>
static void precond(Ctx& c, const Act& a, int l, const cx<T>* v, cx<T>* x) {
  hm_problem* p = c.p;
  DefLevel& D = p->lev[l];
  if (p->lev[l + 1].dbl)
    coarse_branch<T, double>(c, a, l, v);
  else
    coarse_branch<T, float>(c, a, l, v);
  cx<T>* t = (cx<T>*)D.t;
  cx<T>* rt = (cx<T>*)D.rt;
  apply_level<T>(c, a, D, false, ST_RESID, t, v, rt);              // r~ = v - A t
  const cx<T>* r = cslp_apply<T>(c, a, l, rt, (cx<T>*)D.xo);       // r ~ M^-1 r~
  HM_CHECK(launch_add<T>(r, t, x, D.N, p->s, members(c, a)));       // x = r + t
}

// Finest-level preconditioner on complex128 vectors (casts in mixed mode).
static void precond_top(Ctx& c, const Act& a, const c128* v, c128* x) {
  hm_problem* p = c.p;
  const size_t N = p->lev[1].N;
  if (p->mixed) {
    const Batch z = members(c, a);
    HM_CHECK(launch_convert<double, float>(v, (c64*)p->pin_v, N, p->s, z));
    precond<float>(c, a, 1, (const c64*)p->pin_v, (c64*)p->pin_x);
    HM_CHECK(launch_convert<float, double>((const c64*)p->pin_x, x, N, p->s, z));
  } else {
    precond<double>(c, a, 1, v, x);
  }
}

// Outer FGMRES (Algorithm 1 at level 1, FP64, restarted) for every member; b
// and u are member 0's vectors (the others at the member stride).  info: one
// record per member, or null.
static hm_status outer_solve(Ctx& c, const c128* b, c128* u, hm_solve_info* info) {
  const auto t0 = std::chrono::steady_clock::now();
  hm_problem* p = c.p;
  DefLevel& D = p->lev[1];
  KrylovWS& ws = p->outer;
  const size_t N = D.N;
  c128* V = (c128*)ws.V;
  c128* X = (c128*)ws.X;
  c128* w = (c128*)ws.w;
  const hm_config& cf = p->cfg;
  const int nb = (int)c.mem.size();
  struct Outer {
    size_t rec0[K_NKIND];
    double bnorm = 0, rel_true = 0, est_rel = 0;
    int total = 0;
  };
  std::vector<Outer> o(nb);
  Act act;
  for (int i = 0; i < nb; ++i) {
    act.push_back(i);
    for (int kd = 0; kd < K_NKIND; ++kd) o[i].rec0[kd] = c.mem[i]->rec[kd].size();
  }
  member_norms<double>(c, act, b, N, ws.h);
  for (int i = 0; i < nb; ++i) o[i].bnorm = c.mem[i]->host[0].re;
  HM_CHECK(launch_zero<double>(u, N, p->s, members(c, act)));
  while (!act.empty()) {
    HM_CHECK(launch_stencil<double>(D.A64, ST_RESID, u, D.k64, b, p->tmp64, 0.0, p->s,
                                    members(c, act)));
    member_norms<double>(c, act, p->tmp64, N, ws.h);
    std::vector<MemberKrylov> st;       // members that run another restart cycle
    for (int i : act) {
      hm_problem* q = c.mem[i];
      Outer& m = o[i];
      const double rnorm = q->host[0].re;
      m.rel_true = m.bnorm > 0 ? rnorm / m.bnorm : 0.0;
      if (m.bnorm == 0.0 || rnorm <= cf.tol_outer * m.bnorm || m.total >= cf.outer_maxit) continue;
      MemberKrylov k;
      k.i = i;
      k.beta = rnorm;
      k.maxit = std::min(cf.outer_restart, cf.outer_maxit - m.total);
      k.tol = cf.tol_outer;
      const int forced = forced_count(q, K_OUTER);
      if (forced >= 0) {
        k.maxit = forced;
        k.tol = -1;
      }
      if (k.maxit > ws.cap) throw ArgError("outer step count exceeds the restart length");
      k.lsq.init(k.maxit, rnorm);
      st.push_back(std::move(k));
    }
    std::vector<int> run, every;
    for (size_t t = 0; t < st.size(); ++t) {
      every.push_back((int)t);
      if (st[t].maxit > 0) run.push_back((int)t);
    }
    act = members_of(st, every);
    if (act.empty()) break;
    HM_CHECK(launch_scale_dev<double>(p->tmp64, V, ws.h, 1, N, p->s, members(c, act)));
    for (int j = 0; !run.empty(); ++j) {
      const Act a = members_of(st, run);
      const Batch z = members(c, a);
      const double nm = (double)a.size();
      c128* Vj = V + (size_t)j * N;
      c128* Xj = X + (size_t)j * N;
      precond_top(c, a, Vj, Xj);
      timed(p, HM_TK_FIVE_POINT, nm * 40.0 * N, [&] {
        return launch_stencil<double>(D.A64, ST_APPLY, Xj, D.k64, nullptr, w, 0.0, p->s, z);
      });
      for (int i = 0; i <= j; ++i)
        timed(p, HM_TK_MGS, nm * (i > 0 ? 64.0 : 32.0) * N, [&] {
          return launch_mgs_step<double>(w, i > 0 ? V + (size_t)(i - 1) * N : nullptr,
                                         ws.h + i - 1, V + (size_t)i * N, N, rbuf(p, N), ws.h + i,
                                         p->s, p->host + i, z);
        });
      timed(p, HM_TK_MGS, nm * 48.0 * N, [&] {
        return launch_mgs_step<double>(w, Vj, ws.h + j, nullptr, N, rbuf(p, N), ws.h + j + 1, p->s,
                                       p->host + j + 1, z);
      });
      wait_stream(c);
      std::vector<int> next, scale;
      for (int t : run) {
        MemberKrylov& m = st[t];
        Outer& om = o[m.i];
        const c128* hc = c.mem[m.i]->host;
        const double est = m.lsq.add(j, hc);
        om.est_rel = om.bnorm > 0 ? est / om.bnorm : 0.0;
        m.steps = j + 1;
        const bool broke = hc[j + 1].re <= 1e-14 * m.beta;
        if (!broke) scale.push_back(t);
        if (broke || (m.tol >= 0 && est <= m.tol * om.bnorm) || j + 1 >= m.maxit) continue;
        next.push_back(t);
      }
      if (!scale.empty())
        HM_CHECK(launch_scale_dev<double>(w, V + (size_t)(j + 1) * N, ws.h + j + 1, 1, N, p->s,
                                          members(c, members_of(st, scale))));
      run.swap(next);
    }
    for (const auto& m : st) o[m.i].total += m.steps;
    finish_members<double>(c, st, K_OUTER, X, N, u, 1);
  }
  wait_stream(c);
  const double secs =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  bool ok = true;
  for (int i = 0; i < nb; ++i) {
    hm_problem* q = c.mem[i];
    q->last_estimate = o[i].est_rel;
    ok = ok && o[i].rel_true <= cf.tol_outer;
    if (!info) continue;
    auto sum_since = [&](int kind) {
      long s = 0;
      for (size_t r = o[i].rec0[kind]; r < q->rec[kind].size(); ++r) s += q->rec[kind][r];
      return (int)s;
    };
    hm_solve_info& in = info[i];
    in.outer_iters = o[i].total;
    in.level2_iters_total = sum_since(K_LEVEL2);
    in.cslp_iters_total = sum_since(K_CSLP);
    in.mg_coarse_iters_total = sum_since(K_MGC);
    in.rel_res_estimate = o[i].est_rel;
    in.rel_res_true = o[i].rel_true;
    in.seconds = secs;
  }
  return ok ? HM_OK : HM_NOT_CONVERGED;
}

// ---- set-up ------------------------------------------------------------------------

static bool validate(const hm_config* c, std::string* why) {
  auto bad = [&](const char* m) { if (why) *why = m; return false; };
  if (!c) return bad("null config");
  if (c->levels < 2 || c->levels > 6) return bad("levels must be in [2, 6]");
  const int f = 1 << (c->levels - 1);
  if (c->nx < 3 || c->ny < 3) return bad("grid too small");
  if ((c->nx - 1) % f || (c->ny - 1) % f) return bad("(n-1) must be divisible by 2^(levels-1)");
  if ((c->nx - 1) / f + 1 < 3 || (c->ny - 1) / f + 1 < 3) return bad("coarsest level below 3 nodes");
  if (!(c->h > 0) || !std::isfinite(c->h)) return bad("h must be positive");
  if (c->bc != HM_BC_SOMMERFELD && c->bc != HM_BC_DIRICHLET) return bad("unknown boundary condition");
  if (!std::isfinite(c->beta1) || !std::isfinite(c->beta2)) return bad("beta not finite");
  if (c->precision != HM_FP64 && c->precision != HM_MIXED_FP32 && c->precision != HM_MIXED_FP32_ALL)
    return bad("precision");
  if (c->outer_restart < 1 || c->outer_maxit < 1 || c->level2_maxit < 1) return bad("step caps");
  if (c->level2_basis < 0 || c->level2_basis > c->level2_maxit)
    return bad("level2_basis must be in [0, level2_maxit]");
  if (c->mg_nu_pre < 1 || c->mg_nu_post < 0) return bad("smoothing steps");
  if (!(c->tol_outer > 0) || !(c->tol_level2 > 0) || !(c->tol_cslp > 0) || !(c->maxit_coef > 0))
    return bad("tolerances");
  if (c->coarse_steps < 1 || c->coarse_steps > 16) return bad("coarse_steps must be in [1, 16]");
  if (c->tol_levels < 1 || c->tol_levels > 6) return bad("tol_levels must be in [1, 6]");
  if (c->cslp_orth != HM_ORTH_CLASSICAL && c->cslp_orth != HM_ORTH_MODIFIED)
    return bad("cslp_orth must be HM_ORTH_CLASSICAL or HM_ORTH_MODIFIED");
  for (int r : c->reserved)
    if (r != 0) return bad("reserved fields must be zero");
  return true;
}

static bool can_coarsen(int nx, int ny) {
  return (nx - 1) % 2 == 0 && (ny - 1) % 2 == 0 && (nx - 1) / 2 + 1 >= 3 && (ny - 1) / 2 + 1 >= 3;
}

// Lays out the workspace (sizes + pointers) and fills the static level data.
static void plan(hm_problem* p, Carver& cv) {
  const hm_config& c = p->cfg;
  p->L = c.levels;
  p->mixed = c.precision != HM_FP64;
  p->lev.assign(p->L + 2, DefLevel());
  const cd sig_m(c.beta1, c.beta2);
  int mmax = c.outer_restart + 2;
  int nx = c.nx, ny = c.ny;
  auto esz = [](bool dbl) { return dbl ? sizeof(c128) : sizeof(c64); };
  for (int l = 1; l <= p->L; ++l) {
    DefLevel& D = p->lev[l];
    D.l = l; D.nx = nx; D.ny = ny; D.N = (size_t)nx * ny;
    D.hl = c.h * std::ldexp(1.0, l - 1);
    D.sl = std::ldexp(1.0, 2 * (l - 1));
    // mixed: levels 1-2 in FP32, the coarsest-level solve (levels >= 3) in FP64;
    // HM_MIXED_FP32_ALL: every preconditioner level in FP32
    D.dbl = !p->mixed || (l >= 3 && c.precision == HM_MIXED_FP32);
    const size_t es = esz(D.dbl);
    D.k64 = cv.take<double>(D.N);
    if (!D.dbl) D.k32 = cv.take<float>(D.N);
    if (l == 1) {
      set_five_point(D.A64, nx, ny, c.h, 1.0, cd(1, 0), c.bc);
      set_five_point(D.M64, nx, ny, c.h, 1.0, sig_m, c.bc);
      set_five_point(D.A32, nx, ny, c.h, 1.0, cd(1, 0), c.bc);
      set_five_point(D.M32, nx, ny, c.h, 1.0, sig_m, c.bc);
    } else {
      set_wide(D.A64, nx, ny, c.h, l, cd(1, 0), c.bc);
      set_wide(D.M64, nx, ny, c.h, l, sig_m, c.bc);
      set_wide(D.A32, nx, ny, c.h, l, cd(1, 0), c.bc);
      set_wide(D.M32, nx, ny, c.h, l, sig_m, c.bc);
    }
    if (l >= 2) {
      D.fg.cap = !tol_level(c, p->L, l) ? c.coarse_steps
                 : c.level2_basis > 0       ? c.level2_basis
                                            : c.level2_maxit;
      D.fg.N = D.N;
      D.fg.V = cv.take<char>((size_t)(D.fg.cap + 1) * D.N * es);
      D.fg.X = cv.take<char>((size_t)D.fg.cap * D.N * es);
      D.fg.w = cv.take<char>(D.N * es);
      D.fg.h = cv.take<c128>(D.fg.cap + 2);
      D.rhs = cv.take<char>(D.N * es);
      D.sol = cv.take<char>(D.N * es);
      mmax = std::max(mmax, D.fg.cap + 2);
    }
    if (l < p->L) {
      D.t = cv.take<char>(D.N * es);
      D.rt = cv.take<char>(D.N * es);
      D.xo = cv.take<char>(D.N * es);
    }
    if (l <= 2) {
      D.has_mg = true;
      MGHier& H = D.mg;
      H.lv.clear();
      int mx = nx, my = ny;
      double Hs = D.hl;
      for (int q = 0;; ++q) {
        MGLevel m;
        m.nx = mx; m.ny = my; m.N = (size_t)mx * my; m.H = Hs;
        if (q == 0) {
          m.op64 = D.M64;
          m.op32 = D.M32;
        } else {
          set_five_point(m.op64, mx, my, Hs, D.sl, sig_m, c.bc);
          set_five_point(m.op32, mx, my, Hs, D.sl, sig_m, c.bc);
          m.k = cv.take<double>(m.N);
          if (!D.dbl) m.k32 = cv.take<float>(m.N);
          m.b = cv.take<char>(m.N * es);
        }
        m.x = cv.take<char>(m.N * es);
        m.y = cv.take<char>(m.N * es);
        m.r = cv.take<char>(m.N * es);
        H.lv.push_back(m);
        if (!can_coarsen(mx, my)) break;
        mx = (mx - 1) / 2 + 1;
        my = (my - 1) / 2 + 1;
        Hs *= 2;
      }
      MGLevel& last = H.lv.back();
      H.dense = last.N <= (size_t)kDenseMax;
      if (H.dense) {
        H.inv = cv.take<c128>(last.N * last.N);      // FP64 in every precision
        H.tmpA = cv.take<c128>(last.N * last.N);
        H.tmpB = cv.take<c128>(last.N * last.N);
      } else {
        H.maxit = krylov_maxit(last.N, c.maxit_coef);
        H.gm64 = !D.dbl && c.precision == HM_MIXED_FP32;
        const size_t ges = H.gm64 ? sizeof(c128) : es;
        if (H.gm64) {
          H.b64 = cv.take<char>(last.N * ges);
          H.x64 = cv.take<char>(last.N * ges);
        }
        H.gm.cap = H.maxit;
        H.gm.N = last.N;
        H.gm.V = cv.take<char>((size_t)(H.maxit + 1) * last.N * ges);
        H.gm.w = cv.take<char>(last.N * ges);
        H.gm.w2 = cv.take<char>(last.N * ges);
        H.gm.w3 = cv.take<char>(last.N * ges);
        H.gm.h = cv.take<c128>(H.maxit + 2);
        H.gm.H = cv.take<c128>((size_t)(H.maxit + 2) * (H.maxit + 2));
        H.gm.D = cv.take<c128>(3 * (size_t)(H.maxit + 4));
        H.gm.C = cv.take<c128>(3 * (size_t)(H.maxit + 4));
        mmax = std::max(mmax, H.maxit + 2);
        p->host_H_cap = std::max(p->host_H_cap, (size_t)(H.maxit + 2) * (H.maxit + 2));
      }
    } else {
      D.cslp_maxit = krylov_maxit(D.N, c.maxit_coef);
      D.cslp.cap = D.cslp_maxit;
      D.cslp.N = D.N;
      D.cslp.V = cv.take<char>((size_t)(D.cslp_maxit + 1) * D.N * es);
      D.cslp.w = cv.take<char>(D.N * es);
      D.cslp.w2 = cv.take<char>(D.N * es);
      D.cslp.w3 = cv.take<char>(D.N * es);
      D.cslp.h = cv.take<c128>(D.cslp_maxit + 2);
      D.cslp.H = cv.take<c128>((size_t)(D.cslp_maxit + 2) * (D.cslp_maxit + 2));
      D.cslp.D = cv.take<c128>(3 * (size_t)(D.cslp_maxit + 4));
      D.cslp.C = cv.take<c128>(3 * (size_t)(D.cslp_maxit + 4));
      mmax = std::max(mmax, D.cslp_maxit + 2);
      p->host_H_cap = std::max(p->host_H_cap, (size_t)(D.cslp_maxit + 2) * (D.cslp_maxit + 2));
    }
    if (l < p->L) {
      nx = (nx - 1) / 2 + 1;
      ny = (ny - 1) / 2 + 1;
    }
  }
  DefLevel& D1 = p->lev[1];
  KrylovWS& o = p->outer;
  o.cap = c.outer_restart;
  o.N = D1.N;
  o.V = cv.take<c128>((size_t)(o.cap + 1) * D1.N);
  o.X = cv.take<c128>((size_t)o.cap * D1.N);
  o.w = cv.take<c128>(D1.N);
  o.h = cv.take<c128>(o.cap + 2);
  p->tmp64 = cv.take<c128>(D1.N);
  if (p->mixed) {
    p->pin_v = cv.take<c64>(D1.N);
    p->pin_x = cv.take<c64>(D1.N);
  }
  // three Arnoldi steps per sweep take 3 (m + 3) dots per reduction
  p->rb.partials = cv.take<c128>((size_t)kMaxChunks * (3 * mmax + 9));
  p->rb.nchunks = 0;   // chosen per reduction from its length (rbuf)
  p->scal = cv.take<c128>(16);
  p->coef_cap = mmax + 2;
  p->coef = cv.take<c128>(p->coef_cap);
  if (p->batch_io) {
    p->ub = cv.take<c128>(D1.N);
    p->uu = cv.take<c128>(D1.N);
  }
}

}  // namespace hm

namespace hm {

// Gauss-Jordan inversion with partial pivoting (host, FP64), row-major.
static void invert_dense(std::vector<cd>& A, int n) {
  std::vector<cd> I((size_t)n * n, cd(0));
  for (int i = 0; i < n; ++i) I[(size_t)i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    double best = std::abs(A[(size_t)c * n + c]);
    for (int r = c + 1; r < n; ++r) {
      const double v = std::abs(A[(size_t)r * n + c]);
      if (v > best) { best = v; piv = r; }
    }
    if (best == 0.0) throw ArgError("singular coarsest multigrid operator");
    if (piv != c)
      for (int k = 0; k < n; ++k) {
        std::swap(A[(size_t)c * n + k], A[(size_t)piv * n + k]);
        std::swap(I[(size_t)c * n + k], I[(size_t)piv * n + k]);
      }
    const cd d = 1.0 / A[(size_t)c * n + c];
    for (int k = 0; k < n; ++k) {
      A[(size_t)c * n + k] *= d;
      I[(size_t)c * n + k] *= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const cd f = A[(size_t)r * n + c];
      if (f == cd(0)) continue;
      for (int k = 0; k < n; ++k) {
        A[(size_t)r * n + k] -= f * A[(size_t)c * n + k];
        I[(size_t)r * n + k] -= f * I[(size_t)c * n + k];
      }
    }
  }
  A.swap(I);
}

static double omega_rule(double kmax, double H) { return kmax * kmax * H * H <= 1.0 ? 0.8 : 0.5; }

static void initialize(hm_problem* p, const double* k_dev) {
  DefLevel& D1 = p->lev[1];
  HM_CHECK(hipMemcpyAsync(D1.k64, k_dev, sizeof(double) * D1.N, hipMemcpyDeviceToDevice, p->s));
  {
    const size_t N = D1.N;
    HM_CHECK(launch_check_k(D1.k64, N, rbuf(p, N), p->scal, p->s));
    d2h(p, p->scal, 1);
    if (p->host[0].re != 0.0) throw ArgError("wavenumber field has negative or non-finite entries");
  }
  for (int l = 2; l <= p->L; ++l) {
    const DefLevel& F = p->lev[l - 1];
    HM_CHECK(launch_inject<double, double>(F.k64, F.nx, F.ny, p->lev[l].k64, p->s));
  }
  for (int l = 1; l <= p->L; ++l) {
    DefLevel& D = p->lev[l];
    if (!D.dbl) HM_CHECK(launch_convert_real<double, float>(D.k64, D.k32, D.N, p->s));
    const size_t N = D.N;
    HM_CHECK(launch_max_real(D.k64, N, rbuf(p, N), p->scal, p->s));
    d2h(p, p->scal, 1);
    D.kmax = p->host[0].re;
    // k = 0 everywhere with Sommerfeld ghosts leaves the Neumann Laplacian,
    // whose constants span its null space: no solution to approximate
    if (l == 1 && D.kmax == 0.0 && p->cfg.bc == HM_BC_SOMMERFELD)
      throw ArgError("wavenumber field is zero everywhere: the Sommerfeld problem is singular");
    if (!D.has_mg) continue;
    MGHier& H = D.mg;
    for (size_t q = 0; q < H.lv.size(); ++q) {
      MGLevel& m = H.lv[q];
      m.omega = omega_rule(D.kmax, m.H);
      if (q >= 1) {
        const MGLevel& f = H.lv[q - 1];
        const double* kf = q == 1 ? D.k64 : f.k;
        HM_CHECK(launch_inject<double, double>(kf, f.nx, f.ny, m.k, p->s));
        if (!D.dbl) HM_CHECK(launch_convert_real<double, float>(m.k, m.k32, m.N, p->s));
      }
    }
    if (H.dense) {
      const int q = (int)H.lv.size() - 1;
      MGLevel& m = H.lv[q];
      const int n = (int)m.N;
      const double* kq = mgk<double>(D, q);
      HM_CHECK(launch_identity(H.tmpA, n, p->s));
      for (int j = 0; j < n; ++j)
        HM_CHECK(launch_stencil<double>(m.op64, ST_APPLY, H.tmpA + (size_t)j * n, kq, nullptr,
                                        H.tmpB + (size_t)j * n, 0.0, p->s));
      std::vector<c128> cols((size_t)n * n);
      HM_CHECK(hipMemcpyAsync(cols.data(), H.tmpB, sizeof(c128) * cols.size(),
                              hipMemcpyDeviceToHost, p->s));
      HM_CHECK(hipStreamSynchronize(p->s));
      std::vector<cd> A((size_t)n * n);
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
          const c128 v = cols[(size_t)j * n + i];   // (M e_j)_i = M[i][j]
          A[(size_t)i * n + j] = cd(v.re, v.im);
        }
      invert_dense(A, n);
      std::vector<c128> up((size_t)n * n);
      for (size_t i = 0; i < up.size(); ++i) up[i] = mk(A[i].real(), A[i].imag());
      HM_CHECK(hipMemcpyAsync(H.inv, up.data(), sizeof(c128) * up.size(), hipMemcpyHostToDevice, p->s));
      HM_CHECK(hipStreamSynchronize(p->s));
    }
  }
  HM_CHECK(hipStreamSynchronize(p->s));
}

// ---- component access (tests) --------------------------------------------------------

template <typename T>
static const cx<T>* to_level(hm_problem* p, const c128* in, size_t n, void* tmp) {
  if constexpr (sizeof(T) == sizeof(double)) {
    (void)p; (void)n; (void)tmp;
    return (const cx<T>*)in;
  } else {
    HM_CHECK(launch_convert<double, float>(in, (c64*)tmp, n, p->s));
    return (const cx<T>*)tmp;
  }
}
template <typename T>
static cx<T>* out_level(c128* out, void* tmp) {
  if constexpr (sizeof(T) == sizeof(double)) { (void)tmp; return (cx<T>*)out; }
  else return (cx<T>*)tmp;
}
template <typename T>
static void from_level(hm_problem* p, const cx<T>* buf, c128* out, size_t n) {
  if constexpr (sizeof(T) == sizeof(double)) {
    if ((const void*)buf != (const void*)out)
      HM_CHECK(hipMemcpyAsync(out, buf, sizeof(c128) * n, hipMemcpyDeviceToDevice, p->s));
  } else {
    HM_CHECK(launch_convert<float, double>((const c64*)buf, out, n, p->s));
  }
}

template <typename T, typename Tn>
static void op_transfer(hm_problem* p, int l, int which, const c128* in, c128* out) {
  DefLevel& D = p->lev[l];
  DefLevel& C = p->lev[l + 1];
  if (which == HM_OP_ZT) {
    const cx<T>* v = to_level<T>(p, in, D.N, p->pin_v);
    cx<Tn>* o = out_level<Tn>(out, p->pin_x);
    HM_CHECK(launch_restrict_z<T, Tn>(v, D.nx, D.ny, o, p->cfg.bc, p->s));
    from_level<Tn>(p, o, out, C.N);
  } else {
    const cx<Tn>* v = to_level<Tn>(p, in, C.N, p->pin_v);
    cx<T>* o = out_level<T>(out, p->pin_x);
    HM_CHECK(launch_prolong_z<Tn, T>(v, D.nx, D.ny, o, p->cfg.bc, p->s));
    from_level<T>(p, o, out, D.N);
  }
}

template <typename T>
static void op_level(hm_problem* p, int l, int sub, int which, const c128* in, c128* out) {
  Ctx c(p);
  const Act one{0};
  DefLevel& D = p->lev[l];
  size_t nin = D.N, nout = D.N;
  if (which >= HM_OP_MG_M) {
    if (!D.has_mg || sub < 0 || sub >= (int)D.mg.lv.size()) throw ArgError("no such multigrid level");
    if ((which == HM_OP_MG_RESTRICT || which == HM_OP_MG_PROLONG) && sub + 1 >= (int)D.mg.lv.size())
      throw ArgError("no coarser multigrid level");
    nin = nout = D.mg.lv[sub].N;
    if (which == HM_OP_MG_RESTRICT) nout = D.mg.lv[sub + 1].N;
    if (which == HM_OP_MG_PROLONG) nin = D.mg.lv[sub + 1].N;
  }
  const cx<T>* v = to_level<T>(p, in, nin, p->pin_v);
  cx<T>* o = out_level<T>(out, p->pin_x);
  switch (which) {
    case HM_OP_A: apply_level<T>(c, one, D, false, ST_APPLY, v, nullptr, o); break;
    case HM_OP_M: apply_level<T>(c, one, D, true, ST_APPLY, v, nullptr, o); break;
    case HM_OP_VCYCLE: {
      if (!D.has_mg) throw ArgError("level has no multigrid hierarchy");
      const cx<T>* src = v;
      if (D.rt) {                       // the preconditioner's buffer: graph path
        HM_CHECK(hipMemcpyAsync(D.rt, v, sizeof(cx<T>) * D.N, hipMemcpyDeviceToDevice, p->s));
        src = (const cx<T>*)D.rt;
      }
      const cx<T>* r = vcycle<T>(c, one, D, src);
      HM_CHECK(hipMemcpyAsync(o, r, sizeof(cx<T>) * D.N, hipMemcpyDeviceToDevice, p->s));
      break;
    }
    case HM_OP_CSLP: {
      const cx<T>* r = cslp_apply<T>(c, one, l, v, o);
      if (r != o) HM_CHECK(hipMemcpyAsync(o, r, sizeof(cx<T>) * D.N, hipMemcpyDeviceToDevice, p->s));
      break;
    }
    case HM_OP_PRECOND:
      if (l >= p->L) throw ArgError("no preconditioner on the coarsest level");
      precond<T>(c, one, l, v, o);
      break;
    case HM_OP_MG_M: {
      const MGLevel& m = D.mg.lv[sub];
      HM_CHECK(launch_stencil<T>(mgop<T>(m), ST_APPLY, v, mgk<T>(D, sub), nullptr, o, T(0), p->s));
      break;
    }
    case HM_OP_MG_JACOBI: {
      const MGLevel& m = D.mg.lv[sub];
      HM_CHECK(launch_jacobi0<T>(mgop<T>(m), mgk<T>(D, sub), v, o, (T)m.omega, p->s));
      break;
    }
    case HM_OP_MG_RESTRICT: {
      const MGLevel& m = D.mg.lv[sub];
      HM_CHECK(launch_restrict_fw<T>(v, m.nx, m.ny, o, p->cfg.bc, p->s));
      break;
    }
    case HM_OP_MG_PROLONG: {
      const MGLevel& m = D.mg.lv[sub];
      HM_CHECK(launch_zero<T>(o, m.N, p->s));
      HM_CHECK(launch_prolong_bilinear_add<T>(v, m.nx, m.ny, o, p->cfg.bc, p->s));
      break;
    }
    default: throw ArgError("unknown operator");
  }
  from_level<T>(p, o, out, nout);
}

template <typename F>
static hm_status guard(F&& f) {
  try {
    return f();
  } catch (const ArgError& e) {
    g_last_error = e.what();
    return HM_ERR_ARG;
  } catch (const HipError& e) {
    g_last_error = e.what();
    return HM_ERR_HIP;
  } catch (const BasisError& e) {
    g_last_error = e.what();
    return HM_ERR_BASIS;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return HM_ERR_NOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return HM_ERR_STATE;
  }
}

// Planned sizes of one problem: workspace bytes, and the pinned staging the
// problem needs (entries of host / host_coef, and of the Hessenberg mirror).
struct Sizes {
  size_t bytes = 0;
  int host_cap = 0;
  size_t host_H_cap = 0;
  int coef_cap = 0;
};

static Sizes plan_sizes(const hm_config& cfg, bool batch_io) {
  hm_problem tmp;
  tmp.cfg = cfg;
  tmp.batch_io = batch_io;
  Carver cv;
  plan(&tmp, cv);
  Sizes z;
  z.bytes = (cv.off + 255) & ~size_t(255);
  z.coef_cap = tmp.coef_cap;
  z.host_cap = std::max(tmp.coef_cap, 16);
  z.host_H_cap = std::max<size_t>(tmp.host_H_cap, 1);
  return z;
}

static size_t host_stride(const Sizes& z) {
  const size_t b = sizeof(c128) * (2 * (size_t)z.host_cap + z.host_H_cap);
  return (b + 255) & ~size_t(255);
}

// A problem on the workspace at `base`.  host_block: pinned staging laid out as
// host | host_coef | Hessenberg mirror, given by a batch (null: allocated here).
static hm_problem* make_problem(const hm_config& cfg, char* base, hipStream_t stream,
                                bool batch_io, char* host_block, const double* k_dev) {
  hm_problem* p = new hm_problem();
  try {
    p->cfg = cfg;
    p->s = stream;
    p->batch_io = batch_io;
    Carver cv;
    cv.base = base;
    plan(p, cv);
    p->host_cap = std::max(p->coef_cap, 16);
    const size_t hcap = std::max<size_t>(p->host_H_cap, 1);
    if (host_block) {
      p->own_host = false;
      p->host = (c128*)host_block;
      p->host_coef = p->host + p->host_cap;
      p->host_H = p->host_coef + p->host_cap;
    } else {
      HM_CHECK(hipHostMalloc((void**)&p->host, sizeof(c128) * p->host_cap, hipHostMallocDefault));
      HM_CHECK(hipHostMalloc((void**)&p->host_coef, sizeof(c128) * p->host_cap,
                             hipHostMallocDefault));
      HM_CHECK(hipHostMalloc((void**)&p->host_H, sizeof(c128) * hcap, hipHostMallocDefault));
    }
    HM_CHECK(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
    HM_CHECK(hipEventCreateWithFlags(&p->col_ev[0], hipEventDisableTiming));
    HM_CHECK(hipEventCreateWithFlags(&p->col_ev[1], hipEventDisableTiming));
    initialize(p, k_dev);
  } catch (...) {
    hm_destroy_problem(p);
    throw;
  }
  return p;
}

}  // namespace hm

// A batch: members with one configuration, member i's workspace i * dz bytes
// after member 0's, the coefficient rows after the last member.
struct hm_batch {
  std::vector<hm_problem*> mem;
  long long dz = 0, hz = 0;
  char* host_block = nullptr;   // pinned staging of all members, hz apart
  c128* coef = nullptr;         // device, nb rows of coef_ld
  c128* host_coef = nullptr;    // pinned, the same rows
  size_t coef_ld = 0;
};

// ================================ C ABI ======================================

extern "C" {

void hm_default_config(hm_config* c, int nx, int ny, double h) {
  if (!c) return;
  std::memset(c, 0, sizeof(*c));
  c->nx = nx; c->ny = ny; c->h = h;
  c->bc = HM_BC_SOMMERFELD;
  c->beta1 = 1.0; c->beta2 = 0.5;
  c->levels = 3;
  c->tol_outer = 1e-6; c->tol_level2 = 0.3; c->tol_cslp = 0.1; c->maxit_coef = 6.0;
  c->outer_restart = 30; c->outer_maxit = 300; c->level2_maxit = 100;
  c->mg_nu_pre = 1; c->mg_nu_post = 1;
  c->precision = HM_FP64;
  c->coarse_steps = 1; c->tol_levels = 2;
}

size_t hm_workspace_bytes(const hm_config* cfg) {
  std::string why;
  if (!validate(cfg, &why)) {
    g_last_error = why;
    return 0;
  }
  try {
    hm_problem tmp;
    tmp.cfg = *cfg;
    Carver cv;
    plan(&tmp, cv);
    return cv.off;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return 0;
  }
}

hm_status hm_create_problem(const hm_config* cfg, const double* k_dev, void* workspace,
                            size_t workspace_bytes, void* stream, hm_problem** out) {
  if (out) *out = nullptr;
  return guard([&]() -> hm_status {
    std::string why;
    if (!out) throw ArgError("out is null");
    if (!validate(cfg, &why)) throw ArgError(why);
    if (!k_dev || !workspace) throw ArgError("null device pointer");
    if (((uintptr_t)workspace) & 255) throw ArgError("workspace must be 256-byte aligned");
    const size_t need = hm_workspace_bytes(cfg);
    if (workspace_bytes < need) {
      g_last_error = "workspace too small: need " + std::to_string(need) + " bytes";
      return HM_ERR_NOMEM;
    }
    *out = make_problem(*cfg, (char*)workspace, (hipStream_t)stream, false, nullptr, k_dev);
    return HM_OK;
  });
}

hm_status hm_precond_apply(hm_problem* p, const void* v_dev, void* x_dev, void* stream) {
  return guard([&]() -> hm_status {
    if (!p || !v_dev || !x_dev) throw ArgError("null argument");
    if (v_dev == x_dev) throw ArgError("v and x must not alias");
    p->s = (hipStream_t)stream;
    Ctx c(p);
    precond_top(c, Act{0}, (const c128*)v_dev, (c128*)x_dev);
    HM_CHECK(hipStreamSynchronize(p->s));
    return HM_OK;
  });
}

hm_status hm_fgmres_solve(hm_problem* p, const void* b_dev, void* u_dev, hm_solve_info* info,
                          void* stream) {
  return guard([&]() -> hm_status {
    if (!p || !b_dev || !u_dev) throw ArgError("null argument");
    if (b_dev == u_dev) throw ArgError("b and u must not alias");
    p->s = (hipStream_t)stream;
    Ctx c(p);
    return outer_solve(c, (const c128*)b_dev, (c128*)u_dev, info);
  });
}

hm_status hm_apply_operator(hm_problem* p, int level, int sub, int which, const void* in_dev,
                            void* out_dev, void* stream) {
  return guard([&]() -> hm_status {
    if (!p || !in_dev || !out_dev) throw ArgError("null argument");
    if (level < 1 || level > p->L) throw ArgError("level out of range");
    if (in_dev == out_dev) throw ArgError("in and out must not alias");
    p->s = (hipStream_t)stream;
    const bool dbl = p->lev[level].dbl;
    if (which == HM_OP_ZT || which == HM_OP_Z) {
      if (level >= p->L) throw ArgError("no coarser deflation level");
      const bool dn = p->lev[level + 1].dbl;
      if (dbl && dn) op_transfer<double, double>(p, level, which, (const c128*)in_dev, (c128*)out_dev);
      else if (!dbl && dn) op_transfer<float, double>(p, level, which, (const c128*)in_dev, (c128*)out_dev);
      else if (!dbl && !dn) op_transfer<float, float>(p, level, which, (const c128*)in_dev, (c128*)out_dev);
      else throw ArgError("unsupported precision layout");
    } else if (dbl) {
      op_level<double>(p, level, sub, which, (const c128*)in_dev, (c128*)out_dev);
    } else {
      op_level<float>(p, level, sub, which, (const c128*)in_dev, (c128*)out_dev);
    }
    HM_CHECK(hipStreamSynchronize(p->s));
    return HM_OK;
  });
}

hm_status hm_level_shape(const hm_problem* p, int level, int sub, int* nx, int* ny) {
  if (!p || !nx || !ny || level < 1 || level > p->L) return HM_ERR_ARG;
  const DefLevel& D = p->lev[level];
  if (sub == 0) {
    *nx = D.nx; *ny = D.ny;
    return HM_OK;
  }
  if (!D.has_mg || sub < 0 || sub >= (int)D.mg.lv.size()) return HM_ERR_ARG;
  *nx = D.mg.lv[sub].nx;
  *ny = D.mg.lv[sub].ny;
  return HM_OK;
}

hm_status hm_set_replay(hm_problem* p, int kind, const int* counts, int n) {
  if (!p || kind < 0 || kind >= K_NKIND || n < 0 || (n > 0 && !counts)) return HM_ERR_ARG;
  p->rep[kind].assign(counts, counts + n);
  p->rep_pos[kind] = 0;
  return HM_OK;
}

hm_status hm_get_counts(const hm_problem* p, int kind, int* counts, int cap, int* n) {
  if (!p || kind < 0 || kind >= K_NKIND || !n || cap < 0 || (cap > 0 && !counts)) return HM_ERR_ARG;
  const std::vector<int>& r = p->rec[kind];
  *n = (int)r.size();
  for (int i = 0; i < cap && i < (int)r.size(); ++i) counts[i] = r[i];
  return HM_OK;
}

hm_status hm_reset_counts(hm_problem* p) {
  if (!p) return HM_ERR_ARG;
  for (int k = 0; k < K_NKIND; ++k) {
    p->rec[k].clear();
    p->rep_pos[k] = 0;
  }
  return HM_OK;
}

hm_status hm_destroy_problem(hm_problem* p) {
  if (!p) return HM_ERR_ARG;
  for (auto& q : p->pending) p->pool.push_back({q.a, q.b});
  for (auto& e : p->pool) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  for (auto& D : p->lev)
    for (auto& g : D.mg.graphs) (void)hipGraphExecDestroy(g.second);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  for (auto& e : p->col_ev)
    if (e) (void)hipEventDestroy(e);
  if (p->own_host) {
    if (p->host_H) (void)hipHostFree(p->host_H);
    if (p->host) (void)hipHostFree(p->host);
    if (p->host_coef) (void)hipHostFree(p->host_coef);
  }
  delete p;
  return HM_OK;
}

size_t hm_batch_workspace_bytes(const hm_config* cfg, int nb) {
  std::string why;
  if (!validate(cfg, &why)) {
    g_last_error = why;
    return 0;
  }
  if (nb < 1 || nb > kMaxBatch) {
    g_last_error = "batch size must be in [1, " + std::to_string(kMaxBatch) + "]";
    return 0;
  }
  try {
    const Sizes z = plan_sizes(*cfg, true);
    const size_t rows = ((size_t)nb * z.coef_cap * sizeof(c128) + 255) & ~size_t(255);
    return (size_t)nb * z.bytes + rows;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return 0;
  }
}

hm_status hm_create_batch(const hm_config* cfg, int nb, const double* const* k_dev,
                          void* workspace, size_t workspace_bytes, void* stream, hm_batch** out) {
  if (out) *out = nullptr;
  return guard([&]() -> hm_status {
    std::string why;
    if (!out) throw ArgError("out is null");
    if (!validate(cfg, &why)) throw ArgError(why);
    if (nb < 1 || nb > kMaxBatch)
      throw ArgError("batch size must be in [1, " + std::to_string(kMaxBatch) + "]");
    if (!k_dev || !workspace) throw ArgError("null pointer");
    for (int i = 0; i < nb; ++i)
      if (!k_dev[i]) throw ArgError("null wavenumber pointer");
    if (((uintptr_t)workspace) & 255) throw ArgError("workspace must be 256-byte aligned");
    const size_t need = hm_batch_workspace_bytes(cfg, nb);
    if (workspace_bytes < need) {
      g_last_error = "workspace too small: need " + std::to_string(need) + " bytes";
      return HM_ERR_NOMEM;
    }
    const Sizes z = plan_sizes(*cfg, true);
    hm_batch* bt = new hm_batch();
    try {
      bt->dz = (long long)z.bytes;
      bt->hz = (long long)host_stride(z);
      bt->coef_ld = (size_t)z.coef_cap;
      bt->coef = (c128*)((char*)workspace + (size_t)nb * z.bytes);
      HM_CHECK(hipHostMalloc((void**)&bt->host_block, (size_t)nb * bt->hz, hipHostMallocDefault));
      HM_CHECK(hipHostMalloc((void**)&bt->host_coef, sizeof(c128) * nb * bt->coef_ld,
                             hipHostMallocDefault));
      for (int i = 0; i < nb; ++i)
        bt->mem.push_back(make_problem(*cfg, (char*)workspace + (size_t)i * z.bytes,
                                       (hipStream_t)stream, true,
                                       bt->host_block + (size_t)i * bt->hz, k_dev[i]));
      // one layout: every pointer of member i is member 0's plus i * dz
      for (int i = 1; i < nb; ++i)
        if ((char*)bt->mem[i]->uu - (char*)bt->mem[0]->uu != (long long)i * bt->dz ||
            (char*)bt->mem[i]->host_H - (char*)bt->mem[0]->host_H != (long long)i * bt->hz)
          throw std::logic_error("batch members differ in layout");
    } catch (...) {
      hm_destroy_batch(bt);
      throw;
    }
    *out = bt;
    return HM_OK;
  });
}

hm_status hm_batch_solve(hm_batch* bt, const void* const* b_dev, void* const* u_dev,
                         hm_solve_info* info, void* stream) {
  return guard([&]() -> hm_status {
    if (!bt || !b_dev || !u_dev) throw ArgError("null argument");
    const int nb = (int)bt->mem.size();
    for (int i = 0; i < nb; ++i) {
      if (!b_dev[i] || !u_dev[i]) throw ArgError("null vector pointer");
      if (b_dev[i] == u_dev[i]) throw ArgError("b and u must not alias");
    }
    hipStream_t s = (hipStream_t)stream;
    for (hm_problem* q : bt->mem) q->s = s;
    hm_problem* p = bt->mem[0];
    const size_t bytes = sizeof(c128) * p->lev[1].N;
    for (int i = 0; i < nb; ++i)
      HM_CHECK(hipMemcpyAsync(bt->mem[i]->ub, b_dev[i], bytes, hipMemcpyDeviceToDevice, s));
    Ctx c(p);
    c.mem = bt->mem;
    c.dz = bt->dz;
    c.hz = bt->hz;
    c.coef = bt->coef;
    c.host_coef = bt->host_coef;
    c.coef_ld = bt->coef_ld;
    const hm_status st = outer_solve(c, p->ub, p->uu, info);
    for (int i = 0; i < nb; ++i)
      HM_CHECK(hipMemcpyAsync(u_dev[i], bt->mem[i]->uu, bytes, hipMemcpyDeviceToDevice, s));
    HM_CHECK(hipStreamSynchronize(s));
    return st;
  });
}

hm_problem* hm_batch_member(hm_batch* bt, int i) {
  if (!bt || i < 0 || i >= (int)bt->mem.size()) return nullptr;
  return bt->mem[i];
}

hm_status hm_destroy_batch(hm_batch* bt) {
  if (!bt) return HM_ERR_ARG;
  for (hm_problem* q : bt->mem) hm_destroy_problem(q);
  if (bt->host_block) (void)hipHostFree(bt->host_block);
  if (bt->host_coef) (void)hipHostFree(bt->host_coef);
  delete bt;
  return HM_OK;
}

static bool matvec_grid_ok(int nx, int ny, double h) {
  if (nx < 3 || ny < 3 || !(h > 0) || !std::isfinite(h)) {
    g_last_error = "matvec: need nx, ny >= 3 and h > 0";
    return false;
  }
  if ((long long)nx * ny * 5 > 2147483647LL) {
    g_last_error = "matvec: 5*nx*ny exceeds the 32-bit index range";
    return false;
  }
  return true;
}

hm_status hm_matfree_apply(int nx, int ny, double h, const double* k_dev, const void* u_dev,
                           void* v_dev, void* stream) {
  if (!matvec_grid_ok(nx, ny, h)) return HM_ERR_ARG;
  if (!k_dev || !u_dev || !v_dev) return HM_ERR_ARG;
  return guard([&]() -> hm_status {
    OpDesc<double> d;
    set_five_point(d, nx, ny, h, 1.0, cd(1.0, 0.0), HM_BC_SOMMERFELD);
    HM_CHECK(launch_stencil(d, ST_APPLY, (const c128*)u_dev, k_dev, (const c128*)nullptr,
                            (c128*)v_dev, 0.0, (hipStream_t)stream));
    return HM_OK;
  });
}

hm_status hm_csr_assemble(int nx, int ny, double h, const double* k_dev, int* row_ptr_dev,
                          int* col_idx_dev, void* vals_dev, void* stream) {
  if (!matvec_grid_ok(nx, ny, h)) return HM_ERR_ARG;
  if (!k_dev || !row_ptr_dev || !col_idx_dev || !vals_dev) return HM_ERR_ARG;
  return guard([&]() -> hm_status {
    OpDesc<double> d;
    set_five_point(d, nx, ny, h, 1.0, cd(1.0, 0.0), HM_BC_SOMMERFELD);
    HM_CHECK(launch_csr5_assemble(d, k_dev, row_ptr_dev, col_idx_dev, (c128*)vals_dev,
                                  (hipStream_t)stream));
    return HM_OK;
  });
}

hm_status hm_csr_spmv(int nrows, int ncols, const int* row_ptr_dev, const int* col_idx_dev,
                      const void* vals_dev, const void* x_dev, void* y_dev, void* stream) {
  if (nrows < 0 || ncols < 0 || !row_ptr_dev || !col_idx_dev || !vals_dev || !x_dev || !y_dev) {
    g_last_error = "csr_spmv: bad arguments";
    return HM_ERR_ARG;
  }
  if (nrows == 0) return HM_OK;
  return guard([&]() -> hm_status {
    HM_CHECK(launch_csr_spmv(nrows, ncols, row_ptr_dev, col_idx_dev, (const c128*)vals_dev,
                             (const c128*)x_dev, (c128*)y_dev, (hipStream_t)stream));
    return HM_OK;
  });
}

size_t hm_residual_workspace_bytes(void) { return sizeof(c128) * (size_t)kMaxChunks; }

// Arguments of the true-residual entry points; false (with the message set)
// when one is invalid.
static bool residual_args_ok(int nx, int ny, double h, int bc, const double* k_dev,
                             const void* b_dev, const void* u_dev, const void* r_dev,
                             const double* norms_dev) {
  if (nx < 3 || ny < 3 || !(h > 0) || !std::isfinite(h)) {
    g_last_error = "residual: need nx, ny >= 3 and h > 0";
    return false;
  }
  if (bc != HM_BC_SOMMERFELD && bc != HM_BC_DIRICHLET) {
    g_last_error = "residual: unknown boundary condition";
    return false;
  }
  if (!k_dev || !b_dev || !u_dev || !norms_dev) {
    g_last_error = "residual: null pointer";
    return false;
  }
  if (r_dev && r_dev == u_dev) {
    g_last_error = "residual: r must not alias u";
    return false;
  }
  return true;
}

static hm_status residual_launch(int nx, int ny, double h, int bc, const double* k_dev,
                                 const void* b_dev, const void* u_dev, void* r_dev,
                                 double* norms_dev, c128* partials, void* stream) {
  return guard([&]() -> hm_status {
    OpDesc<double> d;
    set_five_point(d, nx, ny, h, 1.0, cd(1.0, 0.0), bc);
    HM_CHECK(launch_residual_norm(d, (const c128*)u_dev, k_dev, (const c128*)b_dev, (c128*)r_dev,
                                  partials, norms_dev, (hipStream_t)stream));
    return HM_OK;
  });
}

hm_status hm_residual(int nx, int ny, double h, int bc, const double* k_dev, const void* b_dev,
                      const void* u_dev, void* r_dev, double* norms_dev, void* workspace,
                      size_t workspace_bytes, void* stream) {
  if (!residual_args_ok(nx, ny, h, bc, k_dev, b_dev, u_dev, r_dev, norms_dev)) return HM_ERR_ARG;
  if (!workspace || ((uintptr_t)workspace & 255)) {
    g_last_error = "residual: workspace must be a 256-byte aligned device pointer";
    return HM_ERR_ARG;
  }
  if (workspace_bytes < hm_residual_workspace_bytes()) {
    g_last_error = "residual: workspace smaller than hm_residual_workspace_bytes()";
    return HM_ERR_NOMEM;
  }
  return residual_launch(nx, ny, h, bc, k_dev, b_dev, u_dev, r_dev, norms_dev, (c128*)workspace,
                         stream);
}

hm_status hm_residual_noalloc(int nx, int ny, double h, int bc, const double* k_dev,
                              const void* b_dev, const void* u_dev, void* r_dev,
                              double* norms_dev, void* stream) {
  if (!residual_args_ok(nx, ny, h, bc, k_dev, b_dev, u_dev, r_dev, norms_dev)) return HM_ERR_ARG;
  return guard([&]() -> hm_status {
    c128* partials = nullptr;
    size_t cap = 0;
    HM_CHECK(scratch_address(&partials, &cap));
    const size_t need = sizeof(c128) * (size_t)reduction_chunks((size_t)nx * (size_t)ny);
    if (need > cap) {
      g_last_error = "residual_noalloc: the reduction needs " + std::to_string(need) +
                     " bytes of scratch, the static array holds " + std::to_string(cap);
      return HM_ERR_ARG;
    }
    return residual_launch(nx, ny, h, bc, k_dev, b_dev, u_dev, r_dev, norms_dev, partials, stream);
  });
}

hm_status hm_set_timing(hm_problem* p, unsigned mask, int every) {
  if (!p || every < 1) return HM_ERR_ARG;
  return guard([&]() -> hm_status {
    HM_CHECK(hipStreamSynchronize(p->s));
    harvest(p);
    p->timing_mask = mask;
    p->timing_every = every;
    for (int c = 0; c < HM_TK_COUNT; ++c) {
      p->t_ms[c] = 0;
      p->t_bytes[c] = 0;
      p->t_launches[c] = 0;
      p->timing_seen[c] = 0;
    }
    return HM_OK;
  });
}

hm_status hm_set_basis_cache(hm_problem* p, double basis_bytes, double recent_bytes) {
  if (!p || std::isnan(basis_bytes) || std::isnan(recent_bytes)) return HM_ERR_ARG;
  const CachePolicy def;
  p->cache.basis = basis_bytes < 0 ? def.basis : basis_bytes;
  p->cache.recent = recent_bytes < 0 ? def.recent : recent_bytes;
  return HM_OK;
}

hm_status hm_set_small_krylov(hm_problem* p, int enable) {
  if (!p) return HM_ERR_ARG;
  p->small_krylov = enable != 0;
  return HM_OK;
}

hm_status hm_set_krylov_steps(hm_problem* p, int steps) {
  if (!p || steps < 1 || steps > HM_KRYLOV_STEPS_MAX) return HM_ERR_ARG;
  p->krylov_steps = steps;
  return HM_OK;
}

hm_status hm_get_timing(const hm_problem* p, int cls, double* ms, double* bytes, long* launches) {
  if (!p || cls < 0 || cls >= HM_TK_COUNT || !ms || !bytes || !launches) return HM_ERR_ARG;
  *ms = p->t_ms[cls];
  *bytes = p->t_bytes[cls];
  *launches = p->t_launches[cls];
  return HM_OK;
}

const char* hm_status_string(hm_status s) {
  switch (s) {
    case HM_OK: return "ok";
    case HM_NOT_CONVERGED: return "not converged";
    case HM_ERR_ARG: return "invalid argument";
    case HM_ERR_NOMEM: return "workspace too small";
    case HM_ERR_HIP: return "HIP error";
    case HM_ERR_STATE: return "invalid state";
    case HM_ERR_BASIS: return "level-2 basis exhausted";
  }
  return "unknown status";
}

const char* hm_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
