/*
 * helmdefl.h -- C ABI of the MI355X (gfx950) implementation of the matrix-free
 * multilevel deflation preconditioner (MADP) inside flexible GMRES for the
 * heterogeneous 2-D Helmholtz equation  -Lap u - k(x,y)^2 u = b
 * (Chen, Dwarka, Vuik, arXiv 2412.04980).
 *
 * Problem statement (Sec. 2 and 2.1 of the paper): rectangle, vertex-centred
 * uniform grid of nx*ny nodes INCLUDING the boundary nodes, spacing h, 5-point
 * second-order finite differences, first-order Sommerfeld radiation condition on
 * all four sides imposed through the ghost point u_ghost = u_mirror + 2 i h k u_b
 * (eq. ghost_sommerfeld), or a homogeneous Dirichlet condition (hm_bc).  The
 * outer solver is FGMRES from a zero initial guess stopping at
 * ||b - A u||_2 / ||b||_2 <= tol_outer (Sec. 4); the preconditioner
 * is MADP (Sec. 4.4): Algorithm 1 applied recursively over `levels` levels with
 * the CSLP  M = -Lap - (beta1 + i beta2) k^2  (eq. CSLP def) approximated by one
 * multigrid V-cycle on levels 1-2 and by GMRES on coarser levels, the
 * Galerkin-derived re-discretised coarse stencils of Sec. 3.3 and the
 * higher-order (quadratic Bezier) deflation vectors.
 *
 * Conventions for every entry point
 *   Layout     node (i, j), 0 <= i < nx (x), 0 <= j < ny (y), index j*nx + i
 *              (x fastest).  Complex vectors are interleaved (re, im) pairs of
 *              double (complex128) -- the layout of torch.complex128.
 *   Ownership  the caller allocates and owns every device buffer (wavenumber
 *              field, right-hand side, solution, workspace).  The library never
 *              allocates or frees device memory.  It allocates a small host
 *              object (hm_problem) and pinned host staging memory, released by
 *              hm_destroy_problem.  The workspace must outlive the problem.
 *   Streams    every call takes a hipStream_t (as void*; NULL = default stream)
 *              and enqueues its work there.  Calls whose control flow depends on
 *              device results (Krylov stopping tests) synchronise that stream;
 *              all others are asynchronous.  A problem must be used from one
 *              stream at a time.
 *   Errors     return codes only.  < 0: nothing was written to the output;
 *              > 0: output written with a warning (e.g. not converged).
 *              hm_last_error() returns a message for the calling thread.
 */
#ifndef HELMDEFL_H
#define HELMDEFL_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hm_problem hm_problem;

typedef enum {
  HM_OK = 0,
  HM_NOT_CONVERGED = 1,   /* output written; tolerance not met within maxit       */
  HM_ERR_ARG = -1,        /* invalid argument (size, pointer, parameter)          */
  HM_ERR_NOMEM = -2,      /* workspace smaller than hm_workspace_bytes()          */
  HM_ERR_HIP = -3,        /* a HIP runtime call or kernel launch failed           */
  HM_ERR_STATE = -4,      /* call not valid in the problem's current state        */
  HM_ERR_BASIS = -5       /* a level-2 solve needed more basis vectors than the
                             problem reserves (hm_config.level2_basis)            */
} hm_status;

/* Boundary condition on all four sides (Sec. 2.1).  HM_BC_DIRICHLET is the
 * homogeneous condition u = 0: boundary nodes keep their place in the grid with
 * decoupled rows d_b u_b (d_b = s_l 4 / h_l^2), no other row reads them, the
 * coarse-level stencils use the ghost value 2 u_b - u_m = -u_m with ghost
 * wavenumber 2 k_b - k_m one step outside (eq. ghost_Dirichlt, Sec. 3.3), and
 * every grid transfer is masked to the interior.  Right-hand sides must vanish
 * on the boundary; the solution then does too. */
typedef enum { HM_BC_SOMMERFELD = 0, HM_BC_DIRICHLET = 1 } hm_bc;

/* Precision of the preconditioner (the outer FGMRES is FP64 in every mode).  The
 * paper computes in FP64 throughout; the mixed modes are this library's.
 * HM_MIXED_FP32 keeps the coarsest problem (the solve on the deepest deflation
 * level, Sec. 4.1) in FP64; HM_MIXED_FP32_ALL runs it in FP32 as well.
 * Reductions accumulate in FP64 throughout, and the dense coarsest multigrid
 * inverse is applied in FP64 in every mode.  In HM_MIXED_FP32 the coarsest
 * multigrid level of levels 1-2, where it is too large for the dense inverse,
 * is solved by FP64 GMRES on cast copies of its right-hand side and solution. */
typedef enum {
  HM_FP64 = 0,          /* every step in complex128                                   */
  HM_MIXED_FP32 = 1,    /* preconditioner levels 1-2 in complex64 with FP32 arithmetic;
                           outer FGMRES (Arnoldi/MGS, Givens, true residual) and the
                           coarsest-level solve (levels >= 3) in complex128           */
  HM_MIXED_FP32_ALL = 2 /* every preconditioner level, the coarsest-level solve
                           included, in complex64 with FP32 arithmetic; outer FGMRES
                           in complex128                                               */
} hm_precision;

typedef struct {
  int nx, ny;            /* nodes incl. boundary; (n-1) divisible by 2^(levels-1)   */
  double h;              /* mesh width                                              */
  int bc;                /* hm_bc                                                   */
  double beta1, beta2;   /* CSLP shift (Sec. 3.1); MADP uses (1, 0.5) (Sec. 4.4)     */
  int levels;            /* deflation levels, >= 2 (MADP default 3)                 */
  double tol_outer;      /* outer relative residual (Sec. 4: 1e-6)                  */
  double tol_level2;     /* level-2 FGMRES relative tolerance (Sec. 4.4: 0.3)       */
  double tol_cslp;       /* Krylov CSLP relative tolerance (Sec. 4.2: 0.1)          */
  double maxit_coef;     /* Krylov CSLP step cap floor(coef * N^(1/4)) (Sec. 4.2: 6) */
  int outer_restart;     /* outer FGMRES restart length (30)                        */
  int outer_maxit;       /* outer FGMRES total step cap (300)                       */
  int level2_maxit;      /* level-2 FGMRES step cap (100)                           */
  int mg_nu_pre, mg_nu_post;  /* Jacobi sweeps of the CSLP V-cycle (1, 1)           */
  int precision;         /* hm_precision                                            */
  int coarse_steps;      /* m: FGMRES steps on every coarse level solved without a
                            tolerance, the coarsest always (Sec. 3.2, cycle type:
                            1 = V-cycle, the MADP setting; 2 = W-cycle); 1..16      */
  int tol_levels;        /* levels 2..tol_levels (above the coarsest) iterate to
                            tol_level2 with at most level2_maxit steps: 2 = MADP;
                            1 = every coarse level takes coarse_steps; 3-4 = the
                            tolerance on the third/fourth levels too (Sec. 4.5)   */
  int cslp_orth;         /* orthogonalisation of the GMRES that approximates the
                            CSLP inverse on levels >= 3 (and the GMRES coarsest
                            multigrid solves): HM_ORTH_CLASSICAL (default, two
                            passes over the basis per step) or HM_ORTH_MODIFIED
                            (the modified Gram-Schmidt of Algorithm 1, j+1
                            passes per step); same Krylov space and iterates in
                            exact arithmetic                                       */
  int level2_basis;      /* level-2 FGMRES basis vectors reserved in the workspace:
                            0 = level2_maxit (default), else 1..level2_maxit.  A
                            smaller basis shrinks the workspace (by 2 level-2
                            vectors per step); a level-2 solve that reaches it
                            before its tolerance and level2_maxit stops the call
                            with HM_ERR_BASIS, and the caller re-creates the
                            problem with a larger basis.  A call that succeeds
                            returns the same results whatever the basis        */
  int reserved[4];       /* must be zero                                            */
} hm_config;

enum { HM_ORTH_CLASSICAL = 0, HM_ORTH_MODIFIED = 1 };

typedef struct {
  int outer_iters;             /* outer FGMRES steps                                 */
  int level2_iters_total;      /* level-2 FGMRES steps summed over the solve         */
  int cslp_iters_total;        /* Krylov CSLP steps on the coarsest level, summed     */
  int mg_coarse_iters_total;   /* GMRES steps of multigrid coarsest solves, summed    */
  double rel_res_estimate;     /* last Givens estimate |g_{m+1}| / ||b||             */
  double rel_res_true;         /* ||b - A u|| / ||b|| recomputed in FP64             */
  double seconds;              /* wall time of the call (host clock)                 */
} hm_solve_info;

/* Fills *cfg with the MADP configuration of Sec. 4.4 for an nx x ny grid of
 * spacing h: 3 levels, beta = (1, 0.5), tolerances 1e-6 / 0.3 / 0.1, cap
 * coefficient 6, restart 30, outer cap 300, level-2 cap 100, V(1,1), FP64. */
void hm_default_config(hm_config* cfg, int nx, int ny, double h);

/* Device workspace bytes a problem with this configuration needs (256-byte
 * aligned start required).  Returns 0 if the configuration is invalid. */
size_t hm_workspace_bytes(const hm_config* cfg);

/* Builds the level hierarchy (Sec. 3.3: sizes n_l = (n-1)/2^(l-1)+1, spacings
 * 2^(l-1) h, wavenumber injected to coarse grids) and the multigrid
 * sub-hierarchies of levels 1-2 inside `workspace`.
 *   k_dev: device, nx*ny doubles, the nodal wavenumber k = 2 pi f / c >= 0
 *          (Sec. 2, eq. wavenum); read during the call only.
 *   workspace: device, >= hm_workspace_bytes(cfg) bytes, 256-byte aligned.
 * Errors: HM_ERR_ARG for invalid cfg or pointers, for a non-finite or negative
 * k (checked on the device), or for k = 0 at every node with Sommerfeld
 * boundaries (the operator is then the Neumann Laplacian, which is singular;
 * with Dirichlet boundaries k = 0 is the Poisson problem and is accepted);
 * HM_ERR_NOMEM for a short workspace.
 * Synchronises `stream`. */
hm_status hm_create_problem(const hm_config* cfg, const double* k_dev, void* workspace,
                            size_t workspace_bytes, void* stream, hm_problem** out);

/* One application of the finest-level MADP preconditioner x = P v (Algorithm 1
 * loop body at level 1: Z^T, recursive coarse FGMRES, Z, A, CSLP V-cycle, x=r+t).
 *   v_dev, x_dev: device, nx*ny complex128, must not alias.
 * Synchronises `stream` (inner Krylov stopping tests). */
hm_status hm_precond_apply(hm_problem* p, const void* v_dev, void* x_dev, void* stream);

/* Solves A u = b by MADP-preconditioned FGMRES (Algorithm 1 at level 1 with
 * restarts), zero initial guess.  b_dev, u_dev: device, nx*ny complex128, no
 * aliasing.  info may be NULL.  Returns HM_NOT_CONVERGED (u written) when the
 * tolerance is not met within outer_maxit steps. */
hm_status hm_fgmres_solve(hm_problem* p, const void* b_dev, void* u_dev, hm_solve_info* info,
                          void* stream);

/* Component access for parity tests.  Applies one building block in the
 * problem's precision, reading and writing complex128 device vectors:
 *   HM_OP_A        level operator: 5-point Helmholtz A (level 1, eq. helm
 *                  operator h) or re-discretised E_l (l >= 2, Sec. 3.3)  N_l -> N_l
 *   HM_OP_M        CSLP of the level (same stencils, shifted k^2 term)    N_l -> N_l
 *   HM_OP_ZT       deflation restriction Z^T, level -> level+1           N_l -> N_{l+1}
 *   HM_OP_Z        deflation interpolation Z, level+1 -> level           N_{l+1} -> N_l
 *   HM_OP_VCYCLE   one multigrid V-cycle for M_l (levels 1-2)             N_l -> N_l
 *   HM_OP_CSLP     the level's CSLP approximation (V-cycle or GMRES)      N_l -> N_l
 *   HM_OP_PRECOND  the level-l MADP preconditioner (Algorithm 1 body)     N_l -> N_l
 *   HM_OP_MG_M     multigrid-level operator of M_l at multigrid level sub
 *   HM_OP_MG_JACOBI  one damped-Jacobi sweep from zero at multigrid level sub
 *   HM_OP_MG_RESTRICT full weighting, multigrid level sub -> sub+1
 *   HM_OP_MG_PROLONG  bilinear interpolation, multigrid level sub+1 -> sub
 * `level` is 1-based; `sub` selects the multigrid level (0 = top) for the
 * HM_OP_MG_* operations and is ignored otherwise.  Synchronises `stream` for the
 * Krylov-based operations. */
enum {
  HM_OP_A = 0, HM_OP_M = 1, HM_OP_ZT = 2, HM_OP_Z = 3, HM_OP_VCYCLE = 4, HM_OP_CSLP = 5,
  HM_OP_PRECOND = 6, HM_OP_MG_M = 7, HM_OP_MG_JACOBI = 8, HM_OP_MG_RESTRICT = 9,
  HM_OP_MG_PROLONG = 10
};
hm_status hm_apply_operator(hm_problem* p, int level, int sub, int which, const void* in_dev,
                            void* out_dev, void* stream);

/* Grid shape of deflation level `level` (1-based) and multigrid level `sub`
 * below it (sub = 0: the deflation level itself).  HM_ERR_ARG if absent. */
hm_status hm_level_shape(const hm_problem* p, int level, int sub, int* nx, int* ny);

/* Fixed-count (replay) mode for parity tests.  kind: 0 = level-2 FGMRES,
 * 1 = coarsest-level Krylov CSLP, 2 = multigrid coarsest GMRES, 3 = outer
 * FGMRES cycles.  After hm_set_replay, each inner solve of that kind takes
 * exactly the next count (tolerance test off), making the preconditioner a
 * fixed map; n = 0 switches replay off.  hm_get_counts copies the counts
 * recorded since the last hm_reset_counts (at most cap) and stores the total
 * number recorded in *n. */
hm_status hm_set_replay(hm_problem* p, int kind, const int* counts, int n);
hm_status hm_get_counts(const hm_problem* p, int kind, int* counts, int cap, int* n);
hm_status hm_reset_counts(hm_problem* p);

/* Kernel timing for roofline measurements.  hm_set_timing(p, mask, every)
 * resets the counters and, for every kernel class whose bit is set in mask,
 * brackets every `every`-th launch of that class (the 1st, (every+1)-th, ...)
 * with HIP events on the problem's stream; mask 0 turns it off.  Each bracket
 * costs a few microseconds of device time, so sampling (every > 1) keeps the
 * measured run close to an untimed one.  hm_get_timing returns, for one class,
 * the summed event time in milliseconds of the bracketed launches, their summed
 * algorithmic bytes (each input array read once, each output written once) and
 * their number. */
enum {
  HM_TK_CGS_DOT = 0,     /* Krylov CSLP: dots of w against the basis (classical GS)    */
  HM_TK_CGS_UPDATE = 1,  /* Krylov CSLP: w -= V h fused with ||w||                       */
  HM_TK_WIDE = 2,        /* 5x5 / 7x7 coarse-level operator applications in Krylov loops  */
  HM_TK_FIVE_POINT = 3,  /* 5-point operator applications in Krylov loops                  */
  HM_TK_MGS = 4,         /* modified Gram-Schmidt steps (outer and level-2 FGMRES)        */
  HM_TK_COUNT = 5
};
hm_status hm_set_timing(hm_problem* p, unsigned mask, int every);
hm_status hm_get_timing(const hm_problem* p, int cls, double* ms, double* bytes, long* launches);

/* Load hints of the two Gram-Schmidt passes of the Krylov CSLP (GMRES with
 * classical Gram-Schmidt, the coarsest-level CSLP approximation of Sec. 4.2 /
 * 4.4).  A basis of (m+1) vectors plus w of at most basis_bytes is read with
 * plain loads, which keep it in the 256 MB Infinity Cache between the passes;
 * a larger one reads its most recent vectors, recent_bytes of them, with plain
 * loads and the older ones with the non-temporal hint.  Defaults 256 MiB and
 * 200 MiB; a negative value restores a default.  The arithmetic and the
 * results are the same for every setting: this is a tuning hook, and it lets
 * small problems run the large-basis code path.  HM_ERR_ARG for NaN or a null
 * problem. */
hm_status hm_set_basis_cache(hm_problem* p, double basis_bytes, double recent_bytes);

/* Device-resident Krylov solves on small coarse levels (the GMRES of the Krylov
 * CSLP, Sec. 4.2, and GMRES coarsest multigrid solves): on a level of at most
 * 1600 nodes whose ghost-extended copy fits in LDS (the 33 x 33 coarsest level
 * of a 129^2 problem), each member's whole GMRES (operator, Gram-Schmidt,
 * Givens rotations, stopping test, back substitution, x = V y) runs in one
 * workgroup, with one launch and one host wait per solve instead of several
 * launches and a wait per step.  Larger levels stay host-driven: there one
 * compute unit streaming the basis is slower than the device-wide steps.
 * The same method and stopping rule (reading R11); rounding differs from the
 * host-driven path in the order of the sums.  enable = 1 (default) or 0 (every
 * level host-driven).  HM_ERR_ARG for a null problem. */
hm_status hm_set_small_krylov(hm_problem* p, int enable);

/* Arnoldi steps per two passes over the basis in the classical Gram-Schmidt
 * GMRES of the Krylov CSLP (Sec. 4.2) on FP64 levels that are not solved in one
 * workgroup.  With steps = S > 1, the block of steps j..j+S-1 applies M to v_j
 * and then S - 1 more times (Y_0 = M v_j, Y_{k+1} = M Y_k); one pass over the
 * basis takes the inner products of [V_0..V_j, Y] with Y, classical
 * Gram-Schmidt runs on the device in the coordinates of [V_0..V_j, Y] (M acting
 * on V through the Hessenberg columns already formed), and a second pass forms
 * v_{j+1}..v_{j+S-1} and the last step's new vector.  The iterates are those of
 * one-step classical Gram-Schmidt in exact arithmetic (reading R18); the basis
 * is read 2/S times per step instead of twice.  FP32 levels keep one step per
 * two passes (the coordinate relations hold only to the basis's
 * orthogonality).  steps: 1 (one step per two passes), 2 or
 * HM_KRYLOV_STEPS_MAX = 3 (default).  HM_ERR_ARG for a null problem or another
 * count. */
#define HM_KRYLOV_STEPS_MAX 3
hm_status hm_set_krylov_steps(hm_problem* p, int steps);

hm_status hm_destroy_problem(hm_problem* p);

/* ---- Lockstep batches: several problems of one configuration per launch -----
 * A batch holds nb (1..16) problems that share one configuration (grid, h,
 * levels, precision, tolerances) but each have their own wavenumber field and
 * right-hand side: several sources in one medium, or several media of one
 * size.  hm_batch_solve runs MADP-FGMRES (Algorithm 1 with the Sec. 4.4
 * configuration, as hm_fgmres_solve) for all members together: every kernel
 * launch sweeps the same level for all members still iterating (one launch,
 * members along the grid's third dimension), while each member keeps its own
 * Krylov least-squares problems and stopping tests on the host.  A member that
 * has met a tolerance drops out of the launches of that solve, so each
 * member's result and step counts are exactly those of hm_fgmres_solve on its
 * own, bit for bit.
 *   hm_batch_workspace_bytes: device bytes for nb members (0 if cfg is invalid
 *     or nb is out of range).
 *   hm_create_batch: k_dev[i] is member i's nodal wavenumber (device, nx*ny
 *     doubles, read during the call); workspace as for hm_create_problem, sized
 *     by hm_batch_workspace_bytes.  Synchronises `stream`.  Errors as
 *     hm_create_problem, plus HM_ERR_ARG for nb outside 1..16.
 *   hm_batch_solve: b_dev[i], u_dev[i] are member i's right-hand side and
 *     solution (device, nx*ny complex128, b_dev[i] != u_dev[i]); info: nb
 *     records or NULL.  Returns HM_NOT_CONVERGED if any member misses the
 *     tolerance (all solutions written).  Synchronises `stream`.
 *   hm_batch_member: member i as a problem handle (counts, replay, timing;
 *     the batch's kernel timing is kept by member 0), or NULL.  Owned by the
 *     batch; it may also be solved on its own with hm_fgmres_solve.
 *   hm_destroy_batch: frees the batch and its members, not the workspace. */
typedef struct hm_batch hm_batch;
size_t hm_batch_workspace_bytes(const hm_config* cfg, int nb);
hm_status hm_create_batch(const hm_config* cfg, int nb, const double* const* k_dev,
                          void* workspace, size_t workspace_bytes, void* stream, hm_batch** out);
hm_status hm_batch_solve(hm_batch* bt, const void* const* b_dev, void* const* u_dev,
                         hm_solve_info* info, void* stream);
hm_problem* hm_batch_member(hm_batch* bt, int i);
hm_status hm_destroy_batch(hm_batch* bt);

/* ---- Matrix-free versus stored-matrix matvec (Appendix B, Table of the
 * matrix-free / CSR comparison) ----------------------------------------------
 * Both forms compute v = A u for the finest-level operator of eq. (helm
 * operator h): the 5-point Helmholtz stencil -Laplace_h - k^2 on an nx x ny
 * node grid with spacing h, first-order Sommerfeld ghosts on all four sides
 * (Sec. 2).  Row-major node order p = y*nx + x; u, v complex128 (interleaved
 * re, im), k float64 per node, all device pointers owned by the caller.
 * nx, ny >= 3; nx*ny*5 must fit in a 32-bit int (grids up to 20723^2).
 * Asynchronous on `stream` (NULL = the default stream); HM_ERR_ARG for bad
 * sizes or null pointers, HM_ERR_HIP for a failed launch.  They need no
 * problem object.
 *
 * hm_matfree_apply: v = A u straight from the stencil (per node: u and its four
 *   neighbours, k, one write).
 * hm_csr_assemble: writes A in CSR form: row_ptr (nx*ny+1 ints), col_idx
 *   (5*nx*ny ints), vals (5*nx*ny complex128).  Every row holds exactly five
 *   entries (centre, west, east, south, north); at a boundary the ghost's
 *   coupling is folded into the mirrored neighbour and the freed slot holds an
 *   explicit zero whose column is the row itself.
 * hm_csr_spmv: y = A x for any CSR matrix with 32-bit indices: nrows rows,
 *   ncols columns, x holds ncols entries, y nrows; row_ptr must be
 *   non-decreasing with row_ptr[nrows] entries in col_idx and vals.  An entry
 *   whose column lies outside [0, ncols) is not read from x: its row's result
 *   is NaN.  Rows are staged per block through LDS. */
hm_status hm_matfree_apply(int nx, int ny, double h, const double* k_dev, const void* u_dev,
                           void* v_dev, void* stream);
hm_status hm_csr_assemble(int nx, int ny, double h, const double* k_dev, int* row_ptr_dev,
                          int* col_idx_dev, void* vals_dev, void* stream);
hm_status hm_csr_spmv(int nrows, int ncols, const int* row_ptr_dev, const int* col_idx_dev,
                      const void* vals_dev, const void* x_dev, void* y_dev, void* stream);

/* ---- True residual (the stopping test of Sec. 4) ------------------------------
 * r = b - A u and its norm for the finest-level operator of eq. (helm operator
 * h): the 5-point Helmholtz stencil -Laplace_h - k^2 on an nx x ny node grid of
 * spacing h with boundary condition bc (hm_bc: Sommerfeld ghosts or the
 * decoupled Dirichlet rows), in FP64.  The relative residual of a solution is
 * norms[0] / norms[1], the quantity FGMRES stops on (Sec. 4: 1e-6).
 *   k_dev: nx*ny doubles; b_dev, u_dev: nx*ny complex128; all device, read only.
 *   r_dev: nx*ny complex128 written with b - A u, or NULL (norms only); it
 *          may be b_dev but not u_dev.
 *   norms_dev: device, 2 doubles: ||b - A u||_2, ||b||_2 (written by the call).
 *   workspace: device, >= hm_residual_workspace_bytes() bytes, 256-byte
 *          aligned: the reduction's partial sums (no state is kept there).
 * One pass over u, k and b (neighbours from cache) plus a fixed-order sum of
 * at most 2048 partials, so the result is bitwise reproducible.  Asynchronous
 * on `stream`; HM_ERR_ARG for bad sizes, pointers, aliasing or alignment,
 * HM_ERR_NOMEM for a short workspace, HM_ERR_HIP for a failed launch. */
size_t hm_residual_workspace_bytes(void);
hm_status hm_residual(int nx, int ny, double h, int bc, const double* k_dev, const void* b_dev,
                      const void* u_dev, void* r_dev, double* norms_dev, void* workspace,
                      size_t workspace_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * true residual as hm_residual, with the reduction's partial sums in a static
 * device array of the library (2048 complex128 = 32 KiB per device, held
 * until the process ends) instead of a caller workspace.  It calls no
 * allocating routine; the first call on a device looks the array's address
 * up once.  Every grid size fits the array (the reduction uses at most 2048
 * partials); a size that would not is rejected with HM_ERR_ARG.  All calls on
 * one device share the array: calls that overlap in time on one device (two
 * streams, two host threads) race and give wrong norms, so serialise them.
 * Each call writes every partial it reads, so nothing needs clearing.
 * Arguments, results and errors otherwise as hm_residual. */
hm_status hm_residual_noalloc(int nx, int ny, double h, int bc, const double* k_dev,
                              const void* b_dev, const void* u_dev, void* r_dev,
                              double* norms_dev, void* stream);

const char* hm_status_string(hm_status s);
const char* hm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HELMDEFL_H */
