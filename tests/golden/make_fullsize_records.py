"""Writes the oracle's records of the full-size workloads into tests/golden/.

The FP64 oracle needs minutes to tens of minutes per solve at these sizes, too
long to run inside a test, so this script runs it once and stores what the GPU
tests compare against.  It calls only `oracle/` (and `workloads/` for the
seeded inputs); no value comes from the GPU library.

Records (numpy .npz, loaded with allow_pickle=False):

  solve_<name>.npz      MADP-preconditioned FGMRES (Algorithm 1, Sec. 4.4
                        configuration, outer tolerance 1e-6 of Sec. 4):
                        outer step count, the level-2 FGMRES counts and the
                        coarsest Krylov-CSLP counts in call order, the Krylov-
                        CSLP steps of every coarse level summed, the true
                        relative residual, ||u||_2, max|u| and the solution on
                        every `stride`-th node in x and y (u[j, i] with i, j
                        multiples of the stride).
  precond_<name>.npz    one application of the level-1 preconditioner
                        (Algorithm 1 loop body) to a seeded complex normal
                        vector (`random`), or to the first outer Krylov vector
                        b / ||b|| of the solve (`rhs`): the inner counts it took
                        (replayed on the GPU to make the preconditioner the
                        same fixed map), max|x|, ||x||_2 and the output on the
                        strided nodes.

Usage:  python tests/golden/make_fullsize_records.py [case ...]
        cases: cfg1_solve cfg1_precond cfg1_precond_rhs cfg3_solve six_level_k400
        (default: all)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads                                   # noqa: E402
from oracle.krylov import CountLog                 # noqa: E402
from oracle.madp import MADP                       # noqa: E402

# seed of the preconditioner input; the GPU test draws the same vector
PRECOND_SEED = 20241205


def precond_input(p, source, seed=PRECOND_SEED):
    """The preconditioner input of a record: a seeded complex normal vector, or
    the first outer Krylov vector b / ||b|| (zero initial guess)."""
    if source == "rhs":
        b = p.rhs()
        return b / np.linalg.norm(b)
    rng = np.random.default_rng(seed)
    n = p.nx * p.ny
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def strided(x, nx, ny, stride):
    return np.ascontiguousarray(x.reshape(ny, nx)[::stride, ::stride]).ravel()


def _meta():
    return dict(threads=np.int64(os.cpu_count() or 0),
                omp=np.bytes_(os.environ.get("OMP_NUM_THREADS", "")))


def record_solve(name, p, levels=3, stride=32, shot=0):
    t0 = time.perf_counter()
    o = MADP(p.nx, p.ny, p.h, p.k, levels=levels)
    setup = time.perf_counter() - t0
    print("%s: set-up %.1f s" % (name, setup), flush=True)
    u, info = o.solve(p.rhs(shot))
    lg = o.log.data
    out = os.path.join(HERE, "solve_%s.npz" % name)
    np.savez(out, nx=np.int64(p.nx), ny=np.int64(p.ny), h=np.float64(p.h),
             levels=np.int64(levels), shot=np.int64(shot), stride=np.int64(stride),
             outer_iters=np.int64(info["outer_iters"]),
             level2_counts=np.asarray(lg.get("level2", []), dtype=np.int64),
             cslp_counts=np.asarray(lg.get("cslp_l%d" % levels, []), dtype=np.int64),
             cslp_total=np.int64(sum(sum(v) for key, v in lg.items() if key.startswith("cslp_l"))),
             mg_coarse_counts=np.asarray(lg.get("mg_coarse", []), dtype=np.int64),
             outer_counts=np.asarray(lg.get("outer", []), dtype=np.int64),
             rel_res_true=np.float64(info["rel_res_true"]),
             u_norm=np.float64(np.linalg.norm(u)), u_absmax=np.float64(np.max(np.abs(u))),
             u_sample=strided(u, p.nx, p.ny, stride),
             seconds=np.float64(info["seconds"]), setup_seconds=np.float64(setup), **_meta())
    print("%s: outer %d, level-2 %d, cslp %d, rel. residual %.3e, %.1f s -> %s" % (
        name, info["outer_iters"], info["level2_iters_total"], info["cslp_iters_total"],
        info["rel_res_true"], info["seconds"], out), flush=True)


def record_precond(name, p, levels=3, stride=32, source="random"):
    t0 = time.perf_counter()
    o = MADP(p.nx, p.ny, p.h, p.k, levels=levels)
    setup = time.perf_counter() - t0
    v = precond_input(p, source)
    o.log = CountLog("record")
    t0 = time.perf_counter()
    x = o.apply(v)
    sec = time.perf_counter() - t0
    lg = o.log.data
    out = os.path.join(HERE, "precond_%s.npz" % name)
    np.savez(out, nx=np.int64(p.nx), ny=np.int64(p.ny), h=np.float64(p.h),
             levels=np.int64(levels), stride=np.int64(stride), seed=np.int64(PRECOND_SEED),
             source=np.bytes_(source),
             level2_counts=np.asarray(lg.get("level2", []), dtype=np.int64),
             cslp_counts=np.asarray(lg.get("cslp_l%d" % levels, []), dtype=np.int64),
             mg_coarse_counts=np.asarray(lg.get("mg_coarse", []), dtype=np.int64),
             x_norm=np.float64(np.linalg.norm(x)), x_absmax=np.float64(np.max(np.abs(x))),
             x_sample=strided(x, p.nx, p.ny, stride),
             seconds=np.float64(sec), setup_seconds=np.float64(setup), **_meta())
    print("%s: precond counts level2 %s cslp %s, %.1f s -> %s" % (
        name, lg.get("level2"), lg.get("cslp_l%d" % levels), sec, out), flush=True)


CASES = {
    # k = 200 on 4097 x 4097 (constant medium, centre source), FP64 method
    "cfg1_solve": lambda: record_solve("constant_k200_4097", workloads.config(1)),
    "cfg1_precond": lambda: record_precond("constant_k200_4097", workloads.config(1)),
    "cfg1_precond_rhs": lambda: record_precond("constant_k200_4097_rhs", workloads.config(1),
                                               source="rhs"),
    # layered-and-faulted stand-in, 4597 x 1453, f = 20 Hz, first surface shot
    "cfg3_solve": lambda: record_solve("layered_f20_shot0", workloads.config(3), stride=16),
    # six-level MADP, constant k = 400 on 641 x 641 (the single-process run of
    # the weak-scaling study, Sec. 5)
    "six_level_k400": lambda: record_solve("constant_k400_641_six_levels",
                                           workloads.constant(639, 400.0), levels=6, stride=8),
}


if __name__ == "__main__":
    names = sys.argv[1:] or list(CASES)
    for n in names:
        CASES[n]()
