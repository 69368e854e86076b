"""Benchmark: MADP-preconditioned FGMRES solves on one MI355X.

One step = one complete solve (outer FGMRES with the 3-level MADP
preconditioner, i.e. every hot-path kernel) of the constant-wavenumber
workload k = 200 on the unit square, 4097 x 4097 nodes (h = 1/4096,
k^3 h^2 = 0.48), Sommerfeld boundaries, point source at the centre, to
relative residual 1e-6, FP64.  Inputs (wavenumber field, right-hand side) are
resident in HBM before timing.  The same workload is also solved with the
mixed-precision preconditioner (FP32 levels 1-2) and reported beside it.

Prints one JSON line: solves/s (value), p50/p99 latency, the roofline of the
dominant kernel class measured with HIP events inside the timed region, and
the CPU oracle baseline (a bounded sample scaled to one solve).

    python bench.py [--steps K] [--warmup W] [--config I] [--no-mixed] [--no-cpu-baseline]

Other measurements, each one JSON line of its own:
    --serving      the request stream (Poisson arrivals, random media, 257^2..2049^2)
    --matvec       matrix-free vs CSR product of the finest operator, 17^2..16385^2
    --complexity   five-level MADP on the wedge stand-in at kh = 0.1745, 145x241..4609x7681
    --variants     MADP-v3, W-cycle, fixed steps and deeper hierarchies on the bench workload
    --shots        every right-hand side of --config I, sequential vs one lockstep batch
    --kernels      the component kernels of --config I one by one, with measured
                   copy / read-stream bandwidth ceilings
    --counter-table CSV...  per-kernel averages of rocprofv3 --pmc counter
                   collections; FETCH_SIZE / WRITE_SIZE scaled by the plain
                   copies of --copy-calibration MIB run in the same process
    --trace-table CSV   per-kernel, per-grid rates of the stencil and transfer
                   kernels from a rocprofv3 kernel trace of a --config I solve
                   (no GPU needed: reads the trace and prints a markdown table)
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E peak
TIMING_EVERY = 16
# calibrated hardware byte counts of the dominant kernel (two rocprofv3 --pmc
# passes, FETCH_SIZE and WRITE_SIZE, scaled by a plain copy of known size),
# taken on one workload (k = 200 on 4097^2, FP64); valid only for that
# workload and while the kernel source is unchanged
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "traffic_gmres_kernels.json")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2412_04980_amd", "csrc", "kernels.hip")


TRAFFIC_WORKLOAD = "constant_k200_4097"


def measured_traffic(kernel_class, workload):
    import hashlib
    if workload != TRAFFIC_WORKLOAD or not os.path.exists(TRAFFIC_RECORD):
        return None
    rec = json.load(open(TRAFFIC_RECORD))
    digest = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    if rec.get("kernels_hip_sha256") != digest or kernel_class not in rec["classes"]:
        return None
    return rec["classes"][kernel_class]["bytes_per_launch"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=1, help="workload index (0-3)")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-timing", action="store_true", help="no per-kernel event timing")
    ap.add_argument("--serving", action="store_true",
                    help="run the request-stream workload instead (Poisson arrivals of "
                         "solves on 257^2..2049^2 random media, FP32 preconditioner)")
    ap.add_argument("--requests", type=int, default=60)
    ap.add_argument("--serving-leg", type=int, default=24, metavar="N",
                    help="default line: also run the first N requests of the request stream "
                         "at --rate (0: skip)")
    ap.add_argument("--rate", type=float, default=50.0, help="offered requests/s")
    ap.add_argument("--max-active", type=int, default=8)
    ap.add_argument("--no-batching", action="store_true",
                    help="serving: one request per stream, no lockstep batches")
    ap.add_argument("--max-members", type=int, default=16,
                    help="serving: right-hand sides per lockstep batch (at most 16)")
    ap.add_argument("--matvec", action="store_true",
                    help="matrix-free versus CSR matvec of the finest operator on grids "
                         "17^2 .. 16385^2 (100 consecutive products per form and size)")
    ap.add_argument("--matvec-max-side", type=int, default=16385)
    ap.add_argument("--complexity", action="store_true",
                    help="five-level MADP on the wedge stand-in at kh = 0.1745, grids "
                         "145x241 (10 Hz) .. 4609x7681 (320 Hz), FP64 and mixed")
    ap.add_argument("--complexity-max-nx", type=int, default=4609)
    ap.add_argument("--variants", action="store_true",
                    help="the method variants (MADP-v3, W-cycle, fixed steps, tolerance on "
                         "level 3, 4 levels) on the benchmark workload, FP64")
    ap.add_argument("--shots", action="store_true",
                    help="all right-hand sides of the workload (config 3: 8 surface shots), "
                         "solved one after another and as one lockstep batch")
    ap.add_argument("--shots-precision", choices=("fp64", "mixed"), default="mixed")
    ap.add_argument("--kernels", action="store_true",
                    help="component kernels of the workload (every level operator, the "
                         "deflation and multigrid transfers, the V-cycles) timed one by one "
                         "through the C ABI, with a plain copy and a read-only stream as "
                         "measured bandwidth ceilings")
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--trace-table", metavar="CSV",
                    help="print the per-grid rates of the stencil and transfer kernels in a "
                         "rocprofv3 kernel-trace CSV of a --config I solve")
    ap.add_argument("--counter-table", nargs="+", metavar="CSV",
                    help="per-kernel averages of rocprofv3 --pmc counter CSVs (FETCH_SIZE and "
                         "WRITE_SIZE calibrated by the copies of --copy-calibration MIB)")
    ap.add_argument("--traffic-out", metavar="JSON",
                    help="counter table: also write the calibrated bytes per launch of the "
                         "Gram-Schmidt passes and the 7x7 scaled apply to this file")
    ap.add_argument("--trace-min-side", type=int, default=1025,
                    help="trace table: smallest grid side listed")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device-to-device three times (a plain copy "
                         "kernel of known size, to calibrate hardware byte counters)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed_solves(hm, torch, prob, b, steps, warmup, timing):
    u = torch.empty_like(b)
    for i in range(warmup):
        hm.fgmres_solve(prob, b, out=u)
        log("warmup solve %d done" % i)
    if timing:
        # bracket every 16th launch of each class: enough samples for the
        # averages, negligible event overhead in the timed solves
        hm.set_timing(prob, (1 << len(hm.TIMING_CLASSES)) - 1, TIMING_EVERY)
    torch.cuda.synchronize()
    lat, infos = [], []
    t_start = time.perf_counter()
    for i in range(steps):
        t0 = time.perf_counter()
        _, info = hm.fgmres_solve(prob, b, out=u)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
        infos.append(info)
        log("timed solve %d: %.3f s, outer %d" % (i, lat[-1], info["outer_iters"]))
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    kt = hm.get_timing(prob) if timing else {}
    if timing:
        hm.set_timing(prob, 0)
    return u, total, lat, infos, kt


def gs_hbm_share(counts, n, es, cls, steps=3):
    """Share of the algorithmic bytes of a Gram-Schmidt pass class that come from
    HBM under the cache-aware loads, estimated from the step counts of the
    coarsest-level Krylov CSLP solves (FP64: `steps` Arnoldi steps per pair of
    passes).  The block at step j reads m = j + 1 basis vectors in pass A (with
    the `steps` vectors M^r v_j) and again in pass B (with them, and `steps`
    vectors written).  When the basis exceeds the 256 MB plain-load limit, the
    vectors older than the 200 MB recent window come from HBM and the rest from
    the Infinity Cache; a smaller basis is cache-resident."""
    vec = float(n) * es
    recent = int(200.0 * 2**20 / vec)
    alg = hbm = 0.0
    for count in counts:
        for j in range(0, count, steps):
            m = j + 1
            alg += (m + steps if cls == "cgs_dot" else m + 2 * steps) * vec
            if (m + 1) * vec > 256.0 * 2**20:
                hbm += max(0, m - recent) * vec
    return hbm / alg if alg else None


def cpu_baseline(problem, info, counts_l3):
    """The oracle timed on a bounded sample of the same workload: its
    coarsest-level Krylov CSLP (GMRES, modified Gram-Schmidt, on the level-3
    grid) with the mean step count of the GPU solve, and one level-1 CSLP
    V-cycle; projected to one solve as (number of coarsest CSLP solves) x
    (GMRES time) + (outer steps) x (V-cycle time), a lower bound on the oracle's
    full solve (all other steps omitted).  BLAS limited to one thread."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import operators as op
    from oracle.krylov import fgmres
    from oracle.multigrid import VCycle

    with threadpool_limits(limits=1):
        nx, ny, h, k = problem.nx, problem.ny, problem.h, problem.k
        sigma = 1 + 0.5j
        k2 = op.inject(k, nx, ny)
        n2x, n2y = (nx - 1) // 2 + 1, (ny - 1) // 2 + 1
        k3 = op.inject(k2, n2x, n2y)
        n3x, n3y = (n2x - 1) // 2 + 1, (n2y - 1) // 2 + 1
        M3 = op.wide_stencil(n3x, n3y, h, 3, k3, sigma)
        m_mean = int(round(float(np.mean(counts_l3)))) if counts_l3 else 1
        rng = np.random.default_rng(0)
        r3 = rng.standard_normal(n3x * n3y) + 1j * rng.standard_normal(n3x * n3y)
        t0 = time.perf_counter()
        fgmres(lambda v: M3 @ v, r3, None, tol=None, maxit=m_mean)
        t_l3 = time.perf_counter() - t0
        log("oracle coarsest CSLP GMRES (%d steps): %.2f s" % (m_mean, t_l3))
        del M3
        M1 = op.five_point(nx, ny, h, k, sigma)
        V1 = VCycle(nx, ny, h, k, M1, sigma, 1.0)
        r1 = rng.standard_normal(nx * ny) + 0j
        t0 = time.perf_counter()
        V1(r1)
        t_v1 = time.perf_counter() - t0
        log("oracle level-1 V-cycle: %.2f s" % t_v1)
    n_l3 = len(counts_l3)
    t_solve = n_l3 * t_l3 + info["outer_iters"] * t_v1
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": 1.0 / t_solve, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "host_cpu": model, "host_cores": os.cpu_count(),
            "sample": "oracle (FP64, SciPy CSR, 1 BLAS thread) on this workload: one "
                      "coarsest-level CSLP GMRES of %d steps (%.2f s) and one level-1 "
                      "V-cycle (%.2f s), projected to one solve as %d x GMRES + %d x "
                      "V-cycle = %.1f s (lower bound: other steps omitted)"
                      % (m_mean, t_l3, t_v1, n_l3, info["outer_iters"], t_solve),
            "projected_seconds_per_solve": t_solve}


def serving_bench(args):
    print(json.dumps(run_serving(args, args.requests, args.rate)), flush=True)


def run_serving(args, n_requests, rate):
    import torch

    import workloads
    from paper_2412_04980_amd.serving import GpuExecutor, Scheduler, jobs_from_requests, summarize

    reqs = workloads.serving_stream(n_requests=n_requests, rate=rate, seed=4)
    jobs = jobs_from_requests(reqs)
    log("serving: %d requests, %d solves, offered %.1f req/s" %
        (len(jobs), sum(len(j.rhs) for j in jobs), rate))
    ex = GpuExecutor()
    free, _ = torch.cuda.mem_get_info()
    # admission budget: a margin below the free memory for the allocator's
    # rounding and for blocks cached at other sizes
    budget = int(0.7 * free)
    # warm-up: one small request per grid class, not timed
    seen = set()
    for j in jobs:
        if j.nx not in seen:
            seen.add(j.nx)
            one = type(j)(j.rid, 0.0, j.nx, j.ny, j.h, j.k, j.rhs[:1])
            ex(one) if args.no_batching else ex.run_group([one])
    torch.cuda.synchronize()
    last = [time.perf_counter()]

    def progress(done, total):
        # a line every 25 requests or 30 s, so a long run shows it is alive
        now = time.perf_counter()
        if done == total or done % 25 == 0 or now - last[0] > 30.0:
            last[0] = now
            log("serving: %d / %d requests done" % (done, total))

    if args.no_batching:
        sched = Scheduler(ex, ex.bytes_needed, budget, max_active=args.max_active, realtime=True,
                          progress=progress)
    else:
        # same-size requests waiting together run as one lockstep batch
        sched = Scheduler(ex.run_group, ex.group_bytes, budget, max_active=args.max_active,
                          realtime=True, group_key=ex.group_key,
                          max_members=min(args.max_members, 16), members=ex.members,
                          progress=progress)
    t0 = time.perf_counter()
    res = sched.run(jobs)
    wall = time.perf_counter() - t0
    summ = summarize(res, wall)
    by_class = {}
    for j, r in zip(jobs, res):
        c = by_class.setdefault("%dx%d" % (j.nx, j.ny), {"requests": 0, "latency_ms": []})
        c["requests"] += 1
        c["latency_ms"].append(r.latency * 1e3)
    import numpy as np
    for c in by_class.values():
        lat = np.array(c.pop("latency_ms"))
        c["p50_ms"], c["p99_ms"] = float(np.percentile(lat, 50)), float(np.percentile(lat, 99))
    out = {"metric": "serving: solves/s + p50/p99 request latency (FP32 preconditioner, FP64 "
                     "FGMRES, rel. residual 1e-6)",
           "value": summ["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
           "higher_is_better": True, "offered_requests_per_s": rate, "requests": len(jobs),
           "max_active": args.max_active, "budget_bytes": budget, "data": "synthetic",
           "batching": {"lockstep": not args.no_batching, "groups": len(sched.groups),
                        "mean_requests_per_group": len(jobs) / max(1, len(sched.groups)),
                        "max_members": 1 if args.no_batching else min(args.max_members, 16)},
           "config": {"workload": "serving stream (Poisson, random media, 257^2..2049^2)"},
           **summ, "by_grid": by_class,
           "max_concurrent": max(e[4] for e in sched.events),
           "level2_basis": {"%dx%d" % key[:2]: b for key, b in sorted(ex.basis.items())},
           "level2_basis_regrows": ex.regrows, "allocator_retries": ex.oom_retries}
    return out


def bandwidth_ceilings(torch, mib=1024, reps=20):
    """Measured ceilings on this GPU: a device-to-device copy (read + write) and
    a read-only stream (a sum over the array), both over `mib` MiB, in GB/s."""
    n = mib * (1 << 20) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    out = {}
    for name, fn, nbytes in (("copy_GBps", lambda: y.copy_(x), 2 * 8 * n),
                             ("read_GBps", lambda: x.sum(), 8 * n)):
        for _ in range(3):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        out[name] = nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    out["array_MiB"] = mib
    del x, y
    torch.cuda.empty_cache()
    return out


# Algorithmic bytes per grid point of the component kernels (each array read or
# written once; es = bytes of a complex value, kb of a wavenumber), on the grid
# named in the table (the fine grid of a transfer).
def _component_bytes(es, kb):
    return {"apply": 2 * es + kb, "deflation_restrict": es + es / 4,
            "deflation_prolong": es / 4 + es, "jacobi_first": 2 * es + kb,
            "full_weighting": es + es / 4, "prolong_bilinear_add+zero": es + es / 4 + 2 * es}


def kernels_bench(args):
    """Each component kernel of the workload's preconditioner applied R times in
    a row through the C ABI (hm_apply_operator) and timed with HIP events on the
    stream; bytes are algorithmic, rates are against the 8 TB/s peak and against
    the measured copy / read ceilings."""
    import ctypes

    import torch

    import paper_2412_04980_amd as hm
    import workloads
    dev = torch.device("cuda:0")
    problem = workloads.config(args.config)
    k = torch.from_numpy(problem.k).to(dev)
    ceil = bandwidth_ceilings(torch)
    log("ceilings: copy %.0f GB/s, read %.0f GB/s" % (ceil["copy_GBps"], ceil["read_GBps"]))
    rows = []
    for prec_name, prec in (("fp64", hm.HM_FP64), ("fp32", hm.HM_MIXED_FP32_ALL)):
        cfg = hm.default_config(problem.nx, problem.ny, problem.h, precision=prec)
        prob = hm.create_problem(cfg, k)
        es, kb = (16, 8) if prec == hm.HM_FP64 else (8, 4)
        per = _component_bytes(es, kb)
        ops = []
        for level in (1, 2, 3):
            ops.append((level, 0, hm.HM_OP_A, "apply", "A/E"))
            ops.append((level, 0, hm.HM_OP_M, "apply", "M (CSLP)"))
            if level < 3:
                ops.append((level, 0, hm.HM_OP_ZT, "deflation_restrict", "Z^T"))
                ops.append((level, 0, hm.HM_OP_Z, "deflation_prolong", "Z"))
                for sub in (0, 1):
                    ops.append((level, sub, hm.HM_OP_MG_JACOBI, "jacobi_first", "MG Jacobi (x=0)"))
                    ops.append((level, sub, hm.HM_OP_MG_RESTRICT, "full_weighting", "MG full weighting"))
                    ops.append((level, sub, hm.HM_OP_MG_PROLONG, "prolong_bilinear_add+zero",
                                "MG bilinear add (+ zero fill)"))
        stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        for level, sub, which, kind, label in ops:
            f = hm.level_shape(prob, level, sub)
            nf = f[0] * f[1]
            if which in (hm.HM_OP_ZT, hm.HM_OP_MG_RESTRICT):
                c = hm.level_shape(prob, level + 1, 0) if which == hm.HM_OP_ZT else \
                    hm.level_shape(prob, level, sub + 1)
                nin, nout = nf, c[0] * c[1]
            elif which in (hm.HM_OP_Z, hm.HM_OP_MG_PROLONG):
                c = hm.level_shape(prob, level + 1, 0) if which == hm.HM_OP_Z else \
                    hm.level_shape(prob, level, sub + 1)
                nin, nout = c[0] * c[1], nf
            else:
                nin = nout = nf
            x = torch.randn(nin, dtype=torch.complex128, device=dev)
            y = torch.empty(nout, dtype=torch.complex128, device=dev)
            call = lambda: hm._lib.hm_apply_operator(prob.handle, level, sub, which,
                                                     ctypes.c_void_p(x.data_ptr()),
                                                     ctypes.c_void_p(y.data_ptr()), stream)
            for _ in range(3):
                assert call() == 0
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(args.kernel_reps):
                call()
            e1.record()
            e1.synchronize()
            us = e0.elapsed_time(e1) * 1e3 / args.kernel_reps
            gbs = per[kind] * nf / (us * 1e-6) / 1e9
            row = {"precision": prec_name, "level": level, "mg_level": sub, "op": label,
                   "grid": "%dx%d" % f, "us": us, "GBps": gbs, "frac_of_peak": gbs / HBM_PEAK_GBS,
                   "frac_of_copy": gbs / ceil["copy_GBps"], "bytes_per_point": per[kind]}
            if prec_name == "fp32":
                row["note"] = "time includes the complex128 <-> complex64 casts of the test hook"
            rows.append(row)
            log("%s L%d/%d %-30s %-10s %8.1f us %7.0f GB/s %.2f" % (
                prec_name, level, sub, label, row["grid"], us, gbs, gbs / HBM_PEAK_GBS))
            del x, y
        prob.close()
        torch.cuda.empty_cache()
    out = {"metric": "component kernel rates (algorithmic bytes / event time)",
           "unit": "GB/s", "n_gpus": 1, "data": "synthetic", "reps": args.kernel_reps,
           "peak_GBps": HBM_PEAK_GBS, "ceilings": ceil,
           "config": {"workload": problem.name, "nx": problem.nx, "ny": problem.ny},
           "table": rows}
    print(json.dumps(out), flush=True)


# ---- per-grid rates from a rocprofv3 kernel trace ------------------------------

def _mg_sides(n):
    """Multigrid sides below an n-node side: halve while n - 1 is even and the
    coarse side keeps at least 3 nodes."""
    out = [n]
    while (n - 1) % 2 == 0 and (n - 1) // 2 + 1 >= 3:
        n = (n - 1) // 2 + 1
        out.append(n)
    return out


def _launch_shapes(nx, ny, levels):
    """Every (nx, ny) grid a solve of this hierarchy launches kernels on: the
    deflation levels and the multigrid levels below them."""
    shapes, x, y = set(), nx, ny
    for _ in range(levels):
        xs, ys = _mg_sides(x), _mg_sides(y)
        for i in range(min(len(xs), len(ys))):
            shapes.add((xs[i], ys[i]))
        x, y = (x - 1) // 2 + 1, (y - 1) // 2 + 1
    return shapes


# launch geometry of the stencil and transfer kernels, as the library computes
# it: block tiles of 64 x 4 threads (two rows per thread for the 5-point and
# wide kernels), eight-block XCD turns; transfers launch 256-thread blocks over
# 248 coarse columns and TRB coarse rows
def _ceil(a, b):
    return (a + b - 1) // b


def _xcd8(n):
    return 8 * _ceil(n, 8)


def _geometry(family, nx, ny, trb=None):
    if family == "five_point":
        return (64 * _xcd8(_ceil(nx, 64) * _ceil(ny, 8)), 4)
    if family == "wide_tiled":
        return (64 * _xcd8(_ceil(nx, 64) * _ceil(ny, 8)), 4)
    if family == "jacobi0":
        return (64 * _ceil(nx, 64), 4 * _ceil(ny, 4))
    if family in ("restrict", "prolong"):
        nxc, nyc = (nx - 1) // 2 + 1, (ny - 1) // 2 + 1
        return (256 * _xcd8(_ceil(nxc, 248) * _ceil(nyc, trb)), 1)
    return None


def _trace_kernel(name):
    """(family, label, bytes per fine point as a function of (es, kb), trb,
    fixed level) for the kernels of the table, else None."""
    import re
    m = re.search(r"k_(five_point|wide_tiled|wide_persist|jacobi0|restrict_rows|prolong_rows)"
                  r"<([^>]*)>", name)
    if not m:
        return None
    fam, targs = m.group(1), [a.strip() for a in m.group(2).split(",")]
    es = 16 if targs[0] == "double" else 8
    kb = es // 2
    mode_names = {0: "apply", 1: "resid", 2: "jacobi", 3: "scaled"}
    mode_bytes = {0: 2 * es + kb, 1: 3 * es + kb, 2: 3 * es + kb, 3: 3 * es + kb}
    if fam == "five_point":
        md = int(targs[1])
        return ("five_point", "k_five_point<%s,%s>" % (targs[0], mode_names[md]),
                mode_bytes[md], None, None)
    if fam in ("wide_tiled", "wide_persist"):
        r, md = int(targs[1]), int(targs[2])
        return (fam, "k_%s<%s,R=%d,%s>" % (fam, targs[0], r, mode_names[md]), mode_bytes[md],
                None, r)
    if fam == "jacobi0":
        return ("jacobi0", "k_jacobi0<%s,R=%s>" % (targs[0], targs[1]), 2 * es + kb, None, None)
    eo = 16 if targs[1] == "double" else 8
    trb = int(targs[3])
    if fam == "restrict_rows":
        kind = "Z^T" if targs[2] == "2" else "full weighting"
        return ("restrict", "restrict %s <%s,%s>" % (kind, targs[0], targs[1]),
                es + eo / 4.0, trb, None)
    zdef = targs[2] == "true"
    kind = "Z" if zdef else "bilinear add"
    return ("prolong", "prolong %s <%s,%s>" % (kind, targs[0], targs[1]),
            (es / 4.0 + eo) if zdef else (es / 4.0 + 2 * eo), trb, None)


def trace_table(args):
    """Average duration and algorithmic-byte rate of every stencil and transfer
    kernel of a solve, per grid, from the rocprofv3 kernel trace.  The grid of a
    launch is found from its launch geometry among the grids of the workload's
    hierarchy; the persistent wide stencils (whose block count follows the
    device's occupancy) are placed by their stencil radius: 5x5 on level 2,
    7x7 on level 3."""
    import csv

    import workloads
    problem = workloads.config(args.config)
    levels = 3
    shapes = _launch_shapes(problem.nx, problem.ny, levels)
    lvl = {l: ((problem.nx - 1) // 2 ** (l - 1) + 1, (problem.ny - 1) // 2 ** (l - 1) + 1)
           for l in range(1, levels + 1)}
    stats = {}
    with open(args.trace_table) as f:
        for row in csv.DictReader(f):
            kk = _trace_kernel(row["Kernel_Name"])
            if kk is None:
                continue
            fam, label, bpp, trb, radius = kk
            gx, gy = int(row["Grid_Size_X"]), int(row["Grid_Size_Y"])
            if fam == "wide_persist":
                cand = [lvl[radius]] if radius in lvl else []
            else:
                cand = [s for s in shapes if _geometry(fam, s[0], s[1], trb) == (gx, gy)]
            if len(cand) != 1:
                continue
            nx, ny = cand[0]
            us = (int(row["End_Timestamp"]) - int(row["Start_Timestamp"])) * 1e-3
            e = stats.setdefault((label, nx, ny), [0, 0.0, bpp])
            e[0] += 1
            e[1] += us
    print("| Kernel | Grid | Launches | Avg us | GB/s | of 8 TB/s |")
    print("|---|---:|---:|---:|---:|---:|")
    for (label, nx, ny), (n, tot, bpp) in sorted(stats.items(), key=lambda t: (-t[0][1], t[0][0])):
        if min(nx, ny) < args.trace_min_side:
            continue
        avg = tot / n
        gbs = bpp * nx * ny / (avg * 1e-6) / 1e9
        side = "%d^2" % nx if nx == ny else "%dx%d" % (nx, ny)
        print("| %s | %s | %d | %.1f | %.0f | %.2f |" % (label, side, n, avg, gbs,
                                                        gbs / HBM_PEAK_GBS))


# ---- per-kernel hardware counters from rocprofv3 --pmc collections -------------

def _short_kernel(name):
    import re
    name = re.sub(r"^void ", "", name)
    name = name.replace("hm::(anonymous namespace)::", "")
    depth, out = 0, []
    for ch in name:                      # drop the argument list
        if ch == "(" and depth == 0:
            break
        depth += ch == "<"
        depth -= ch == ">"
        out.append(ch)
    return "".join(out).strip()


# kernel classes of the bench line and the kernels each one times
TRAFFIC_CLASSES = {
    "cgs_dot": ("k_multidots<double, true, 3>", "k_multidots<double, false, 3>",
                "k_multidots<double, true, 2>", "k_multidots<double, false, 2>",
                "k_multidot<double, true>", "k_multidot<double, false>"),
    "cgs_update_norm": ("k_updates<double, true, 3>", "k_updates<double, false, 3>",
                        "k_updates<double, true, 2>", "k_updates<double, false, 2>",
                        "k_cgs_update_norm<double, true>", "k_cgs_update_norm<double, false>"),
    "wide_stencil_apply": ("k_wide_persist<double, 3, 3>",),
}


def counter_table(args):
    """Average of every counter per dispatch and kernel over the given rocprofv3
    counter-collection CSVs.  FETCH_SIZE and WRITE_SIZE (KiB) are also given
    as bytes scaled by what the same counter reads for the plain copies of
    --copy-calibration MiB that ran first in the profiled process (the largest
    copy dispatches); --traffic-out writes those bytes per launch for the
    kernel classes of the bench line."""
    import csv
    import hashlib
    from collections import defaultdict
    sums = defaultdict(lambda: defaultdict(float))
    disp = defaultdict(lambda: defaultdict(set))
    copies = defaultdict(list)
    for path in args.counter_table:
        with open(path) as f:
            for row in csv.DictReader(f):
                kname = _short_kernel(row["Kernel_Name"])
                cname, val = row["Counter_Name"], float(row["Counter_Value"])
                key = (path, row["Dispatch_Id"])
                if kname.startswith("__amd_rocclr_copyBuffer"):
                    copies[cname].append(val)
                    continue
                sums[kname][cname] += val
                disp[kname][cname].add(key)
    factor = {}
    if args.copy_calibration:
        true_kib = args.copy_calibration * 1024.0
        for cname in ("FETCH_SIZE", "WRITE_SIZE"):
            if copies.get(cname):
                big = sorted(copies[cname])[-3:]
                factor[cname] = (sum(big) / len(big)) / true_kib
    names = sorted({c for k in sums for c in sums[k]})
    print("| kernel | dispatches | " + " | ".join("%s / dispatch" % c for c in names) +
          "".join(" | %s MB (calibrated)" % c for c in names if c in factor) + " |")
    print("|---|---:|" + "---:|" * (len(names) + sum(1 for c in names if c in factor)))
    per = {}
    for k in sorted(sums):
        n = max(len(v) for v in disp[k].values())
        avg = {c: sums[k][c] / max(1, len(disp[k][c])) for c in names if c in sums[k]}
        per[k] = (n, avg)
        cells = ["%.1f" % avg[c] if c in avg else "" for c in names]
        cal = ["%.1f" % (avg[c] * 1024 / factor[c] / 1e6) if c in avg else ""
               for c in names if c in factor]
        print("| `%s` | %d | %s |" % (k, n, " | ".join(cells + cal)))
    if factor:
        print("\ncalibration: " + ", ".join("%s reads %.3f of the copied bytes" % (c, f)
                                          for c, f in factor.items()))
    if args.traffic_out and len(factor) == 2:
        classes = {}
        for cls, kernels in TRAFFIC_CLASSES.items():
            present = [k for k in kernels if k in per]
            if not present:
                continue
            n = sum(per[k][0] for k in present)
            fetch = sum(per[k][1].get("FETCH_SIZE", 0.0) * per[k][0] for k in present) / n
            write = sum(per[k][1].get("WRITE_SIZE", 0.0) * per[k][0] for k in present) / n
            classes[cls] = {"kernel": " + ".join(present), "fetch_kib_per_dispatch": fetch,
                            "write_kib_per_dispatch": write,
                            "bytes_per_launch": 1024 * (fetch / factor["FETCH_SIZE"] +
                                                        write / factor["WRITE_SIZE"])}
        rec = {"fetch_factor": factor["FETCH_SIZE"], "write_factor": factor["WRITE_SIZE"],
               "classes": classes,
               "kernels_hip_sha256": hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest(),
               "workload": "%s (FP64), one solve" % TRAFFIC_WORKLOAD}
        with open(args.traffic_out, "w") as f:
            json.dump(rec, f, indent=1)


# Per-row byte and flop counts of the two matvec forms (complex128 vectors,
# float64 wavenumber, 32-bit indices).  "compulsory": every array touched once
# (the HBM floor); "model": the per-row accounting of Appendix B (every value
# read per use, result read and written) with 16-byte complex values.
MATVEC_BYTES = {"matfree": {"compulsory": 16 + 8 + 16, "model": 5 * 16 + 8 + 16},
                "csr": {"compulsory": 5 * 16 + 5 * 4 + 4 + 16 + 16,
                        "model": 5 * (16 + 4 + 16) + 4 + 2 * 16}}
# matrix-free: k^2 and the centre coefficient (2), five real-by-complex
# products (10), four complex additions (8); CSR: five complex multiply-adds
MATVEC_FLOPS = {"matfree": 20, "csr": 40}


def matvec_bench(args, reps=100):
    import torch

    import paper_2412_04980_amd as hm
    dev = torch.device("cuda:0")
    gen = torch.Generator(device=dev)
    rows = []
    side = 17
    while side <= args.matvec_max_side:
        n = side * side
        h = 1.0 / (side - 1)
        gen.manual_seed(side)
        k = 20.0 + 40.0 * torch.rand(n, dtype=torch.float64, device=dev, generator=gen)
        u = torch.randn(n, dtype=torch.complex128, device=dev, generator=gen)
        v = torch.empty_like(u)
        y = torch.empty_like(u)
        rp, ci, va = hm.csr_assemble(side, side, h, k)
        times = {}
        for form in ("matfree", "csr"):
            def once():
                if form == "matfree":
                    hm.matfree_apply(side, side, h, k, u, out=v)
                else:
                    hm.csr_spmv(rp, ci, va, u, out=y)
            for _ in range(3):
                once()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(reps):
                once()
            e1.record()
            e1.synchronize()
            times[form] = e0.elapsed_time(e1) / reps
        diff = float((v - y).abs().max() / v.abs().max())
        row = {"side": side, "N": n, "max_rel_diff": diff}
        for form in ("matfree", "csr"):
            ms = times[form]
            row[form] = {"ms": ms,
                         "GBs": MATVEC_BYTES[form]["compulsory"] * n / ms / 1e6,
                         "GBs_model": MATVEC_BYTES[form]["model"] * n / ms / 1e6,
                         "GFLOPs": MATVEC_FLOPS[form] * n / ms / 1e6}
        row["time_ratio_csr_over_matfree"] = times["csr"] / times["matfree"]
        log("N=%11d  matfree %.4f ms %7.1f GB/s | csr %.4f ms %7.1f GB/s | ratio %.2f" % (
            n, times["matfree"], row["matfree"]["GBs"], times["csr"], row["csr"]["GBs"],
            row["time_ratio_csr_over_matfree"]))
        rows.append(row)
        del k, u, v, y, rp, ci, va
        torch.cuda.empty_cache()
        side = 2 * (side - 1) + 1
    big = rows[-1]
    out = {"metric": "matvec time, matrix-free vs CSR, complex FP64 5-point Sommerfeld operator",
           "value": big["time_ratio_csr_over_matfree"], "unit": "x (CSR time / matrix-free time)",
           "n_gpus": 1, "higher_is_better": True, "dtype": "f64", "data": "synthetic",
           "reps_per_size": reps,
           "bytes_per_row": MATVEC_BYTES, "flops_per_row": MATVEC_FLOPS,
           "roofline": {"bound": "hbm", "kernel": "matrix-free 5-point apply",
                        "N": big["N"], "achieved": big["matfree"]["GBs"],
                        "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": big["matfree"]["GBs"] / HBM_PEAK_GBS},
           "roofline_csr": {"bound": "hbm", "achieved": big["csr"]["GBs"], "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": big["csr"]["GBs"] / HBM_PEAK_GBS},
           "config": {"workload": "matvec sweep, square grids 17^2 .. %d^2, k uniform in "
                                  "[20, 60]" % rows[-1]["side"]},
           "table": rows}
    print(json.dumps(out), flush=True)


# Five-level wedge solves at kh = 0.1745 (the complexity study of Sec. 4.5):
# (nx, frequency); the domain is 600 m x 1000 m, so ny = (nx - 1) * 5 / 3 + 1.
COMPLEXITY_SIZES = [(145, 10.0), (289, 20.0), (577, 40.0), (1153, 80.0), (2305, 160.0),
                    (4609, 320.0)]


def complexity_bench(args):
    import torch

    import paper_2412_04980_amd as hm
    import workloads
    dev = torch.device("cuda:0")
    rows = []
    for nx, f in COMPLEXITY_SIZES:
        if nx > args.complexity_max_nx:
            break
        p = workloads.wedge(f=f, h=600.0 / (nx - 1))
        k = torch.from_numpy(p.k).to(dev)
        b = torch.from_numpy(p.rhs()).to(dev)
        row = {"nx": p.nx, "ny": p.ny, "unknowns": p.nx * p.ny, "f_hz": f}
        for label, prec in (("fp64", hm.HM_FP64), ("mixed", hm.HM_MIXED_FP32)):
            prob = hm.create_problem(hm.default_config(p.nx, p.ny, p.h, levels=5, precision=prec),
                                     k)
            try:
                u = torch.empty_like(b)
                hm.fgmres_solve(prob, b, out=u)           # warm-up (graph capture, caches)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, info = hm.fgmres_solve(prob, b, out=u)
                torch.cuda.synchronize()
                sec = time.perf_counter() - t0
            finally:
                prob.close()
            row[label] = {"seconds": sec, "outer_iters": info["outer_iters"],
                          "level2_iters_total": info["level2_iters_total"],
                          "rel_res_true": info["rel_res_true"]}
            log("%dx%d f=%g %s: %.3f s, outer %d, level-2 %d, rel_res %.2e" % (
                p.nx, p.ny, f, label, sec, info["outer_iters"], info["level2_iters_total"],
                info["rel_res_true"]))
        rows.append(row)
        del k, b, u
        torch.cuda.empty_cache()
    big = rows[-1]
    out = {"metric": "five-level MADP solve time, wedge stand-in at kh = 0.1745",
           "value": big["fp64"]["seconds"], "unit": "s per solve (largest grid, FP64)",
           "n_gpus": 1, "higher_is_better": False, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "wedge stand-in, 5 levels, kh = 0.1745, %dx%d .. %dx%d" % (
               rows[0]["nx"], rows[0]["ny"], big["nx"], big["ny"])},
           "table": rows}
    print(json.dumps(out), flush=True)


VARIANTS = [("MADP", {}),
            ("MADP-v3 (level-2 tol 0.1)", {"tol_level2": 0.1}),
            ("W-cycle (m = 2 on coarse levels)", {"coarse_steps": 2}),
            ("fixed m = 1 on every coarse level", {"tol_levels": 1}),
            ("4 levels", {"levels": 4}),
            ("4 levels, W-cycle", {"levels": 4, "coarse_steps": 2}),
            ("4 levels, tol 0.3 on levels 2-3", {"levels": 4, "tol_levels": 3}),
            ("5 levels", {"levels": 5}),
            ("6 levels", {"levels": 6}),
            ("modified Gram-Schmidt in the Krylov CSLP", {"cslp_orth": 1})]


def variants_bench(args):
    import torch

    import paper_2412_04980_amd as hm
    import workloads
    dev = torch.device("cuda:0")
    problem = workloads.config(args.config)
    k = torch.from_numpy(problem.k).to(dev)
    b = torch.from_numpy(problem.rhs(0)).to(dev)
    rows = []
    for name, kw in VARIANTS:
        cfg = hm.default_config(problem.nx, problem.ny, problem.h, **kw)
        prob = hm.create_problem(cfg, k)
        try:
            u = torch.empty_like(b)
            hm.fgmres_solve(prob, b, out=u)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info = hm.fgmres_solve(prob, b, out=u)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
        finally:
            prob.close()
        torch.cuda.empty_cache()
        rows.append({"variant": name, "settings": kw, "seconds": sec,
                     "outer_iters": info["outer_iters"],
                     "level2_iters_total": info["level2_iters_total"],
                     "cslp_iters_total": info["cslp_iters_total"],
                     "rel_res_true": info["rel_res_true"]})
        log("%-36s %.3f s  outer %d  level-2 %d  Krylov CSLP %d  rel_res %.2e" % (
            name, sec, info["outer_iters"], info["level2_iters_total"], info["cslp_iters_total"],
            info["rel_res_true"]))
    out = {"metric": "solve time per method variant", "value": rows[0]["seconds"],
           "unit": "s per solve (MADP)", "n_gpus": 1, "higher_is_better": False,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": problem.name, "nx": problem.nx, "ny": problem.ny},
           "table": rows}
    print(json.dumps(out), flush=True)


def shots_bench(args):
    """Every right-hand side of one medium: sequential solves on one problem against
    one lockstep batch of all of them (members share the medium).  The timed
    region of each leg holds every solve of its shots; one untimed pass first."""
    import numpy as np
    import torch

    import paper_2412_04980_amd as hm
    import workloads

    dev = torch.device("cuda:0")
    problem = workloads.config(args.config)
    nrhs = len(problem.sources)
    if nrhs > hm.MAX_BATCH:
        raise SystemExit("at most %d right-hand sides per batch" % hm.MAX_BATCH)
    prec = hm.HM_MIXED_FP32 if args.shots_precision == "mixed" else hm.HM_FP64
    cfg = hm.default_config(problem.nx, problem.ny, problem.h, precision=prec)
    k = torch.from_numpy(problem.k).to(dev)
    bs = [torch.from_numpy(problem.rhs(s)).to(dev) for s in range(nrhs)]
    log("shots: %s, %d right-hand sides, %s" % (problem.name, nrhs, args.shots_precision))
    prob = hm.create_problem(cfg, k)
    seq = [torch.empty_like(b) for b in bs]
    hm.fgmres_solve(prob, bs[0], out=seq[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq_infos = [hm.fgmres_solve(prob, b, out=u)[1] for b, u in zip(bs, seq)]
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    prob.close()
    log("sequential: %.3f s" % t_seq)
    bt = hm.create_batch(cfg, [k] * nrhs)
    outs = [torch.empty_like(b) for b in bs]
    hm.batch_solve(bt, bs, outs=outs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, bat_infos = hm.batch_solve(bt, bs, outs=outs)
    torch.cuda.synchronize()
    t_bat = time.perf_counter() - t0
    bt.close()
    log("lockstep batch: %.3f s" % t_bat)
    same = all(torch.equal(a, b) for a, b in zip(seq, outs))
    res = {"metric": "shots: solves/s, sequential solves vs one lockstep batch",
           "value": nrhs / t_bat, "unit": "solves/s", "n_gpus": 1, "higher_is_better": True,
           "dtype": "f32 precond / f64 outer" if prec == hm.HM_MIXED_FP32 else "f64",
           "data": "synthetic",
           "config": {"workload": problem.name, "nx": problem.nx, "ny": problem.ny,
                      "right_hand_sides": nrhs},
           "sequential": {"seconds": t_seq, "solves_per_s": nrhs / t_seq},
           "lockstep_batch": {"seconds": t_bat, "solves_per_s": nrhs / t_bat},
           "speedup": t_seq / t_bat,
           "bitwise_equal_to_sequential": same,
           "outer_iters": [i["outer_iters"] for i in bat_infos],
           "max_rel_res_true": max(i["rel_res_true"] for i in bat_infos),
           "sequential_outer_iters": [i["outer_iters"] for i in seq_infos]}
    print(json.dumps(res), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (independent "
              "solves shard across GPUs with no exchange)",
              file=sys.stderr)
        sys.exit(2)
    if args.trace_table:
        trace_table(args)
        return
    if args.counter_table:
        counter_table(args)
        return
    import numpy as np
    import torch

    import paper_2412_04980_amd as hm
    import workloads

    if args.serving:
        serving_bench(args)
        return
    if args.matvec:
        matvec_bench(args)
        return
    if args.complexity:
        complexity_bench(args)
        return
    if args.variants:
        variants_bench(args)
        return
    if args.shots:
        shots_bench(args)
        return
    if args.kernels:
        kernels_bench(args)
        return
    dev = torch.device("cuda:0")
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 16
        src = torch.ones(n, dtype=torch.complex128, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 3 x %d MiB device-to-device" % args.copy_calibration)
        del src, dst
    problem = workloads.config(args.config)
    k = torch.from_numpy(problem.k).to(dev)
    b = torch.from_numpy(problem.rhs(0)).to(dev)
    cfg = hm.default_config(problem.nx, problem.ny, problem.h)
    t0 = time.perf_counter()
    prob = hm.create_problem(cfg, k)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    log("fp64 problem set up in %.3f s" % setup_s)
    u64, total, lat, infos, kt = timed_solves(hm, torch, prob, b, args.steps, args.warmup,
                                              not args.no_timing)
    hm.reset_counts(prob)
    hm.fgmres_solve(prob, b, out=torch.empty_like(b))
    counts_l3 = hm.get_counts(prob, hm.KIND_CSLP)
    shape_l3 = hm.level_shape(prob, cfg.levels)
    prob.close()
    lat_ms = np.array(lat) * 1e3
    info = infos[-1]
    res = {
        "metric": "solves/s + p50/p99 latency, FP32-precond vs FP64, at rel. residual 1e-6",
        "value": args.steps / total,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": float(total / args.steps * 1e3),
        "p50_ms": float(np.percentile(lat_ms, 50)),
        "p99_ms": float(np.percentile(lat_ms, 99)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": problem.name, "nx": problem.nx, "ny": problem.ny,
                   "h": problem.h, "k": float(problem.k[0]) if args.config in (0, 1) else None,
                   "levels": cfg.levels, "precond": "MADP (tol L2 0.3, V-cycle L1-L2, "
                                                    "GMRES CSLP L3)"},
        "solve": {"outer_iters": info["outer_iters"],
                  "level2_iters_total": info["level2_iters_total"],
                  "cslp_iters_total": info["cslp_iters_total"],
                  "rel_res_true": info["rel_res_true"], "setup_s": setup_s},
    }
    if kt:
        classes = {name: {"ms": ms, "launches": n, "GBps": (by / (ms * 1e-3) / 1e9) if ms else 0.0,
                          "bytes": by}
                   for name, (ms, by, n) in kt.items()}
        dom = max(classes, key=lambda c: classes[c]["ms"])
        d = classes[dom]
        res["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": d["GBps"],
                           "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": d["GBps"] / HBM_PEAK_GBS, "traffic": measured_traffic(dom, problem.name),
                           "avg_launch_us": d["ms"] * 1e3 / max(d["launches"], 1),
                           "algorithmic_bytes_per_launch": d["bytes"] / max(d["launches"], 1)}
        res["roofline"]["bytes"] = ("algorithmic: every array read or written once, whether "
                                    "HBM or the 256 MB Infinity Cache serves it")
        if dom in ("cgs_dot", "cgs_update_norm"):
            share = gs_hbm_share(counts_l3, shape_l3[0] * shape_l3[1], 16, dom)
            if share is not None:
                res["roofline"]["hbm_only_estimate"] = {
                    "share_of_bytes": share, "achieved": d["GBps"] * share,
                    "frac": d["GBps"] * share / HBM_PEAK_GBS,
                    "model": "basis vectors older than the 200 MB recent window of bases above "
                             "256 MB, per pass of the recorded Krylov CSLP counts (three steps "
                             "per pair of passes)"}
        # measured ceilings of this GPU (a plain copy, a read-only stream), taken
        # after the timed region with the solver's memory released
        ceil = bandwidth_ceilings(torch)
        res["roofline"]["ceilings"] = ceil
        res["roofline"]["frac_of_read_ceiling"] = d["GBps"] / ceil["read_GBps"]
        res["roofline"]["frac_of_copy_ceiling"] = d["GBps"] / ceil["copy_GBps"]
        res["roofline"]["sampled_launches"] = d["launches"]
        res["roofline"]["sampling"] = "every %d-th launch of the class" % TIMING_EVERY
        res["kernel_classes"] = {c: {"est_ms_per_solve": v["ms"] * TIMING_EVERY / args.steps,
                                     "GBps": v["GBps"],
                                     "timed_launches": v["launches"]}
                                 for c, v in classes.items()}
        # algorithmic bytes of the timed classes (the Krylov passes, the stencils of
        # the Krylov loops and the MGS steps) per solve over the solve time
        est_bytes = sum(v["bytes"] for v in classes.values()) * TIMING_EVERY / args.steps
        res["timed_classes_effective_GBps"] = est_bytes / (total / args.steps) / 1e9
    if not args.no_mixed:
        cfgm = hm.default_config(problem.nx, problem.ny, problem.h, precision=hm.HM_MIXED_FP32)
        probm = hm.create_problem(cfgm, k)
        um, totm, latm, infm, _ = timed_solves(hm, torch, probm, b, args.steps, args.warmup, False)
        probm.close()
        err = float(torch.linalg.vector_norm(um - u64) / torch.linalg.vector_norm(u64))
        lm = np.array(latm) * 1e3
        res["mixed"] = {"value": args.steps / totm, "unit": "solves/s",
                        "p50_ms": float(np.percentile(lm, 50)),
                        "p99_ms": float(np.percentile(lm, 99)),
                        "outer_iters": infm[-1]["outer_iters"],
                        "rel_res_true": infm[-1]["rel_res_true"],
                        "rel_err_vs_fp64_solution": err, "dtype": "f32 precond / f64 outer"}
        # every preconditioner level in FP32, the coarsest problem included
        cfga = hm.default_config(problem.nx, problem.ny, problem.h,
                                 precision=hm.HM_MIXED_FP32_ALL)
        proba = hm.create_problem(cfga, k)
        ua, tota, lata, infa, _ = timed_solves(hm, torch, proba, b, args.steps, args.warmup, False)
        proba.close()
        erra = float(torch.linalg.vector_norm(ua - u64) / torch.linalg.vector_norm(u64))
        la = np.array(lata) * 1e3
        res["mixed_all_levels"] = {
            "value": args.steps / tota, "unit": "solves/s",
            "p50_ms": float(np.percentile(la, 50)), "p99_ms": float(np.percentile(la, 99)),
            "outer_iters": infa[-1]["outer_iters"], "rel_res_true": infa[-1]["rel_res_true"],
            "rel_err_vs_fp64_solution": erra,
            "dtype": "f32 preconditioner incl. coarsest problem / f64 outer"}
    if args.serving_leg > 0 and args.config == 1:
        # a bounded run of the request stream (the serving workload), so the line
        # also carries a serving measurement: requests over 257^2..2049^2 grids
        torch.cuda.empty_cache()
        srv = run_serving(args, args.serving_leg, args.rate)
        res["serving"] = {key: srv[key] for key in (
            "metric", "value", "unit", "offered_requests_per_s", "requests", "batching",
            "config") if key in srv}
        for key in ("p50_latency_ms", "p99_latency_ms", "mean_queue_wait_ms", "solves",
                    "wall_s", "requests_per_s", "max_rel_res", "by_grid", "level2_basis",
                    "level2_basis_regrows", "allocator_retries"):
            if key in srv:
                res["serving"][key] = srv[key]
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(problem, info, counts_l3)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
