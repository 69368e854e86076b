"""Continuous-batching request loop for MADP-FGMRES solves on one GPU.

Requests (a grid, a wavenumber field and 1..n right-hand sides) arrive over
time.  The scheduler admits them in arrival order whenever a worker slot is
free and the device memory the request needs (its solver workspace plus its
vectors, `bytes_needed`) fits in the budget that running requests leave.  Each
admitted request runs on its own worker thread with its own HIP stream: its
level hierarchy and Krylov bases stay resident for all of its right-hand sides,
and its kernels overlap on the device with those of the other running requests.
When a request finishes, its memory returns to the budget and the next waiting
request is admitted, without waiting for the others (no batch barrier).

The scheduler is independent of the GPU: `Scheduler` takes an `execute(job)`
callable and a `bytes_needed(job)` estimate, so the admission logic runs with a
simulated executor on the CPU as well.  `GpuExecutor` is the MI355X executor that
calls the library's C ABI through the binding; every solver step runs in the
library's kernels.
"""
import collections
import threading
import time
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field


@dataclass
class Job:
    rid: int
    arrival: float                 # seconds after the start of the run
    nx: int
    ny: int
    h: float
    k: object                      # float64 nodal wavenumber (numpy, nx*ny)
    rhs: list                      # complex128 right-hand sides (numpy, nx*ny each)
    meta: dict = field(default_factory=dict)


@dataclass
class JobResult:
    rid: int
    arrival: float
    admitted: float
    finished: float
    infos: list
    solutions: list = None

    @property
    def latency(self):
        return self.finished - self.arrival

    @property
    def wait(self):
        return self.admitted - self.arrival


class Scheduler:
    """Admits jobs FIFO under a slot limit and a memory budget; runs them concurrently."""

    def __init__(self, execute, bytes_needed, budget_bytes, max_active=4, realtime=True):
        if max_active < 1:
            raise ValueError("max_active must be >= 1")
        self.execute = execute
        self.bytes_needed = bytes_needed
        self.budget = int(budget_bytes)
        self.max_active = max_active
        self.realtime = realtime
        self.events = []               # (time, kind, rid, in_use_bytes, active)

    def run(self, jobs):
        """Runs all jobs; returns their results in arrival order.  With
        realtime=False every job is available at time 0 (arrival times ignored)."""
        jobs = sorted(jobs, key=lambda j: (j.arrival, j.rid))
        for j in jobs:
            if self.bytes_needed(j) > self.budget:
                raise ValueError("request %d needs %d bytes, more than the whole budget %d"
                                 % (j.rid, self.bytes_needed(j), self.budget))
        cond = threading.Condition()          # re-entrant lock inside
        pending = collections.deque(jobs)     # not yet arrived
        waiting = collections.deque()         # arrived, not admitted (FIFO)
        results = {}
        state = {"in_use": 0, "active": 0, "error": None}
        t0 = time.perf_counter()

        def clock():
            return time.perf_counter() - t0

        def arrival(job):
            return job.arrival if self.realtime else 0.0

        def finished(job, admitted, need, fut):
            with cond:
                state["in_use"] -= need
                state["active"] -= 1
                try:
                    infos, sols = fut.result()
                    results[job.rid] = JobResult(job.rid, arrival(job), admitted, clock(), infos,
                                                 sols)
                except BaseException as e:    # re-raised by run()
                    state["error"] = e
                self.events.append((clock(), "finish", job.rid, state["in_use"], state["active"]))
                cond.notify_all()

        pool = ThreadPoolExecutor(max_workers=self.max_active)
        try:
            with cond:
                while True:
                    if state["error"] is not None:
                        raise state["error"]
                    t = clock()
                    while pending and arrival(pending[0]) <= t:
                        waiting.append(pending.popleft())
                    # admit in arrival order while a slot and the memory are free
                    while waiting and state["active"] < self.max_active:
                        job = waiting[0]
                        need = self.bytes_needed(job)
                        if state["in_use"] + need > self.budget:
                            break
                        waiting.popleft()
                        state["in_use"] += need
                        state["active"] += 1
                        admitted = clock()
                        self.events.append((admitted, "admit", job.rid, state["in_use"],
                                            state["active"]))
                        fut = pool.submit(self.execute, job)
                        fut.add_done_callback(
                            lambda f, job=job, admitted=admitted, need=need:
                            finished(job, admitted, need, f))
                    if not (pending or waiting or state["active"]):
                        break
                    timeout = 0.5
                    if pending:
                        timeout = min(timeout, max(0.0, arrival(pending[0]) - clock()))
                    cond.wait(timeout=timeout)
        finally:
            pool.shutdown(wait=True)
        if state["error"] is not None:
            raise state["error"]
        return [results[j.rid] for j in jobs]


def summarize(results, wall_seconds):
    import numpy as np
    lat = np.array([r.latency for r in results]) * 1e3
    wait = np.array([r.wait for r in results]) * 1e3
    n_solves = sum(len(r.infos) for r in results)
    return {
        "requests": len(results),
        "solves": n_solves,
        "wall_s": wall_seconds,
        "requests_per_s": len(results) / wall_seconds,
        "solves_per_s": n_solves / wall_seconds,
        "p50_latency_ms": float(np.percentile(lat, 50)),
        "p99_latency_ms": float(np.percentile(lat, 99)),
        "mean_queue_wait_ms": float(wait.mean()),
        "max_rel_res": max(i["rel_res_true"] for r in results for i in r.infos),
    }


class GpuExecutor:
    """Runs one request on the GPU: uploads its medium, builds its hierarchy in a
    fresh workspace, solves every right-hand side, frees everything.  Each worker
    thread owns one stream (default priority)."""

    def __init__(self, precision=None, keep_solutions=False, device="cuda:0", overrides=None):
        import torch

        import paper_2412_04980_amd as hm
        self.torch = torch
        self.hm = hm
        self.precision = hm.HM_MIXED_FP32 if precision is None else precision
        self.keep = keep_solutions
        self.device = torch.device(device)
        self.overrides = dict(overrides or {})
        self._local = threading.local()

    def config(self, job):
        return self.hm.default_config(job.nx, job.ny, job.h, precision=self.precision,
                                      **self.overrides)

    def bytes_needed(self, job):
        n = job.nx * job.ny
        return self.hm.workspace_bytes(self.config(job)) + 256 + 8 * n + 2 * 16 * n + (1 << 20)

    def _stream(self):
        s = getattr(self._local, "stream", None)
        if s is None:
            s = self.torch.cuda.Stream(device=self.device)
            self._local.stream = s
        return s

    def __call__(self, job):
        torch, hm = self.torch, self.hm
        s = self._stream()
        infos, sols = [], []
        with torch.cuda.stream(s):
            k = torch.from_numpy(job.k).to(self.device)
            prob = hm.create_problem(self.config(job), k, stream=s)
            try:
                u = torch.empty(job.nx * job.ny, dtype=torch.complex128, device=self.device)
                for rhs in job.rhs:
                    b = torch.from_numpy(rhs).to(self.device)
                    _, info = hm.fgmres_solve(prob, b, out=u, stream=s)
                    infos.append(info)
                    if self.keep:
                        sols.append(u.cpu().numpy())
            finally:
                s.synchronize()
                prob.close()
        return infos, (sols if self.keep else None)


def jobs_from_requests(requests):
    """Jobs from workloads.serving_stream() requests (one right-hand side per source)."""
    out = []
    for r in requests:
        p = r.problem
        out.append(Job(r.rid, r.arrival, p.nx, p.ny, p.h, p.k,
                       [p.rhs(s) for s in range(len(p.sources))], {"name": p.name}))
    return out
