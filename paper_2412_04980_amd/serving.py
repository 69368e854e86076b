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

With grouping on (`group_key`), a request admitted at the head of the queue
takes along the waiting requests of the same grid class (same key) that fit in
the member limit and the memory budget, and the group runs as one lockstep
batch of the library (hm_create_batch / hm_batch_solve): every right-hand side
of every request in the group is a batch member with its request's medium, and
each kernel launch sweeps the same level of all members still iterating.  Each
member's result is bitwise that of its solve alone.

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
    """Admits jobs FIFO under a slot limit and a memory budget; runs them concurrently.

    Without grouping, execute(job) and bytes_needed(job) take one job.  With
    group_key set, they take a list of jobs (a group of one key, at most
    max_members members counted by members(job)) and execute returns one
    (infos, solutions) pair per job of the group."""

    def __init__(self, execute, bytes_needed, budget_bytes, max_active=4, realtime=True,
                 group_key=None, max_members=1, members=None, progress=None):
        if max_active < 1:
            raise ValueError("max_active must be >= 1")
        self.execute = execute
        self.bytes_needed = bytes_needed
        self.budget = int(budget_bytes)
        self.max_active = max_active
        self.realtime = realtime
        self.group_key = group_key
        self.max_members = max(1, int(max_members))
        self.members = members or (lambda job: 1)
        self.progress = progress       # called as progress(done, total) after each group
        self.events = []               # (time, kind, rid, in_use_bytes, active)
        self.groups = []               # rids of each admitted group, in admission order

    def _need(self, group):
        return self.bytes_needed(group if self.group_key is not None else group[0])

    def _group(self, waiting, in_use):
        """The head job and, with grouping, the waiting jobs of its key that fit."""
        head = waiting[0]
        group = [head]
        if self.group_key is None:
            return group
        key = self.group_key(head)
        count = self.members(head)
        for job in list(waiting)[1:]:
            if self.group_key(job) != key or count + self.members(job) > self.max_members:
                continue
            if in_use + self._need(group + [job]) > self.budget:
                break
            group.append(job)
            count += self.members(job)
        return group

    def run(self, jobs):
        """Runs all jobs; returns their results in arrival order.  With
        realtime=False every job is available at time 0 (arrival times ignored)."""
        jobs = sorted(jobs, key=lambda j: (j.arrival, j.rid))
        for j in jobs:
            if self._need([j]) > self.budget:
                raise ValueError("request %d needs %d bytes, more than the whole budget %d"
                                 % (j.rid, self._need([j]), self.budget))
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

        def finished(group, admitted, need, fut):
            with cond:
                state["in_use"] -= need
                state["active"] -= 1
                try:
                    out = fut.result()
                    if self.group_key is None:
                        out = [out]
                    done = clock()
                    for job, (infos, sols) in zip(group, out):
                        results[job.rid] = JobResult(job.rid, arrival(job), admitted, done,
                                                     infos, sols)
                except BaseException as e:    # re-raised by run()
                    state["error"] = e
                self.events.append((clock(), "finish", group[0].rid, state["in_use"],
                                    state["active"]))
                if self.progress is not None:
                    self.progress(len(results), len(jobs))
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
                        group = self._group(waiting, state["in_use"])
                        need = self._need(group)
                        if state["in_use"] + need > self.budget:
                            break
                        for job in group:
                            waiting.remove(job)
                        state["in_use"] += need
                        state["active"] += 1
                        admitted = clock()
                        self.groups.append([job.rid for job in group])
                        self.events.append((admitted, "admit", group[0].rid, state["in_use"],
                                            state["active"]))
                        fut = pool.submit(self.execute,
                                          group if self.group_key is not None else group[0])
                        fut.add_done_callback(
                            lambda f, group=group, admitted=admitted, need=need:
                            finished(group, admitted, need, f))
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


def solve_with_regrow(run, basis, cap, exhausted):
    """Calls run(basis) until it does not raise `exhausted`, doubling the
    reserved level-2 basis each time (at most cap; 0 means cap already).
    Returns (result, basis used, number of regrows)."""
    grows = 0
    while True:
        try:
            return run(basis), basis, grows
        except exhausted:
            if basis == 0 or basis >= cap:
                raise
            basis = min(2 * basis, cap)
            grows += 1


class GpuExecutor:
    """Runs one request on the GPU: uploads its medium, builds its hierarchy in a
    fresh workspace, solves every right-hand side, frees everything.  Each worker
    thread owns one stream (default priority).  run_group / group_bytes /
    group_key / members are the grouped counterparts for a Scheduler with
    grouping: the right-hand sides of the group's requests become the members
    of lockstep batches of at most MAX_BATCH members.

    Each grid class reserves a level-2 basis of level2_basis vectors (initially
    `basis`, 0 = the full step cap) instead of the cap of 100: a solve that
    needs more raises BasisExhausted, and the request is re-run on a problem
    with twice the basis, which the class keeps from then on.  Results do not
    depend on the basis; admission counts the basis the class has when the
    group is admitted."""

    def __init__(self, precision=None, keep_solutions=False, device="cuda:0", overrides=None,
                 basis=16):
        import torch

        import paper_2412_04980_amd as hm
        self.torch = torch
        self.hm = hm
        self.precision = hm.HM_MIXED_FP32 if precision is None else precision
        self.keep = keep_solutions
        self.device = torch.device(device)
        self.overrides = dict(overrides or {})
        self._local = threading.local()
        self._lock = threading.Lock()
        self.basis0 = int(basis)
        self.basis = {}                # grid class -> reserved level-2 basis
        self.regrows = 0
        self.oom_retries = 0

    def _basis(self, key):
        with self._lock:
            return self.basis.get(key, self.basis0)

    def config(self, job, basis=None):
        if basis is None:
            basis = self._basis(self.group_key(job))
        cfg = self.hm.default_config(job.nx, job.ny, job.h, precision=self.precision,
                                     **self.overrides)
        cfg.level2_basis = min(basis, cfg.level2_maxit)
        return cfg

    def _regrowing(self, job, run):
        """run(cfg) with the class's basis, re-run with a larger one on
        BasisExhausted; the class keeps the largest basis it needed."""
        key = self.group_key(job)
        cap = self.config(job, 0).level2_maxit
        out, used, grows = solve_with_regrow(
            lambda basis: self._retry_oom(lambda: run(self.config(job, basis))),
            self._basis(key), cap, self.hm.BasisExhausted)
        with self._lock:
            self.regrows += grows
            if used == 0 or used > self.basis.get(key, self.basis0):
                self.basis[key] = used
        return out

    def bytes_needed(self, job):
        n = job.nx * job.ny
        return self.hm.workspace_bytes(self.config(job)) + 256 + 8 * n + 2 * 16 * n + (1 << 20)

    def group_key(self, job):
        return (job.nx, job.ny, job.h)

    def members(self, job):
        return len(job.rhs)

    def group_bytes(self, jobs):
        n = jobs[0].nx * jobs[0].ny
        nm = sum(len(j.rhs) for j in jobs)
        ws = self.hm.batch_workspace_bytes(self.config(jobs[0]), min(nm, self.hm.MAX_BATCH))
        return ws + 256 + 8 * n * len(jobs) + 2 * 16 * n * nm + (1 << 20)

    def run_group(self, jobs):
        """Solves every right-hand side of the jobs (one grid class) in lockstep
        batches; returns one (infos, solutions) pair per job."""
        torch, hm = self.torch, self.hm
        s = self._stream()
        members = [(q, r) for q, job in enumerate(jobs) for r in range(len(job.rhs))]
        infos = [[None] * len(job.rhs) for job in jobs]
        sols = [[None] * len(job.rhs) for job in jobs]
        with torch.cuda.stream(s):
            ks = [torch.from_numpy(job.k).to(self.device) for job in jobs]
            for c0 in range(0, len(members), hm.MAX_BATCH):
                chunk = members[c0:c0 + hm.MAX_BATCH]

                def run(cfg, chunk=chunk):
                    bt = hm.create_batch(cfg, [ks[q] for q, _ in chunk], stream=s)
                    try:
                        bs = [torch.from_numpy(jobs[q].rhs[r]).to(self.device) for q, r in chunk]
                        us, out = hm.batch_solve(bt, bs, stream=s)
                        return [(u.cpu().numpy() if self.keep else None, d)
                                for u, d in zip(us, out)]
                    finally:
                        s.synchronize()
                        bt.close()

                for (q, r), (u, d) in zip(chunk, self._regrowing(jobs[0], run)):
                    infos[q][r] = d
                    sols[q][r] = u
        return [(infos[q], sols[q] if self.keep else None) for q in range(len(jobs))]

    def _retry_oom(self, fn, attempts=600, pause=0.05):
        """fn(), retried while the device allocator reports out of memory: the
        admission budget counts workspace bytes, but the caching allocator can
        hold them in blocks of other sizes (workspaces of other classes and
        batch sizes), so a fresh workspace may not fit until cached blocks are
        released and other groups finish."""
        for i in range(attempts):
            try:
                return fn()
            except self.torch.OutOfMemoryError:
                if i + 1 == attempts:
                    raise
                with self._lock:
                    self.oom_retries += 1
                self.torch.cuda.empty_cache()
                time.sleep(pause)

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

            def run(cfg):
                infos, sols = [], []
                prob = hm.create_problem(cfg, k, stream=s)
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
                return infos, sols

            infos, sols = self._regrowing(job, run)
        return infos, (sols if self.keep else None)


def jobs_from_requests(requests):
    """Jobs from workloads.serving_stream() requests (one right-hand side per source)."""
    out = []
    for r in requests:
        p = r.problem
        out.append(Job(r.rid, r.arrival, p.nx, p.ny, p.h, p.k,
                       [p.rhs(s) for s in range(len(p.sources))], {"name": p.name}))
    return out
