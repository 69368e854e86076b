"""Serving on the GPU: requests of different grid sizes and media, run
concurrently by the continuous-batching scheduler (several in flight, each on
its own stream), give exactly the results of the same requests solved alone,
and every result meets the outer tolerance against the oracle's matrix."""
import numpy as np
import pytest

import paper_2412_04980_amd as hm
import workloads
from oracle import operators as op
from paper_2412_04980_amd.serving import GpuExecutor, Job, Scheduler

pytestmark = pytest.mark.gpu


def small_jobs(seed=11, n_jobs=6):
    rng = np.random.default_rng(seed)
    jobs = []
    for rid in range(n_jobs):
        n = int(rng.choice([65, 129]))
        h = 1.0 / (n - 1)
        k0 = (0.5 / h**2) ** (1.0 / 3.0)
        c = workloads.gaussian_random_velocity(n, rng)
        k = k0 * 2500.0 / c
        ns = int(rng.integers(1, 4))
        rhs = [workloads.point_source(n, n, h, int(rng.integers(8, n - 8)), int(rng.integers(8, n - 8)))
               for _ in range(ns)]
        jobs.append(Job(rid, 0.0, n, n, h, k, rhs))
    return jobs


@pytest.mark.parametrize("precision", [hm.HM_FP64, hm.HM_MIXED_FP32])
def test_results_identical_alone_and_in_the_mix(precision):
    jobs = small_jobs()
    ex = GpuExecutor(precision=precision, keep_solutions=True)
    budget = 4 * max(ex.bytes_needed(j) for j in jobs)
    sched = Scheduler(ex, ex.bytes_needed, budget, max_active=3, realtime=False)
    mixed = sched.run(jobs)
    assert max(e[4] for e in sched.events) >= 2           # really concurrent
    for j, r in zip(jobs, mixed):
        alone_infos, alone = ex(j)
        assert len(alone) == len(r.solutions) == len(j.rhs)
        for s, (ua, um) in enumerate(zip(alone, r.solutions)):
            assert np.array_equal(ua, um), (j.rid, s)
        A = op.five_point(j.nx, j.ny, j.h, j.k, 1.0)
        for s, rhs in enumerate(j.rhs):
            assert np.linalg.norm(rhs - A @ r.solutions[s]) <= 1e-6 * np.linalg.norm(rhs)
            assert r.infos[s]["outer_iters"] == alone_infos[s]["outer_iters"]


@pytest.mark.parametrize("precision", [hm.HM_FP64, hm.HM_MIXED_FP32])
def test_grouped_requests_run_as_lockstep_batches(precision):
    """With grouping, same-size requests waiting together run as one lockstep
    batch (every right-hand side a member); each result is bitwise the result
    of the request solved alone."""
    jobs = small_jobs(seed=12, n_jobs=8)
    ex = GpuExecutor(precision=precision, keep_solutions=True)
    budget = 4 * max(ex.group_bytes([j]) for j in jobs) + sum(ex.group_bytes([j]) for j in jobs)
    sched = Scheduler(ex.run_group, ex.group_bytes, budget, max_active=2, realtime=False,
                      group_key=ex.group_key, max_members=hm.MAX_BATCH, members=ex.members)
    grouped = sched.run(jobs)
    assert any(len(g) > 1 for g in sched.groups)           # batches of several requests
    by_rid = {j.rid: j for j in jobs}
    for g in sched.groups:
        assert len({(by_rid[r].nx, by_rid[r].ny) for r in g}) == 1
    for j, r in zip(jobs, grouped):
        alone_infos, alone = ex(j)
        for s, (ua, um) in enumerate(zip(alone, r.solutions)):
            assert np.array_equal(ua, um), (j.rid, s)
            assert r.infos[s]["outer_iters"] == alone_infos[s]["outer_iters"]
