"""CPU tests of the serving scheduler with a simulated executor: FIFO admission,
the slot limit, the memory budget, continuous (non-batch) admission and error
propagation."""
import threading
import time

import pytest

from paper_2412_04980_amd.serving import Job, Scheduler, summarize


def job(rid, arrival, size, work=0.02):
    return Job(rid, arrival, 3, 3, 1.0, None, [None], {"size": size, "work": work})


class FakeExecutor:
    def __init__(self):
        self.lock = threading.Lock()
        self.active = 0
        self.max_seen = 0
        self.order = []

    def __call__(self, j):
        with self.lock:
            self.active += 1
            self.max_seen = max(self.max_seen, self.active)
            self.order.append(j.rid)
        time.sleep(j.meta["work"])
        with self.lock:
            self.active -= 1
        return [{"rel_res_true": 1e-7, "rid": j.rid}], None


def test_fifo_and_slot_limit():
    ex = FakeExecutor()
    s = Scheduler(ex, lambda j: j.meta["size"], budget_bytes=100, max_active=2, realtime=False)
    res = s.run([job(i, 0.0, 10) for i in range(6)])
    assert [r.rid for r in res] == list(range(6))
    assert ex.order == list(range(6))
    assert ex.max_seen == 2


def test_memory_budget_limits_concurrency():
    ex = FakeExecutor()
    s = Scheduler(ex, lambda j: j.meta["size"], budget_bytes=100, max_active=8, realtime=False)
    s.run([job(i, 0.0, 60) for i in range(4)])
    assert ex.max_seen == 1                      # 60 + 60 > 100
    assert all(e[3] <= 100 for e in s.events)


def test_continuous_admission_no_batch_barrier():
    # a long job must not hold back short ones behind it once slots free up
    ex = FakeExecutor()
    s = Scheduler(ex, lambda j: j.meta["size"], budget_bytes=100, max_active=2, realtime=False)
    jobs = [job(0, 0.0, 10, work=0.3)] + [job(i, 0.0, 10, work=0.01) for i in range(1, 6)]
    t0 = time.perf_counter()
    res = s.run(jobs)
    assert time.perf_counter() - t0 < 0.6
    finish = {r.rid: r.finished for r in res}
    assert all(finish[i] < finish[0] for i in range(1, 6))


def test_realtime_arrivals_respected():
    ex = FakeExecutor()
    s = Scheduler(ex, lambda j: j.meta["size"], budget_bytes=100, max_active=4, realtime=True)
    res = s.run([job(0, 0.0, 10, 0.01), job(1, 0.15, 10, 0.01)])
    assert res[1].admitted >= 0.15
    assert res[1].latency < 0.15
    summ = summarize(res, 0.2)
    assert summ["requests"] == 2 and summ["solves"] == 2


def test_oversized_request_rejected():
    s = Scheduler(FakeExecutor(), lambda j: j.meta["size"], budget_bytes=50, max_active=2)
    with pytest.raises(ValueError):
        s.run([job(0, 0.0, 60)])


def test_executor_error_propagates():
    def bad(j):
        raise RuntimeError("boom")
    s = Scheduler(bad, lambda j: 1, budget_bytes=10, max_active=2, realtime=False)
    with pytest.raises(RuntimeError):
        s.run([job(0, 0.0, 1), job(1, 0.0, 1)])


class FakeGroupExecutor:
    def __init__(self):
        self.groups = []

    def __call__(self, group):
        self.groups.append([j.rid for j in group])
        time.sleep(0.01)
        return [([{"rel_res_true": 1e-7}] * len(j.rhs), None) for j in group]


def gjob(rid, key, nrhs=1, size=10):
    return Job(rid, 0.0, key, key, 1.0, None, [None] * nrhs, {"size": size})


def test_grouping_takes_same_key_jobs_within_member_and_memory_limits():
    ex = FakeGroupExecutor()
    jobs = [gjob(0, 65, 2), gjob(1, 129), gjob(2, 65, 3), gjob(3, 65, 2), gjob(4, 129, 1),
            gjob(5, 65, 1)]
    s = Scheduler(ex, lambda g: sum(j.meta["size"] for j in g), budget_bytes=1000, max_active=1,
                  realtime=False, group_key=lambda j: j.nx, max_members=6,
                  members=lambda j: len(j.rhs))
    res = s.run(jobs)
    assert [r.rid for r in res] == list(range(6))
    # head 0 (2) takes 2 (3) and 5 (1): 6 members, 3 (2) does not fit; then the
    # 129 class, then the rest
    assert s.groups == [[0, 2, 5], [1, 4], [3]]
    assert ex.groups == s.groups
    assert all(len(r.infos) == len(j.rhs) for r, j in zip(res, jobs))
    # the memory budget also bounds a group
    s2 = Scheduler(FakeGroupExecutor(), lambda g: sum(j.meta["size"] for j in g), budget_bytes=25,
                   max_active=1, realtime=False, group_key=lambda j: j.nx, max_members=16,
                   members=lambda j: len(j.rhs))
    s2.run([gjob(i, 65) for i in range(5)])
    assert s2.groups == [[0, 1], [2, 3], [4]]


def test_progress_callback_counts_every_request():
    seen = []
    ex = FakeExecutor()
    s = Scheduler(ex, lambda j: j.meta["size"], budget_bytes=100, max_active=3, realtime=False,
                  progress=lambda done, total: seen.append((done, total)))
    s.run([job(i, 0.0, 10, work=0.005) for i in range(7)])
    assert len(seen) == 7                        # one call per finished group (one job each)
    assert [d for d, _ in seen] == sorted(d for d, _ in seen)
    assert seen[-1] == (7, 7) and all(t == 7 for _, t in seen)
