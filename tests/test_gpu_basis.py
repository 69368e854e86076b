"""A level-2 basis smaller than the step cap (config level2_basis): a solve whose
level-2 solves fit in it gives bitwise the result of the default (full) basis;
one that needs more stops with BasisExhausted instead of returning a different
result; the serving executor then re-creates the problem with a larger basis
and returns the default result."""
import numpy as np
import pytest
import torch

import paper_2412_04980_amd as hm
import workloads
from paper_2412_04980_amd.serving import GpuExecutor, Job

pytestmark = pytest.mark.gpu


def solve(p, rhs, **kw):
    cfg = hm.default_config(p.nx, p.ny, p.h, **kw)
    prob = hm.create_problem(cfg, torch.from_numpy(p.k).cuda())
    try:
        u, info = hm.fgmres_solve(prob, torch.from_numpy(rhs).cuda())
        return u.cpu().numpy(), info, hm.get_counts(prob, hm.KIND_LEVEL2)
    finally:
        prob.close()


def batch(p, rhss, **kw):
    cfg = hm.default_config(p.nx, p.ny, p.h, **kw)
    k = torch.from_numpy(p.k).cuda()
    bt = hm.create_batch(cfg, [k] * len(rhss))
    try:
        us, _ = hm.batch_solve(bt, [torch.from_numpy(b).cuda() for b in rhss])
        return [u.cpu().numpy() for u in us]
    finally:
        bt.close()


@pytest.mark.parametrize("precision", [hm.HM_FP64, hm.HM_MIXED_FP32])
def test_small_level2_basis_gives_the_default_result_or_stops(precision):
    p = workloads.config(0)
    b = p.rhs()
    u0, info0, counts = solve(p, b, precision=precision)
    m = max(counts)
    print("level-2 steps per call", counts)
    assert m >= 2
    u1, info1, counts1 = solve(p, b, precision=precision, level2_basis=m)
    assert counts1 == counts and info1["outer_iters"] == info0["outer_iters"]
    assert np.array_equal(u0, u1)
    with pytest.raises(hm.BasisExhausted):
        solve(p, b, precision=precision, level2_basis=m - 1)
    # the same in a lockstep batch (two sources in one medium)
    b2 = workloads.point_source(p.nx, p.ny, p.h, 40, 90)
    m2 = max(m, max(solve(p, b2, precision=precision)[2]))
    ref = batch(p, [b, b2], precision=precision)
    got = batch(p, [b, b2], precision=precision, level2_basis=m2)
    assert all(np.array_equal(x, y) for x, y in zip(ref, got))
    with pytest.raises(hm.BasisExhausted):
        batch(p, [b, b2], precision=precision, level2_basis=m - 1)


def test_serving_executor_regrows_the_basis():
    p = workloads.config(0)
    job = Job(0, 0.0, p.nx, p.ny, p.h, p.k, [p.rhs()])
    ref = GpuExecutor(precision=hm.HM_FP64, keep_solutions=True, basis=0)
    ex = GpuExecutor(precision=hm.HM_FP64, keep_solutions=True, basis=1)
    _, s0 = ref(job)
    infos, s1 = ex(job)
    assert ex.regrows >= 1 and ex.basis[ex.group_key(job)] >= 2
    assert np.array_equal(s0[0], s1[0]) and infos[0]["status"] == hm.HM_OK
    # the grouped path starts from the class's grown basis: no further regrow
    grown = ex.regrows
    [(_, s2)] = ex.run_group([job])
    assert ex.regrows == grown and np.array_equal(s0[0], s2[0])
