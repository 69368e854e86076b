"""Several Arnoldi steps per two passes over the basis (hm_set_krylov_steps; three
steps are the default on FP64 levels solved host-driven) against the oracle and
against one step per two passes.

A block of steps forms its Hessenberg columns by classical Gram-Schmidt in the
coordinates of [V_0..V_j, M v_j, M^2 v_j, ...] from one pass of inner products,
so it agrees with one-step classical Gram-Schmidt to rounding: the same counts,
the Krylov CSLP within 1e-12, the replayed preconditioner within 1e-11 of the
oracle.  The small one-workgroup path is switched off here so that the blocks
run on the small grids."""
import numpy as np
import pytest
import torch

import paper_2412_04980_amd as hm
import workloads
from oracle.krylov import CountLog
from oracle.madp import MADP

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
BLOCKS = (2, hm.KRYLOV_STEPS_MAX)


def gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def host(t):
    return t.cpu().numpy()


def relerr(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def medium(nx, ny, kval, seed, spread=0.25):
    rng = np.random.default_rng(seed)
    return kval * rng.uniform(1 - spread, 1 + spread, nx * ny)


def make(nx, ny, h, k, steps=hm.KRYLOV_STEPS_MAX, small=False, **overrides):
    cfg = hm.default_config(nx, ny, h)
    for key, val in overrides.items():
        setattr(cfg, key, val)
    p = hm.create_problem(cfg, gpu(k))
    hm.set_small_krylov(p, small)
    hm.set_krylov_steps(p, steps)
    return p


def replay_all(prob, log):
    for kind, key in ((hm.KIND_LEVEL2, "level2"), (hm.KIND_CSLP, "cslp_l3"),
                      (hm.KIND_MG_COARSE, "mg_coarse"), (hm.KIND_OUTER, "outer")):
        hm.set_replay(prob, kind, [int(c) for c in log.data.get(key, [])])


def replay_off(prob):
    for kind in range(4):
        hm.set_replay(prob, kind, [])


@pytest.fixture(scope="module")
def grid():
    nx, ny, h = 65, 81, 1.0 / 64
    k = medium(nx, ny, 16.0, 3)
    return nx, ny, h, k, MADP(nx, ny, h, k, levels=3)


@pytest.mark.parametrize("steps", BLOCKS)
@pytest.mark.parametrize("seed", [5, 6, 7])
def test_krylov_cslp_blocks_match_oracle(grid, seed, steps):
    nx, ny, h, k, o = grid
    lev = o.levels[3]
    x = workloads.smooth_field(lev.nx, lev.ny, seed, sigma=1.0)
    o.log = CountLog("record")
    ref = o.cslp(3, x)
    counts = o.log.data["cslp_l3"]
    p = make(nx, ny, h, k, steps)
    q = make(nx, ny, h, k, 1)
    try:
        got = host(hm.apply_operator(p, 3, hm.HM_OP_CSLP, gpu(x)))
        one = host(hm.apply_operator(q, 3, hm.HM_OP_CSLP, gpu(x)))
        print("steps", counts, "blocks of %d vs oracle %.2e, vs one step %.2e"
              % (steps, relerr(got, ref), relerr(got, one)))
        assert hm.get_counts(p, hm.KIND_CSLP) == counts == hm.get_counts(q, hm.KIND_CSLP)
        assert relerr(got, ref) <= 1e-11
        assert relerr(got, one) <= 1e-12
        # every fixed step count, whole blocks and a shorter last block
        for fixed in (1, 2, 3, 4, 5, 7, 8, 11):
            o.log = CountLog("replay", {"cslp_l3": [fixed]})
            ref = o.cslp(3, x)
            hm.set_replay(p, hm.KIND_CSLP, [fixed])
            try:
                got = host(hm.apply_operator(p, 3, hm.HM_OP_CSLP, gpu(x)))
            finally:
                hm.set_replay(p, hm.KIND_CSLP, [])
            assert relerr(got, ref) <= 1e-11, fixed
    finally:
        p.close()
        q.close()


def test_replayed_preconditioner_and_solve_with_blocks(grid):
    nx, ny, h, k, o = grid
    p = make(nx, ny, h, k)
    try:
        v = np.random.default_rng(12).standard_normal(nx * ny) + 0j
        o.log = CountLog("record")
        ref = o.apply(v)
        replay_all(p, o.log)
        try:
            got = host(hm.precond_apply(p, gpu(v)))
        finally:
            replay_off(p)
        assert relerr(got, ref) <= 1e-11
        b = workloads.point_source(nx, ny, h, 30, 40)
        u_ref, info_ref = o.solve(b)
        u, info = hm.fgmres_solve(p, gpu(b))
        u = host(u)
        assert info["rel_res_true"] <= 1e-6
        assert abs(info["outer_iters"] - info_ref["outer_iters"]) <= 1
        assert np.linalg.norm(u - u_ref) <= 1e-5 * np.linalg.norm(u_ref)
    finally:
        p.close()


@pytest.mark.parametrize("precision", [hm.HM_FP64, hm.HM_MIXED_FP32, hm.HM_MIXED_FP32_ALL])
def test_blocks_match_one_step_in_every_precision(precision):
    """A 257^2 random medium (65^2 coarsest level): when that level is FP64
    (HM_FP64, HM_MIXED_FP32) the solve equals the one-step solve to rounding;
    with every level in FP32 both run one step per two passes, and the results
    are identical."""
    n = 257
    h = 1.0 / (n - 1)
    rng = np.random.default_rng(21)
    k0 = (0.5 / h**2) ** (1.0 / 3.0)
    k = k0 * 2500.0 / workloads.gaussian_random_velocity(n, rng)
    b = workloads.point_source(n, n, h, 100, 140)
    p = make(n, n, h, k, small=True, precision=precision)
    q = make(n, n, h, k, 1, small=True, precision=precision)
    try:
        up, ip = hm.fgmres_solve(p, gpu(b))
        uq, iq = hm.fgmres_solve(q, gpu(b))
        cp, cq = hm.get_counts(p, hm.KIND_CSLP), hm.get_counts(q, hm.KIND_CSLP)
        diff = relerr(host(up), host(uq))
        print("precision %d: outer %d / %d, cslp %d / %d, solution rel. diff %.2e"
              % (precision, ip["outer_iters"], iq["outer_iters"], sum(cp), sum(cq), diff))
        assert ip["rel_res_true"] <= 1e-6 and iq["rel_res_true"] <= 1e-6
        if precision == hm.HM_MIXED_FP32_ALL:
            assert np.array_equal(host(up), host(uq)) and cp == cq
        else:
            assert ip["outer_iters"] == iq["outer_iters"] and cp == cq
            assert diff <= 1e-9
    finally:
        p.close()
        q.close()


@pytest.mark.parametrize("steps", BLOCKS)
def test_blocks_in_a_batch_equal_alone(steps):
    """Bitwise: a member's blocks in a lockstep batch run the same kernels on the
    same data as alone (the coefficient kernel's sums do not depend on timing)."""
    nx, ny, h = 65, 81, 1.0 / 64
    ks = [medium(nx, ny, 16.0, s) for s in (3, 4)]
    bs = [workloads.point_source(nx, ny, h, 30, 40), workloads.point_source(nx, ny, h, 20, 60)]
    cfg = hm.default_config(nx, ny, h)
    bt = hm.create_batch(cfg, [gpu(k) for k in ks])
    try:
        for m in bt.members:
            hm.set_small_krylov(m, False)
            hm.set_krylov_steps(m, steps)
        us, _ = hm.batch_solve(bt, [gpu(b) for b in bs])
        us = [host(u) for u in us]
    finally:
        bt.close()
    for k, b, ub in zip(ks, bs, us):
        p = make(nx, ny, h, k, steps)
        try:
            u, _ = hm.fgmres_solve(p, gpu(b))
            assert np.array_equal(host(u), ub)
        finally:
            p.close()
