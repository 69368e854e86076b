"""GPU tests of lockstep batches (hm_create_batch / hm_batch_solve): several
problems of one configuration solved with one launch per sweep of a level.

Each member's solution, solve record and inner step counts must equal, bit
for bit, those of the same problem solved on its own with hm_fgmres_solve
(which the parity tests pin to the oracle), for
  * FP64 and the mixed build, three and four levels;
  * Dirichlet boundaries with the W-cycle, and the tolerance on three levels;
  * a grid whose multigrid coarsest level is too large for the dense solve
    (GMRES inside the V-cycle, eager instead of a captured graph);
  * two levels, where the coarsest level's CSLP is a V-cycle;
  * every preconditioner level in FP32 with the modified Gram-Schmidt Krylov
    CSLP;
  * members that stop after different numbers of outer steps, a zero
    right-hand side, the largest batch (16 members) and a batch of one;
  * a second solve on the same batch (graphs reused per member set);
  * per-member replayed step counts and kernel timing inside a batch.
"""
import numpy as np
import pytest
import torch

import paper_2412_04980_amd as hm
import workloads

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
INFO_KEYS = ("outer_iters", "level2_iters_total", "cslp_iters_total", "mg_coarse_iters_total",
             "rel_res_estimate", "rel_res_true")


def gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def media(n, scales, seed):
    """Random media with k0^3 h^2 = 0.5 scaled per member (larger k, more steps)."""
    h = 1.0 / (n - 1)
    k0 = (0.5 / h**2) ** (1.0 / 3.0)
    rng = np.random.default_rng(seed)
    return h, [s * k0 * 2500.0 / workloads.gaussian_random_velocity(n, rng) for s in scales]


def sources(n, h, nb, seed):
    rng = np.random.default_rng(seed)
    return [workloads.point_source(n, n, h, int(rng.integers(4, n - 4)), int(rng.integers(4, n - 4)))
            for _ in range(nb)]


def solve_alone(cfg, k, b):
    prob = hm.create_problem(cfg, gpu(k))
    try:
        u, info = hm.fgmres_solve(prob, gpu(b))
        counts = [hm.get_counts(prob, kind) for kind in range(4)]
        return u.cpu(), info, counts
    finally:
        prob.close()


def batch_vs_alone(cfg, ks, bss):
    """Solves the batch once per list of right-hand sides in bss and compares
    every member with its solve alone; returns the batch records."""
    bt = hm.create_batch(cfg, [gpu(k) for k in ks])
    records = []
    try:
        for bs in bss:
            for m in bt.members:
                hm.reset_counts(m)
            us, infos = hm.batch_solve(bt, [gpu(b) for b in bs])
            counts = [[hm.get_counts(m, kind) for kind in range(4)] for m in bt.members]
            for i, (k, b) in enumerate(zip(ks, bs)):
                ua, ia, ca = solve_alone(cfg, k, b)
                assert torch.equal(us[i].cpu(), ua), "member %d solution differs" % i
                for key in INFO_KEYS:
                    assert infos[i][key] == ia[key], (i, key, infos[i][key], ia[key])
                assert counts[i] == ca, "member %d inner counts differ" % i
            records.append(infos)
    finally:
        bt.close()
    return records


CASES = {
    "fp64_l3": (129, (1.0, 1.3, 1.6), dict(levels=3)),
    "mixed_l4": (257, (1.0, 1.4, 1.2), dict(levels=4, precision=hm.HM_MIXED_FP32)),
    "dirichlet_w": (129, (1.0, 1.5), dict(levels=3, bc=hm.HM_BC_DIRICHLET, coarse_steps=2)),
    "tol3_l4": (129, (1.2, 1.0), dict(levels=4, tol_levels=3)),
    "krylov_mg_coarsest": (149, (1.0, 1.3), dict(levels=3)),
    "two_levels": (65, (1.0, 1.3, 1.1), dict(levels=2)),
    "all_fp32_mgs": (129, (1.0, 1.4), dict(levels=3, precision=hm.HM_MIXED_FP32_ALL,
                                            cslp_orth=hm.HM_ORTH_MODIFIED)),
}


@pytest.mark.parametrize("name", list(CASES))
def test_batch_members_equal_their_solves_alone(name):
    n, scales, kw = CASES[name]
    print("batch case", name, flush=True)
    h, ks = media(n, scales, seed=len(name))
    cfg = hm.default_config(n, n, h, **kw)
    (infos,) = batch_vs_alone(cfg, ks, [sources(n, h, len(ks), seed=7)])
    assert all(i["rel_res_true"] <= 1e-6 for i in infos)
    if name == "fp64_l3":
        # the members stop after different numbers of outer steps, so later
        # sweeps run on a subset of the batch
        assert len({i["outer_iters"] for i in infos}) > 1


def test_zero_rhs_member_and_second_solve():
    n = 129
    h, ks = media(n, (1.0, 1.2, 1.4), seed=5)
    cfg = hm.default_config(n, n, h)
    first = sources(n, h, 3, seed=1)
    first[1] = np.zeros_like(first[1])
    second = sources(n, h, 3, seed=2)
    rec = batch_vs_alone(cfg, ks, [first, second])
    assert rec[0][1]["outer_iters"] == 0 and rec[0][1]["rel_res_true"] == 0.0


def test_largest_batch_and_batch_of_one():
    n = 33
    h, ks = media(n, [1.0 + 0.05 * i for i in range(hm.MAX_BATCH)], seed=9)
    cfg = hm.default_config(n, n, h)
    batch_vs_alone(cfg, ks, [sources(n, h, len(ks), seed=3)])
    batch_vs_alone(cfg, ks[:1], [sources(n, h, 1, seed=4)])


def test_batch_argument_errors():
    n = 33
    h, ks = media(n, (1.0, 1.1), seed=2)
    cfg = hm.default_config(n, n, h)
    bt = hm.create_batch(cfg, [gpu(k) for k in ks])
    try:
        b = gpu(sources(n, h, 1, seed=1)[0])
        with pytest.raises(ValueError):
            hm.batch_solve(bt, [b])
        with pytest.raises(hm.HelmDeflError):
            hm.batch_solve(bt, [b, b], outs=[b, torch.empty_like(b)])
    finally:
        bt.close()
    bad = gpu(np.full(n * n, -1.0))
    with pytest.raises(hm.HelmDeflError):
        hm.create_batch(cfg, [gpu(ks[0]), bad])


def test_batch_with_replayed_counts_and_timing():
    """Per-member replayed step counts (a member's fixed-count parity mode) and
    kernel timing on member 0 work inside a batch: every member equals its
    replayed solve alone bit for bit, and the timed classes record launches
    whose bytes count every member of the launch.  The coarsest level is
    host-driven here (hm_set_small_krylov off): the one-workgroup solve of small
    levels has no per-step launches to time."""
    n = 65
    h, ks = media(n, (1.0, 1.3), seed=13)
    cfg = hm.default_config(n, n, h)
    bs = sources(n, h, 2, seed=14)
    # record each member's counts alone, then replay them in the batch
    recorded = []
    for k, b in zip(ks, bs):
        p = hm.create_problem(cfg, gpu(k))
        hm.set_small_krylov(p, False)
        try:
            hm.fgmres_solve(p, gpu(b))
            recorded.append([hm.get_counts(p, kind) for kind in range(4)])
        finally:
            p.close()
    bt = hm.create_batch(cfg, [gpu(k) for k in ks])
    try:
        for m, counts in zip(bt.members, recorded):
            hm.set_small_krylov(m, False)
            for kind in range(4):
                hm.set_replay(m, kind, counts[kind])
        hm.set_timing(bt.members[0], (1 << 5) - 1, 1)
        us, infos = hm.batch_solve(bt, [gpu(b) for b in bs])
        timing = hm.get_timing(bt.members[0])
    finally:
        bt.close()
    for i, (k, b) in enumerate(zip(ks, bs)):
        p = hm.create_problem(cfg, gpu(k))
        hm.set_small_krylov(p, False)
        try:
            for kind in range(4):
                hm.set_replay(p, kind, recorded[i][kind])
            u, info = hm.fgmres_solve(p, gpu(b))
        finally:
            p.close()
        assert torch.equal(us[i], u)
        assert infos[i]["outer_iters"] == info["outer_iters"]
    ms, by, launches = timing["cgs_dot"]
    assert launches > 0 and ms > 0 and by > 0
    assert sum(t[2] for t in timing.values()) > launches
