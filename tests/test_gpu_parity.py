"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Component tests compare every building block element by element on seeded
random inputs (several tiles plus ragged edges: 33 x 41 nodes at level 1);
solver tests compare the preconditioner in fixed-count (replay) mode, where the
oracle's inner iteration counts make both sides the same map, and full solves
with the gates of the method: true relative residual <= 1e-6, solution error
<= 1e-5 against the oracle and outer iteration counts within +-1 (FP64).

Tolerances: FP64 building blocks 1e-13 (relative to the largest entry; the two
sides differ only in the order of the stencil sums); the preconditioner in
replay mode 1e-11 (it nests three Krylov solves; the coarsest CSLP GMRES uses
classical Gram-Schmidt on the GPU and modified Gram-Schmidt in the oracle);
FP32 building blocks 2e-6 (a few float roundings of O(1) values).
"""
import numpy as np
import pytest
import torch

import paper_2412_04980_amd as hm
import workloads
from oracle.krylov import CountLog
from oracle.madp import MADP

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def host(t):
    return t.cpu().numpy()


def relerr(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def rand_c(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def medium(nx, ny, kval, seed, spread=0.25):
    rng = np.random.default_rng(seed)
    return kval * rng.uniform(1 - spread, 1 + spread, nx * ny)


def make(nx, ny, h, k, **overrides):
    cfg = hm.default_config(nx, ny, h)
    for key, val in overrides.items():
        setattr(cfg, key, val)
    return hm.create_problem(cfg, gpu(k))


@pytest.fixture(scope="module")
def small():
    nx, ny, h = 33, 41, 1.0 / 32
    k = medium(nx, ny, 11.0, 1)
    o = MADP(nx, ny, h, k, levels=3)
    p64 = make(nx, ny, h, k)
    p32 = make(nx, ny, h, k, precision=hm.HM_MIXED_FP32)
    yield nx, ny, h, k, o, p64, p32
    p64.close()
    p32.close()


@pytest.mark.parametrize("level", [1, 2, 3])
@pytest.mark.parametrize("which", [hm.HM_OP_A, hm.HM_OP_M])
def test_level_operators(small, level, which):
    nx, ny, h, k, o, p64, p32 = small
    lev = o.levels[level]
    x = rand_c(lev.N, 10 + level)
    ref = (lev.A if which == hm.HM_OP_A else lev.M) @ x
    got = host(hm.apply_operator(p64, level, which, gpu(x)))
    assert relerr(got, ref) <= 1e-13
    got32 = host(hm.apply_operator(p32, level, which, gpu(x)))
    tol = 2e-6 if level <= 2 else 1e-13          # level 3 stays FP64 in mixed mode
    assert relerr(got32, ref) <= tol


@pytest.mark.parametrize("level", [1, 2])
def test_deflation_transfers(small, level):
    nx, ny, h, k, o, p64, p32 = small
    Z = o.levels[level].Z
    xf = rand_c(Z.shape[0], 20 + level)
    xc = rand_c(Z.shape[1], 30 + level)
    assert relerr(host(hm.apply_operator(p64, level, hm.HM_OP_ZT, gpu(xf))), Z.T @ xf) <= 1e-14
    assert relerr(host(hm.apply_operator(p64, level, hm.HM_OP_Z, gpu(xc))), Z @ xc) <= 1e-14
    assert relerr(host(hm.apply_operator(p32, level, hm.HM_OP_ZT, gpu(xf))), Z.T @ xf) <= 2e-6
    assert relerr(host(hm.apply_operator(p32, level, hm.HM_OP_Z, gpu(xc))), Z @ xc) <= 2e-6


@pytest.mark.parametrize("level", [1, 2])
def test_multigrid_components(small, level):
    nx, ny, h, k, o, p64, p32 = small
    V = o.mg[level]
    assert hm.level_shape(p64, level, len(V.levels) - 1) == (V.levels[-1].nx, V.levels[-1].ny)
    for q, lv in enumerate(V.levels):
        x = rand_c(lv.nx * lv.ny, 40 + q)
        assert relerr(host(hm.apply_operator(p64, level, hm.HM_OP_MG_M, gpu(x), sub=q)),
                      lv.M @ x) <= 1e-13
        assert relerr(host(hm.apply_operator(p64, level, hm.HM_OP_MG_JACOBI, gpu(x), sub=q)),
                      lv.omega * x / lv.diag) <= 1e-13
        if q + 1 < len(V.levels):
            assert relerr(host(hm.apply_operator(p64, level, hm.HM_OP_MG_RESTRICT, gpu(x), sub=q)),
                          V.R[q] @ x) <= 1e-14
            c = rand_c(V.levels[q + 1].nx * V.levels[q + 1].ny, 50 + q)
            assert relerr(host(hm.apply_operator(p64, level, hm.HM_OP_MG_PROLONG, gpu(c), sub=q)),
                          V.P[q] @ c) <= 1e-14


@pytest.mark.parametrize("level", [1, 2])
def test_vcycle(small, level):
    """The V-cycle runs as a captured HIP graph after its first use: replay it
    several times on different inputs, with unrelated eager work and
    synchronisations in between, and check every replay against the oracle."""
    nx, ny, h, k, o, p64, p32 = small
    for rep in range(4):
        x = rand_c(o.levels[level].N, 60 + 10 * rep + level)
        ref = o.mg[level](x)
        assert relerr(host(hm.apply_operator(p64, level, hm.HM_OP_VCYCLE, gpu(x))), ref) <= 1e-12
        assert relerr(host(hm.apply_operator(p32, level, hm.HM_OP_VCYCLE, gpu(x))), ref) <= 1e-5
        hm.apply_operator(p64, level, hm.HM_OP_A, gpu(x))          # eager work between replays
        torch.cuda.synchronize()


def test_coarsest_cslp_gmres(small):
    nx, ny, h, k, o, p64, p32 = small
    lev = o.levels[3]
    x = rand_c(lev.N, 70)
    o.log = CountLog("record")
    ref = o.cslp(3, x)
    counts = o.log.data["cslp_l3"]
    hm.reset_counts(p64)
    got = host(hm.apply_operator(p64, 3, hm.HM_OP_CSLP, gpu(x)))
    assert hm.get_counts(p64, hm.KIND_CSLP) == counts
    assert relerr(got, ref) <= 1e-11


def test_modified_gram_schmidt_option(small):
    """HM_ORTH_MODIFIED runs the Krylov CSLP with the oracle's modified
    Gram-Schmidt: the same counts and 1e-12 on the coarsest solve, replayed
    preconditioner applications at 1e-11, and a solve that meets the gates."""
    nx, ny, h, k, o, p64, p32 = small
    pm = make(nx, ny, h, k, cslp_orth=hm.HM_ORTH_MODIFIED)
    try:
        lev = o.levels[3]
        x = rand_c(lev.N, 71)
        o.log = CountLog("record")
        ref = o.cslp(3, x)
        hm.reset_counts(pm)
        got = host(hm.apply_operator(pm, 3, hm.HM_OP_CSLP, gpu(x)))
        assert hm.get_counts(pm, hm.KIND_CSLP) == o.log.data["cslp_l3"]
        assert relerr(got, ref) <= 1e-12
        v = rand_c(nx * ny, 83)
        o.log = CountLog("record")
        ref = o.apply(v)
        _replay_all(pm, o.log)
        try:
            got = host(hm.precond_apply(pm, gpu(v)))
        finally:
            _replay_off(pm)
        assert relerr(got, ref) <= 1e-11
        b = workloads.point_source(nx, ny, h, 16, 20)
        u_ref, info_ref = o.solve(b)
        u, info = hm.fgmres_solve(pm, gpu(b))
        u = host(u)
        assert info["rel_res_true"] <= 1e-6
        assert abs(info["outer_iters"] - info_ref["outer_iters"]) <= 1
        assert np.linalg.norm(u - u_ref) <= 1e-5 * np.linalg.norm(u_ref)
    finally:
        pm.close()


def _replay_all(prob, log):
    for kind, key in ((hm.KIND_LEVEL2, "level2"), (hm.KIND_CSLP, "cslp_l3"),
                      (hm.KIND_MG_COARSE, "mg_coarse"), (hm.KIND_OUTER, "outer")):
        hm.set_replay(prob, kind, log.data.get(key, []))


def _replay_off(prob):
    for kind in range(4):
        hm.set_replay(prob, kind, [])


def test_precond_apply_replay(small):
    nx, ny, h, k, o, p64, p32 = small
    v = rand_c(nx * ny, 80)
    o.log = CountLog("record")
    ref = o.apply(v)
    _replay_all(p64, o.log)
    try:
        got = host(hm.precond_apply(p64, gpu(v)))
    finally:
        _replay_off(p64)
    assert relerr(got, ref) <= 1e-11


def test_precond_apply_free_counts_match(small):
    nx, ny, h, k, o, p64, p32 = small
    v = rand_c(nx * ny, 81)
    o.log = CountLog("record")
    ref = o.apply(v)
    hm.reset_counts(p64)
    got = host(hm.precond_apply(p64, gpu(v)))
    assert hm.get_counts(p64, hm.KIND_LEVEL2) == o.log.data["level2"]
    assert relerr(got, ref) <= 1e-10


def test_precond_mixed_close_to_fp64(small):
    nx, ny, h, k, o, p64, p32 = small
    v = rand_c(nx * ny, 82)
    o.log = CountLog("record")
    ref = o.apply(v)
    _replay_all(p32, o.log)
    try:
        got = host(hm.precond_apply(p32, gpu(v)))
    finally:
        _replay_off(p32)
    assert relerr(got, ref) <= 1e-4


def test_two_level_precond_apply():
    """Two levels: level 2 is the coarsest, its coarse problem takes one FGMRES
    step and its CSLP is a V-cycle, so no inner solve stops on a tolerance and
    one application is a fixed map on both sides.  Three applications in a row
    (the coarsest FGMRES and the V-cycle reuse their buffers) each match the
    oracle: 1e-11 in FP64 as the replayed three-level preconditioner, 1e-4 in
    the mixed modes (with two levels both run every level in FP32)."""
    nx, ny, h = 33, 41, 1.0 / 32
    k = medium(nx, ny, 11.0, 4)
    o = MADP(nx, ny, h, k, levels=2)
    precs = (hm.HM_FP64, hm.HM_MIXED_FP32, hm.HM_MIXED_FP32_ALL)
    probs = [make(nx, ny, h, k, levels=2, precision=prec) for prec in precs]
    try:
        for rep in range(3):
            v = rand_c(nx * ny, 90 + rep)
            ref = o.apply(v)
            for prec, p in zip(precs, probs):
                got = host(hm.precond_apply(p, gpu(v)))
                assert relerr(got, ref) <= (1e-11 if prec == hm.HM_FP64 else 1e-4), (rep, prec)
    finally:
        for p in probs:
            p.close()


def _solve_pair(prob_name, nx, ny, h, k, src, precision=hm.HM_FP64):
    o = MADP(nx, ny, h, k, levels=3)
    b = workloads.point_source(nx, ny, h, *src)
    u_ref, info_ref = o.solve(b)
    p = make(nx, ny, h, k, precision=precision)
    try:
        u, info = hm.fgmres_solve(p, gpu(b))
    finally:
        p.close()
    u = host(u)
    err = np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref)
    print("%s prec=%d outer gpu=%d oracle=%d rel_res=%.3e err=%.3e" % (
        prob_name, precision, info["outer_iters"], info_ref["outer_iters"],
        info["rel_res_true"], err))
    return o, u, info, u_ref, info_ref, err


def test_solve_fp64_config0():
    p = workloads.config(0)
    o, u, info, u_ref, info_ref, err = _solve_pair("config0", p.nx, p.ny, p.h, p.k, p.sources[0])
    assert info["status"] == hm.HM_OK
    assert info["rel_res_true"] <= 1e-6
    b = p.rhs()
    A = o.levels[1].A
    assert np.linalg.norm(b - A @ u) <= 1e-6 * np.linalg.norm(b)
    assert abs(info["outer_iters"] - info_ref["outer_iters"]) <= 1
    assert err <= 1e-5


def test_solve_mixed_config0():
    p = workloads.config(0)
    o, u, info, u_ref, info_ref, err = _solve_pair("config0", p.nx, p.ny, p.h, p.k, p.sources[0],
                                                   hm.HM_MIXED_FP32)
    b = p.rhs()
    A = o.levels[1].A
    assert info["status"] == hm.HM_OK
    assert np.linalg.norm(b - A @ u) <= 1e-6 * np.linalg.norm(b)
    assert err <= 1e-5


def test_solve_all_fp32_levels_config0_and_wedge():
    """Every preconditioner level in FP32 (the coarsest problem included): the FP64
    outer FGMRES still meets 1e-6 against the oracle's matrix, the solution is
    within 1e-5 of the oracle's, and the outer count stays within one step."""
    p = workloads.config(0)
    o, u, info, u_ref, info_ref, err = _solve_pair("config0", p.nx, p.ny, p.h, p.k, p.sources[0],
                                                   hm.HM_MIXED_FP32_ALL)
    b = p.rhs()
    assert info["status"] == hm.HM_OK
    assert np.linalg.norm(b - o.levels[1].A @ u) <= 1e-6 * np.linalg.norm(b)
    assert abs(info["outer_iters"] - info_ref["outer_iters"]) <= 1
    assert err <= 1e-5
    nx, ny, h = 121, 201, 5.0                   # wedge medium at a fifth of the resolution
    k = 2 * np.pi * 8.0 / workloads.wedge_velocity(nx, ny, h)
    o, u, info, u_ref, info_ref, err = _solve_pair("wedge", nx, ny, h, k, (60, 1),
                                                   hm.HM_MIXED_FP32_ALL)
    b = workloads.point_source(nx, ny, h, 60, 1)
    assert np.linalg.norm(b - o.levels[1].A @ u) <= 1e-6 * np.linalg.norm(b)
    assert abs(info["outer_iters"] - info_ref["outer_iters"]) <= 1
    assert err <= 1e-5


def test_solve_heterogeneous_gmres_coarsest_multigrid():
    # 93 x 93: the multigrid hierarchies end on 24 x 24 = 576 > 512 nodes, so the
    # coarsest multigrid solve is GMRES (nonlinear) on both sides
    nx = ny = 93
    h = 1.0 / 92
    k = medium(nx, ny, 16.0, 5)
    o, u, info, u_ref, info_ref, err = _solve_pair("gmres-coarse", nx, ny, h, k, (40, 50))
    assert info["rel_res_true"] <= 1e-6
    assert abs(info["outer_iters"] - info_ref["outer_iters"]) <= 1
    assert err <= 1e-5
    assert info["mg_coarse_iters_total"] > 0


def test_replayed_solve_matches_oracle_closely():
    nx = ny = 65
    h = 1.0 / 64
    k = medium(nx, ny, 14.0, 6)
    o = MADP(nx, ny, h, k, levels=3)
    b = workloads.point_source(nx, ny, h, 20, 33)
    u_ref, info_ref = o.solve(b)
    p = make(nx, ny, h, k)
    try:
        _replay_all(p, o.log)
        u, info = hm.fgmres_solve(p, gpu(b))
    finally:
        p.close()
    assert info["outer_iters"] == info_ref["outer_iters"]
    assert relerr(host(u), u_ref) <= 1e-9


def test_zero_rhs_gives_zero():
    nx = ny = 17
    p = make(nx, ny, 1 / 16, np.full(nx * ny, 3.0))
    try:
        u, info = hm.fgmres_solve(p, torch.zeros(nx * ny, dtype=torch.complex128, device=DEV))
    finally:
        p.close()
    assert info["outer_iters"] == 0 and info["status"] == hm.HM_OK
    assert not host(u).any()


def test_rejects_bad_wavenumber():
    nx = ny = 17
    k = np.full(nx * ny, 3.0)
    k[100] = np.nan
    with pytest.raises(hm.HelmDeflError) as e:
        make(nx, ny, 1 / 16, k)
    assert e.value.status == hm.HM_ERR_ARG
    k[100] = -1.0
    with pytest.raises(hm.HelmDeflError):
        make(nx, ny, 1 / 16, k)


@pytest.mark.parametrize("restart,maxit", [(3, 300), (30, 3), (4, 6)])
def test_restarts_and_step_cap_match_the_oracle(restart, maxit):
    """Outer restarts and the outer step cap: restart 3 converges through
    several restart cycles; a cap of 3 (or 6 steps in restarts of 4) stops
    short of the tolerance with HM_NOT_CONVERGED and the solution written.  The
    solution agrees with the oracle's run of the same settings (1e-5); a capped
    run takes exactly the oracle's steps and ends at its residual, a converged
    one within one outer step of it.  The reported true residual is that of
    the returned solution."""
    p = workloads.config(0)
    b = p.rhs()
    o = MADP(p.nx, p.ny, p.h, p.k, levels=3)
    u_ref, info_ref = o.solve(b, restart=restart, maxit=maxit)
    prob = make(p.nx, p.ny, p.h, p.k, outer_restart=restart, outer_maxit=maxit)
    try:
        u, info = hm.fgmres_solve(prob, gpu(b))
    finally:
        prob.close()
    u = host(u)
    A = o.levels[1].A
    rel = np.linalg.norm(b - A @ u) / np.linalg.norm(b)
    rel_ref = np.linalg.norm(b - A @ u_ref) / np.linalg.norm(b)
    converged = rel_ref <= 1e-6
    assert info["status"] == (hm.HM_OK if converged else hm.HM_NOT_CONVERGED)
    assert abs(info["rel_res_true"] - rel) <= 1e-9 * max(rel, 1e-12)
    assert np.linalg.norm(u - u_ref) <= 1e-5 * np.linalg.norm(u_ref)
    if converged:
        assert abs(info["outer_iters"] - info_ref["outer_iters"]) <= 1
        assert rel <= 1e-6
    else:
        # the same iterate after the same number of steps
        assert info["outer_iters"] == info_ref["outer_iters"] == maxit
        assert abs(rel - rel_ref) <= 1e-6 * rel_ref and rel > 1e-6


def test_rejects_zero_wavenumber_with_sommerfeld():
    """k = 0 everywhere with Sommerfeld ghosts is the Neumann Laplacian, whose
    constants span its null space: creation fails with an argument error (with
    Dirichlet boundaries the same field is the Poisson problem and is solved,
    see the Dirichlet tests)."""
    nx = ny = 17
    with pytest.raises(hm.HelmDeflError) as e:
        make(nx, ny, 1 / 16, np.zeros(nx * ny))
    assert e.value.status == hm.HM_ERR_ARG and "singular" in str(e.value)
    k = np.zeros(nx * ny)
    k[40] = 1e-3                      # one nonzero node is enough
    make(nx, ny, 1 / 16, k).close()


def test_rejects_short_workspace():
    nx = ny = 17
    cfg = hm.default_config(nx, ny, 1 / 16)
    ws = torch.empty(1024, dtype=torch.uint8, device=DEV)
    with pytest.raises(hm.HelmDeflError) as e:
        hm.create_problem(cfg, gpu(np.full(nx * ny, 3.0)), workspace=ws)
    assert e.value.status == hm.HM_ERR_NOMEM


def test_two_problems_are_independent():
    nx = ny = 33
    h = 1 / 32
    k1, k2 = medium(nx, ny, 9.0, 7), medium(nx, ny, 12.0, 8)
    b = workloads.point_source(nx, ny, h, 16, 16)
    pa = make(nx, ny, h, k1)
    pb = make(nx, ny, h, k2)
    try:
        ua, _ = hm.fgmres_solve(pa, gpu(b))
        ub, _ = hm.fgmres_solve(pb, gpu(b))
        ua2, _ = hm.fgmres_solve(pa, gpu(b))
    finally:
        pa.close()
        pb.close()
    assert torch.equal(ua, ua2)
    assert not torch.equal(ua, ub)


@pytest.mark.parametrize("levels", [4, 5, 6])
def test_deeper_hierarchies(levels):
    """4- to 6-level MADP (the fourth- to sixth-level stencils of Appendix A;
    six levels end on 5 x 5 nodes): one FGMRES step on every level below 2,
    Krylov CSLP on levels >= 3."""
    nx = ny = 129
    h = 1.0 / 128
    k = medium(nx, ny, 20.0, 3, spread=0.2)
    o = MADP(nx, ny, h, k, levels=levels)
    b = workloads.point_source(nx, ny, h, 60, 70)
    u_ref, info_ref = o.solve(b)
    p = make(nx, ny, h, k, levels=levels)
    try:
        hm.reset_counts(p)
        u, info = hm.fgmres_solve(p, gpu(b))
        got = hm.get_counts(p, hm.KIND_CSLP)
    finally:
        p.close()
    # per level-3..(L-1) preconditioner call the coarser solves run first; the
    # GPU records all Krylov CSLP solves in call order
    order = []
    seqs = {l: list(o.log.data["cslp_l%d" % l]) for l in range(3, levels + 1)}

    def expand(l):                      # the CSLP calls made by one Prec_l, l >= 3
        if l + 1 == levels:
            order.append(seqs[levels].pop(0))
        else:
            expand(l + 1)
        order.append(seqs[l].pop(0))
    while seqs[levels]:
        if levels == 3:
            order.append(seqs[3].pop(0))
        else:
            expand(3)
    assert got == order
    assert abs(info["outer_iters"] - info_ref["outer_iters"]) <= 1
    assert np.linalg.norm(host(u) - u_ref) / np.linalg.norm(u_ref) <= 1e-5
    assert info["rel_res_true"] <= 1e-6


@pytest.mark.parametrize("precision", [hm.HM_FP64, hm.HM_MIXED_FP32, hm.HM_MIXED_FP32_ALL])
def test_small_krylov_matches_host_driven(precision):
    """The one-workgroup GMRES of small coarse levels (hm_set_small_krylov)
    against the host-driven path on the 129^2, k = 20 workload, whose coarsest
    level (33^2) takes it: the same step counts, the Krylov CSLP and replayed
    preconditioner applications to rounding, and the same solve."""
    nx = ny = 129
    h = 1.0 / 128
    k = np.full(nx * ny, 20.0)
    tol = 1e-11 if precision != hm.HM_MIXED_FP32_ALL else 1e-5
    a = make(nx, ny, h, k, precision=precision)
    bh = make(nx, ny, h, k, precision=precision)
    hm.set_small_krylov(bh, False)
    try:
        for seed in (90, 91):
            x = workloads.smooth_field(33, 33, seed, sigma=1.5)
            hm.reset_counts(a)
            hm.reset_counts(bh)
            ra = host(hm.apply_operator(a, 3, hm.HM_OP_CSLP, gpu(x)))
            rb = host(hm.apply_operator(bh, 3, hm.HM_OP_CSLP, gpu(x)))
            assert hm.get_counts(a, hm.KIND_CSLP) == hm.get_counts(bh, hm.KIND_CSLP)
            assert relerr(ra, rb) <= tol
        b = workloads.point_source(nx, ny, h, 64, 64)
        hm.reset_counts(a)
        hm.reset_counts(bh)
        ua, ia = hm.fgmres_solve(a, gpu(b))
        ub, ib = hm.fgmres_solve(bh, gpu(b))
        assert ia["outer_iters"] == ib["outer_iters"]
        assert hm.get_counts(a, hm.KIND_LEVEL2) == hm.get_counts(bh, hm.KIND_LEVEL2)
        assert ia["rel_res_true"] <= 1e-6 and ib["rel_res_true"] <= 1e-6
        assert relerr(host(ua), host(ub)) <= (1e-9 if precision == hm.HM_FP64 else 1e-5)
    finally:
        a.close()
        bh.close()
