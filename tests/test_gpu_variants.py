"""GPU parity of the method variants against the oracle (same variants, same
inputs):

  * MADP-v3 (level-2 tolerance 0.1, Sec. 4.4);
  * W-cycle (two FGMRES steps on the coarse levels without a tolerance,
    Sec. 3.2), on three and four levels;
  * fixed steps on every coarse level (tol_levels = 1);
  * the tolerance extended to the third level (tol_levels = 3, Sec. 4.5).

Preconditioner applications are compared in replay mode where every inner
count is replayable (1e-11) and free-running otherwise (1e-10, equal counts);
full solves by the gates of the method (outer steps +-1, solution error <= 1e-5,
true relative residual <= 1e-6).
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


def medium(n, kval, seed, spread=0.2):
    rng = np.random.default_rng(seed)
    return kval * rng.uniform(1 - spread, 1 + spread, n * n)


def rand_c(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def make(n, h, k, **kw):
    return hm.create_problem(hm.default_config(n, n, h, **kw), gpu(k))


VARIANTS = {
    "v3": dict(levels=3, tol_level2=0.1),
    "w3": dict(levels=3, coarse_steps=2),
    "w4": dict(levels=4, coarse_steps=2),
    "fixed1": dict(levels=3, tol_levels=1),
    "tol3": dict(levels=4, tol_levels=3),
}


def oracle_kw(kw):
    return {key: kw[key] for key in ("levels", "tol_level2", "coarse_steps", "tol_levels")
            if key in kw}


@pytest.mark.parametrize("name", ["v3", "w3", "fixed1"])
def test_precond_replay(name):
    kw = VARIANTS[name]
    n, h = 65, 1.0 / 64
    k = medium(n, 14.0, 21)
    o = MADP(n, n, h, k, **oracle_kw(kw))
    v = rand_c(n * n, 22)
    o.log = CountLog("record")
    ref = o.apply(v)
    p = make(n, h, k, **kw)
    try:
        for kind, key in ((hm.KIND_LEVEL2, "level2"), (hm.KIND_CSLP, "cslp_l3"),
                          (hm.KIND_MG_COARSE, "mg_coarse")):
            hm.set_replay(p, kind, o.log.data.get(key, []))
        got = host(hm.precond_apply(p, gpu(v)))
    finally:
        p.close()
    assert relerr(got, ref) <= 1e-11


@pytest.mark.parametrize("name", ["w4", "tol3"])
def test_precond_free_running(name):
    kw = VARIANTS[name]
    n, h = 65, 1.0 / 64
    k = medium(n, 12.0, 23)
    o = MADP(n, n, h, k, **oracle_kw(kw))
    v = rand_c(n * n, 24)
    o.log = CountLog("record")
    ref = o.apply(v)
    p = make(n, h, k, **kw)
    try:
        hm.reset_counts(p)
        got = host(hm.precond_apply(p, gpu(v)))
        assert hm.get_counts(p, hm.KIND_LEVEL2) == o.log.data["level2"]
    finally:
        p.close()
    assert relerr(got, ref) <= 1e-10


@pytest.mark.parametrize("name", sorted(VARIANTS))
def test_variant_solves_match_oracle(name):
    kw = VARIANTS[name]
    n, h = 129, 1.0 / 128
    k = medium(n, 40.0, 25)
    o = MADP(n, n, h, k, **oracle_kw(kw))
    b = workloads.point_source(n, n, h, 50, 70)
    u_ref, info_ref = o.solve(b)
    p = make(n, h, k, **kw)
    try:
        u, info = hm.fgmres_solve(p, gpu(b))
    finally:
        p.close()
    err = np.linalg.norm(host(u) - u_ref) / np.linalg.norm(u_ref)
    print("%s outer gpu=%d oracle=%d level2 gpu=%d oracle=%d err=%.2e" % (
        name, info["outer_iters"], info_ref["outer_iters"], info["level2_iters_total"],
        info_ref["level2_iters_total"], err))
    assert info["status"] == hm.HM_OK
    assert info["rel_res_true"] <= 1e-6
    assert abs(info["outer_iters"] - info_ref["outer_iters"]) <= 1
    assert err <= 1e-5
