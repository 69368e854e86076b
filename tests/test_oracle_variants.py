"""Pins of the oracle's method variants (oracle.madp: coarse_steps, tol_levels,
tol_level2).

  * cycle type (Sec. 3.2): with m FGMRES steps on a coarse system of n unknowns
    and m >= n, and a linear preconditioner, the Krylov space is the whole space,
    so the coarse solve is exact and the preconditioner equals the A-DEF1 closed
    form M^-1 (v - A Z E^-1 Z^T v) + Z E^-1 Z^T v built from dense solves;
    the coarse residual does not grow with m (FGMRES minimises it over nested
    spaces that share their first direction);
  * per-level tolerance (Sec. 4.5): with the tolerance extended to level 3 and
    set to 1e-13, the level-2 preconditioner equals its closed form with the
    exact E_3^-1; with the MADP setting (one step on level 3) it does not;
  * MADP-v3 (Sec. 4.4, tolerance 0.1 on level 2): every level-2 solve ends with
    a true relative residual <= 0.1; tol_levels = 1 makes level 2 take exactly
    coarse_steps steps.
"""
import numpy as np
import scipy.sparse.linalg as spla

from oracle.madp import MADP


def _medium(n, kval, seed):
    rng = np.random.default_rng(seed)
    return kval * rng.uniform(0.8, 1.2, n * n)


def _rand(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def _exact(M):
    lu = spla.splu(M.tocsc())
    return lu.solve


def _closed_form(lev, lev_c, v):
    """A-DEF1 with exact E^-1 and exact M^-1 from dense / sparse direct solves."""
    E = lev_c.A.toarray()
    Z = lev.Z
    t = Z @ np.linalg.solve(E, Z.T @ v)
    return spla.spsolve(lev.M.tocsc(), v - lev.A @ t) + t


def _relerr(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_enough_coarse_steps_make_the_coarse_solve_exact():
    n, h = 9, 1.0 / 8
    k = _medium(n, 4.0, 1)
    m = MADP(n, n, h, k, levels=2, coarse_steps=25)
    m.cslp_override = {1: _exact(m.levels[1].M)}
    v = _rand(n * n, 2)
    assert m.levels[2].N == 25
    assert _relerr(m.apply(v), _closed_form(m.levels[1], m.levels[2], v)) <= 1e-9
    m.coarse_steps = 1                             # the V-cycle setting differs
    assert _relerr(m.apply(v), _closed_form(m.levels[1], m.levels[2], v)) > 1e-3


def test_coarse_residual_does_not_grow_with_steps():
    n, h = 33, 1.0 / 32
    k = _medium(n, 10.0, 3)
    m = MADP(n, n, h, k, levels=3)
    v_hat = m.levels[1].Z.T @ _rand(n * n, 4)
    E2 = m.levels[2].A
    m.tol_levels = 1                               # level 2 takes coarse_steps steps
    res = []
    for steps in (1, 2, 3, 4):
        m.coarse_steps = steps
        res.append(np.linalg.norm(v_hat - E2 @ m.coarse(1, v_hat)))
    assert all(res[i + 1] <= res[i] * (1 + 1e-12) for i in range(3))
    assert res[-1] < res[0]


def test_tolerance_on_level3_reaches_the_exact_level3_solve():
    n, h = 17, 1.0 / 16
    k = _medium(n, 3.0, 5)
    m = MADP(n, n, h, k, levels=4, tol_levels=3, tol_level2=1e-13, level2_maxit=200)
    for l in (2, 3, 4):
        m.cslp_override[l] = _exact(m.levels[l].M)
    assert [m.levels[l].N for l in (2, 3, 4)] == [81, 25, 9]
    v = _rand(m.levels[2].N, 6)
    ref = _closed_form(m.levels[2], m.levels[3], v)
    assert _relerr(m.precond(2, v), ref) <= 1e-9
    m.tol_levels = 2                               # MADP: one step on level 3
    assert _relerr(m.precond(2, v), ref) > 1e-3


def test_madp_v3_level2_residuals_within_tolerance():
    n, h = 33, 1.0 / 32
    k = _medium(n, 10.0, 7)
    m = MADP(n, n, h, k, levels=3, tol_level2=0.1)
    E2 = m.levels[2].A
    for seed in (8, 9, 10):
        v_hat = m.levels[1].Z.T @ _rand(n * n, seed)
        x = m.coarse(1, v_hat)
        assert np.linalg.norm(v_hat - E2 @ x) <= 0.1 * np.linalg.norm(v_hat) * (1 + 1e-10)


def test_tol_levels_one_fixes_the_level2_step_count():
    n, h = 33, 1.0 / 32
    k = _medium(n, 10.0, 11)
    for steps in (1, 2):
        m = MADP(n, n, h, k, levels=3, tol_levels=1, coarse_steps=steps)
        m.apply(_rand(n * n, 12))
        assert m.log.data["level2"] == [steps]
