"""Pins of the oracle's (F)GMRES (oracle.krylov) against dense linear algebra."""
import numpy as np
import pytest

from oracle.krylov import CountLog, fgmres, fgmres_restarted, givens


def _system(n=40, seed=0):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) + 4 * np.eye(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return A, b


def test_givens_zeroes_second_component():
    for a, b in [(1 + 2j, 3.0), (0j, 2.0), (-1j, 0.5), (2.0, 0.0)]:
        c, s = givens(a, b)
        assert abs(c * c + abs(s) ** 2 - 1) < 1e-15
        assert abs(-np.conj(s) * a + c * b) < 1e-15


def test_gmres_matches_dense_solve():
    A, b = _system()
    x, steps, est = fgmres(lambda v: A @ v, b, None, tol=1e-12, maxit=60)
    xd = np.linalg.solve(A, b)
    assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)
    assert est <= 1e-12


def test_gmres_terminates_in_n_steps():
    A, b = _system(n=12, seed=3)
    x, steps, est = fgmres(lambda v: A @ v, b, None, tol=None, maxit=12)
    assert np.linalg.norm(A @ x - b) <= 1e-10 * np.linalg.norm(b)


@pytest.mark.parametrize("m", [1, 3, 7, 15])
def test_estimate_equals_true_residual(m):
    A, b = _system(seed=5)
    x, steps, est = fgmres(lambda v: A @ v, b, None, tol=None, maxit=m)
    assert steps == m
    assert abs(est - np.linalg.norm(b - A @ x) / np.linalg.norm(b)) <= 1e-10


def test_fgmres_exact_preconditioner_one_step():
    A, b = _system(seed=7)
    Ainv = np.linalg.inv(A)
    x, steps, est = fgmres(lambda v: A @ v, b, lambda v: Ainv @ v, tol=1e-10, maxit=5)
    assert steps == 1
    assert np.linalg.norm(A @ x - b) <= 1e-10 * np.linalg.norm(b)


def test_fgmres_variable_preconditioner_reaches_tolerance():
    A, b = _system(seed=9)
    D = np.diag(A)
    calls = []

    def prec(v):                       # changes every call: truly flexible
        calls.append(1)
        return v / D * (1.0 + 0.1 * len(calls) % 3)
    x, steps, est = fgmres(lambda v: A @ v, b, prec, tol=1e-8, maxit=40)
    assert np.linalg.norm(A @ x - b) <= 1.01e-8 * np.linalg.norm(b)


def test_restarted_reaches_tolerance():
    A, b = _system(n=60, seed=11)
    A = A + 10 * np.eye(60)
    u, its, rel = fgmres_restarted(lambda v: A @ v, b, None, tol=1e-9, restart=5, maxit=400)
    assert its > 5                      # really restarted
    assert rel <= 1e-9
    assert np.linalg.norm(A @ u - b) <= 1e-9 * np.linalg.norm(b)


def test_count_log_replay_is_identical():
    A, b = _system(seed=13)
    log = CountLog("record")
    x1, s1, _ = fgmres(lambda v: A @ v, b, None, tol=1e-3, maxit=50, log=log, kind="g")
    rep = CountLog("replay", log.data)
    x2, s2, _ = fgmres(lambda v: A @ v, b, None, tol=0.5, maxit=2, log=rep, kind="g")
    assert s1 == s2 and np.array_equal(x1, x2)


def test_zero_rhs():
    A, b = _system()
    x, steps, est = fgmres(lambda v: A @ v, 0 * b, None, tol=1e-6, maxit=5)
    assert steps == 0 and not x.any()


def _krylov_minimiser(A, b, M, j):
    """argmin ||b - A x|| over x in M K_j(A M, b), from an orthonormal basis of
    the explicit Krylov matrix [b, (AM) b, ..., (AM)^{j-1} b] (M = I: GMRES)."""
    cols = [b]
    for _ in range(j - 1):
        cols.append(A @ (M @ cols[-1]))
    Q, _ = np.linalg.qr(np.stack(cols, axis=1))
    y = np.linalg.lstsq(A @ (M @ Q), b, rcond=None)[0]
    return M @ (Q @ y)


@pytest.mark.parametrize("j", [1, 2, 4, 7])
@pytest.mark.parametrize("preconditioned", [False, True])
def test_iterate_minimises_the_residual_over_the_krylov_space(j, preconditioned):
    """The defining property of (F)GMRES with a fixed preconditioner: after
    exactly j steps from zero, x_j minimises ||b - A x|| over M K_j(AM, b).
    Checked at every j, not only at convergence, so a wrong rotation sign, a
    transposed Hessenberg or a misplaced update fails at the step it enters."""
    A, b = _system(n=30, seed=3)
    rng = np.random.default_rng(4)
    M = np.eye(30) + 0.1 * (rng.standard_normal((30, 30)) + 1j * rng.standard_normal((30, 30)))
    if not preconditioned:
        M = np.eye(30)
    x, steps, est = fgmres(lambda v: A @ v, b, (lambda v: M @ v) if preconditioned else None,
                           tol=None, maxit=j)
    assert steps == j
    xr = _krylov_minimiser(A, b, M, j)
    assert np.linalg.norm(x - xr) <= 1e-10 * np.linalg.norm(xr)
    # the estimate is that minimal residual
    assert abs(est - np.linalg.norm(b - A @ xr) / np.linalg.norm(b)) <= 1e-12
