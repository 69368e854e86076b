"""Pins of the oracle's Dirichlet variant (homogeneous u = 0 on the boundary,
ghost point of eq. ghost_Dirichlt on the coarse levels; oracle.operators).

  * the finest operator's interior block equals the textbook Dirichlet matrix
    built independently as kron(I, T) + kron(T, I) - sigma diag(k^2) with
    T = tridiag(-1, 2, -1) / H^2, and boundary rows are decoupled;
  * constant k: the discrete sine modes, which vanish on the boundary, are
    eigenvectors with the closed-form eigenvalue;
  * coarse levels, constant k: on every row whose stencil reaches at most the
    one-step ghost layer, the sine modes are eigenvectors with the stencil's
    symbol sum (L/h^2 - sigma K k^2) cos(a tx) cos(b ty), because the Dirichlet
    ghost -u_m is exactly the odd extension of the mode and the ghost
    wavenumber 2k_b - k_m equals k;
  * the masked transfers keep boundary-free vectors boundary-free;
  * the MADP solve equals a direct sparse solve, vanishes on the boundary and
    equals the interior-only textbook problem there;
  * a manufactured solution that vanishes on the boundary is reached at second
    order.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workloads
from oracle import operators as op
from oracle import stencils
from oracle.madp import MADP

D = op.DIRICHLET


def _tridiag(n, H):
    return sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]) / H**2


def _sine(nx, ny, p, q):
    i = np.arange(nx)
    j = np.arange(ny)
    return np.outer(np.sin(q * np.pi * j / (ny - 1)), np.sin(p * np.pi * i / (nx - 1))).ravel()


@pytest.mark.parametrize("sigma", [1.0, 1.0 + 0.5j])
def test_five_point_interior_block_is_the_textbook_matrix(sigma):
    nx, ny, H = 9, 7, 0.125
    rng = np.random.default_rng(1)
    k = rng.uniform(2.0, 5.0, nx * ny)
    A = op.five_point(nx, ny, H, k, sigma, bc=D).toarray()
    m = op.interior_mask(nx, ny).astype(bool)
    ki = k[m]
    ref = (sp.kron(sp.eye(ny - 2), _tridiag(nx - 2, H)) + sp.kron(_tridiag(ny - 2, H),
           sp.eye(nx - 2)) - sigma * sp.diags(ki**2)).toarray()
    assert np.allclose(A[np.ix_(m, m)], ref, rtol=0, atol=1e-12)
    assert np.count_nonzero(A[np.ix_(m, ~m)]) == 0
    assert np.count_nonzero(A[np.ix_(~m, m)]) == 0
    assert np.allclose(np.diag(A)[~m], 4.0 / H**2)


def test_five_point_sine_modes():
    nx, ny, H, kval = 17, 13, 1.0 / 16, 7.0
    A = op.five_point(nx, ny, H, np.full(nx * ny, kval), 1.0, bc=D)
    for p, q in ((1, 1), (3, 2), (7, 5)):
        v = _sine(nx, ny, p, q)
        lam = 4 / H**2 * (np.sin(p * np.pi / (2 * (nx - 1))) ** 2 +
                          np.sin(q * np.pi / (2 * (ny - 1))) ** 2) - kval**2
        assert np.allclose(A @ v, lam * v, rtol=0, atol=1e-9 * abs(lam))


@pytest.mark.parametrize("level", [2, 3])
def test_coarse_stencils_sine_modes_away_from_double_ghosts(level):
    nx = ny = 17
    h, kval, sigma = 1.0 / 64, 9.0, 1.0 + 0.5j
    W = op.wide_stencil(nx, ny, h, level, np.full(nx * ny, kval), sigma, bc=D)
    L, K = stencils.stencils_2d_float(level)
    r = L.shape[0] // 2
    # rows whose every nonzero tap lies in the grid or one step out in one direction
    exact = np.zeros((ny, nx), dtype=bool)
    for j in range(1, ny - 1):
        for i in range(1, nx - 1):
            ok = True
            for b in range(-r, r + 1):
                for a in range(-r, r + 1):
                    if L[b + r, a + r] == 0 and K[b + r, a + r] == 0:
                        continue
                    x, y = i + a, j + b
                    ox = 0 if 0 <= x < nx else (1 if x in (-1, nx) else 2)
                    oy = 0 if 0 <= y < ny else (1 if y in (-1, ny) else 2)
                    if ox + oy > 1:
                        ok = False
            exact[j, i] = ok
    exact = exact.ravel()
    assert exact.sum() > 0.5 * (nx - 2) * (ny - 2)
    for p, q in ((1, 1), (2, 5), (6, 3)):
        tx, ty = p * np.pi / (nx - 1), q * np.pi / (ny - 1)
        v = _sine(nx, ny, p, q)
        sym = sum((L[b + r, a + r] / h**2 - sigma * K[b + r, a + r] * kval**2) *
                  np.cos(a * tx) * np.cos(b * ty)
                  for b in range(-r, r + 1) for a in range(-r, r + 1))
        Wv = W @ v
        assert np.allclose(Wv[exact], sym * v[exact], rtol=0, atol=1e-9 * abs(sym))


def test_masked_transfers_keep_vectors_boundary_free():
    nxc, nyc = 9, 7
    nxf, nyf = 2 * nxc - 1, 2 * nyc - 1
    rng = np.random.default_rng(2)
    vf = rng.standard_normal(nxf * nyf) * op.interior_mask(nxf, nyf)
    vc = rng.standard_normal(nxc * nyc) * op.interior_mask(nxc, nyc)
    bf = ~op.interior_mask(nxf, nyf).astype(bool)
    bcm = ~op.interior_mask(nxc, nyc).astype(bool)
    Z = op.deflation_z(nxc, nyc, D)
    assert np.all((Z.T @ vf)[bcm] == 0) and np.all((Z @ vc)[bf] == 0)
    assert np.all((op.full_weighting(nxf, nyf, D) @ vf)[bcm] == 0)
    assert np.all((op.bilinear_prolongation(nxc, nyc, D) @ vc)[bf] == 0)
    # masking is the only change: on boundary-free vectors the interior values agree
    Zs = op.deflation_z(nxc, nyc)
    inner = ~bcm
    assert np.allclose((Z.T @ vf)[inner], (Zs.T @ vf)[inner])


@pytest.mark.parametrize("kval,n", [(0.0, 33), (6.0, 33), (12.0, 41)])
def test_madp_dirichlet_solve_is_the_textbook_solution(kval, n):
    """kval = 0 is the degenerate case of the method: the Poisson problem, with
    the CSLP equal to the operator itself."""
    h = 1.0 / (n - 1)
    rng = np.random.default_rng(3)
    k = kval * rng.uniform(0.9, 1.1, n * n)
    m = MADP(n, n, h, k, levels=3, bc=D)
    b = workloads.point_source(n, n, h, n // 2, n // 2 + 3)
    u, info = m.solve(b, tol=1e-11)
    ud = spla.spsolve(m.levels[1].A.tocsc(), b)
    assert np.linalg.norm(u - ud) <= 1e-8 * np.linalg.norm(ud)
    inner = op.interior_mask(n, n).astype(bool)
    assert np.all(np.abs(u[~inner]) <= 1e-12 * np.abs(u).max())
    T = _tridiag(n - 2, h)
    Ai = sp.kron(sp.eye(n - 2), T) + sp.kron(T, sp.eye(n - 2)) - sp.diags(k[inner] ** 2)
    ui = spla.spsolve(Ai.tocsc(), b[inner])
    assert np.linalg.norm(u[inner] - ui) <= 1e-8 * np.linalg.norm(ui)


def test_manufactured_solution_second_order():
    """u = sin(pi x) sin(2 pi y) (1 + x y) vanishes on the boundary of the unit
    square; with f = -Lap u - k^2 u the Dirichlet discretisation converges to it
    at second order."""
    kval = 6.0
    errs = []
    for n in (17, 33, 65, 129):
        h = 1.0 / (n - 1)
        x = np.arange(n) * h
        Y, X = np.meshgrid(x, x, indexing="ij")
        s1, c1 = np.sin(np.pi * X), np.cos(np.pi * X)
        s2, c2 = np.sin(2 * np.pi * Y), np.cos(2 * np.pi * Y)
        g = 1 + X * Y
        u = s1 * s2 * g
        lap = (-(np.pi**2) * s1 * s2 * g + 2 * np.pi * c1 * s2 * Y
               - 4 * np.pi**2 * s1 * s2 * g + 4 * np.pi * s1 * c2 * X)
        f = (-lap - kval**2 * u).ravel().astype(np.complex128)
        inner = op.interior_mask(n, n).astype(bool)
        f[~inner] = 0.0
        A = op.five_point(n, n, h, np.full(n * n, kval), 1.0, bc=D)
        uh = spla.spsolve(A.tocsc(), f)
        errs.append(np.max(np.abs(uh - u.ravel())))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert all(1.9 <= r <= 2.1 for r in rates), (errs, rates)
