"""Pins of the assembled operators (oracle.operators).

Checked against what the mathematics fixes, not against a retyped formula:
the discrete plane-wave symbol of the 5-point operator, the complex symmetry
that the paper states for the Sommerfeld system (after the boundary-row
scaling), second-order convergence of a manufactured solution with
inhomogeneous Sommerfeld data, and interpolation identities of the transfers.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import operators as op


def _grid(n, h):
    x = np.arange(n) * h
    Y, X = np.meshgrid(x, x, indexing="ij")
    return X.ravel(), Y.ravel()


@pytest.mark.parametrize("sigma", [1.0, 1.0 + 0.5j])
def test_five_point_plane_wave_symbol(sigma):
    n, h = 21, 1.0 / 20
    rng = np.random.default_rng(0)
    k = rng.uniform(3, 9, n * n)
    X, Y = _grid(n, h)
    al, be = 2.1, -4.3
    u = np.exp(1j * (al * X + be * Y))
    Au = op.five_point(n, n, h, k, sigma) @ u
    sym = (4 - 2 * np.cos(al * h) - 2 * np.cos(be * h)) / h**2 - sigma * k**2
    ii = np.arange(n * n) % n
    jj = np.arange(n * n) // n
    interior = (ii > 0) & (ii < n - 1) & (jj > 0) & (jj < n - 1)
    assert np.allclose(Au[interior], (sym * u)[interior], rtol=1e-12, atol=1e-9)


def test_sommerfeld_system_is_complex_symmetric_after_row_scaling():
    """Sec. 2.1: with Sommerfeld conditions the matrix is symmetric; with the ghost
    eliminated this holds once boundary rows are halved (corners quartered)."""
    nx, ny, h = 9, 7, 0.1
    k = np.random.default_rng(1).uniform(1, 5, nx * ny)
    A = op.five_point(nx, ny, h, k, 1.0 + 0.5j)
    ii = np.arange(nx * ny) % nx
    jj = np.arange(nx * ny) // nx
    w = np.where((ii == 0) | (ii == nx - 1), 0.5, 1.0) * np.where((jj == 0) | (jj == ny - 1), 0.5, 1.0)
    S = (sp.diags(w) @ A).toarray()
    assert np.allclose(S, S.T, rtol=0, atol=1e-12 * np.abs(S).max())
    assert not np.allclose(S, S.conj().T)          # non-Hermitian


def _manufactured_error(n, kval=5.0):
    h = 1.0 / (n - 1)
    X, Y = _grid(n, h)
    al, be = 0.3, 0.7
    phi = np.exp(1j * (al * X + be * Y))
    w = 1 + X * Y
    u = phi * w
    f = phi * ((al**2 + be**2 - kval**2) * w - 2j * (al * Y + be * X))
    ux = phi * (1j * al * w + Y)
    uy = phi * (1j * be * w + X)
    b = f.copy()
    ii = np.arange(n * n) % n
    jj = np.arange(n * n) // n
    # g = du/dn - i k u on each side; ghost elimination adds 2 g / h to the row
    for mask, dn in (((ii == 0), -ux), ((ii == n - 1), ux), ((jj == 0), -uy), ((jj == n - 1), uy)):
        g = dn - 1j * kval * u
        b = b + np.where(mask, 2 * g / h, 0)
    A = op.five_point(n, n, h, np.full(n * n, kval), 1.0)
    uh = spla.spsolve(A.tocsc(), b)
    return np.max(np.abs(uh - u))


def test_manufactured_solution_second_order():
    errs = [_manufactured_error(n) for n in (17, 33, 65, 129)]
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert all(1.9 <= r <= 2.1 for r in rates), (errs, rates)


def test_deflation_z_interpolates_linear_functions():
    nc = 9
    Z = op.deflation_z(nc, nc)
    nf = 2 * nc - 1
    Xc, Yc = _grid(nc, 2.0)
    Xf, Yf = _grid(nf, 1.0)
    c = 3.0 + 0.5 * Xc - 1.25 * Yc
    f = Z @ c
    ii = np.arange(nf * nf) % nf
    jj = np.arange(nf * nf) // nf
    inner = (ii >= 2) & (ii <= nf - 3) & (jj >= 2) & (jj <= nf - 3)
    assert np.allclose(f[inner], (3.0 + 0.5 * Xf - 1.25 * Yf)[inner], atol=1e-13)
    # boundary truncation (reading R4): fine corner gets (6/8)^2 of coarse corner
    # plus the neighbours' 1/8 weights
    e = np.zeros(nc * nc); e[0] = 1.0
    assert np.isclose((Z @ e)[0], (6 / 8) ** 2)


def test_full_weighting_is_quarter_bilinear_transpose():
    nxf, nyf = 17, 9
    R = op.full_weighting(nxf, nyf)
    P = op.bilinear_prolongation(op.coarse_size(nxf, 2), op.coarse_size(nyf, 2))
    assert abs(R - P.T / 4).max() < 1e-15


def test_bilinear_exact_on_bilinear_functions():
    nc = 6
    P = op.bilinear_prolongation(nc, nc)
    Xc, Yc = _grid(nc, 2.0)
    Xf, Yf = _grid(2 * nc - 1, 1.0)
    assert np.allclose(P @ (1 + Xc + 2 * Yc + 0.5 * Xc * Yc), 1 + Xf + 2 * Yf + 0.5 * Xf * Yf)


def test_injection():
    f = np.arange(5 * 7, dtype=float)
    c = op.inject(f, 5, 7)
    assert c.tolist() == [f[j * 5 + i] for j in range(0, 7, 2) for i in range(0, 5, 2)]


def test_wide_stencil_consistent_with_scaled_continuous_operator():
    """The Galerkin scale: on constant k the level-3 operator applied to a smooth
    plane wave approximates s_3 (-Delta - k^2) u = 16 (a^2 + b^2 - k^2) u on
    interior rows.  (The boundary-row rule, reading R7, is parity unpinned.)"""
    n1 = 4 * 16 + 1
    h = 1.0 / (n1 - 1)
    n3 = op.coarse_size(n1, 4)
    k = np.full(n3 * n3, 3.0)
    W = op.wide_stencil(n3, n3, h, 3, k, 1.0)
    X, Y = _grid(n3, 4 * h)
    al, be = 1.0, 2.0
    u = np.exp(1j * (al * X + be * Y))
    Wu = W @ u
    cont = 16 * (al**2 + be**2 - 9.0) * u
    ii = np.arange(n3 * n3) % n3
    jj = np.arange(n3 * n3) // n3
    interior = (ii >= 3) & (ii <= n3 - 4) & (jj >= 3) & (jj <= n3 - 4)
    assert np.allclose(Wu[interior], cont[interior], rtol=2e-2)


@pytest.mark.parametrize("bc", ["sommerfeld", "dirichlet"])
def test_five_point_rows_match_the_assembled_matrix(bc):
    """The per-row evaluation used for sampled checks on grids too large to
    assemble equals the assembled operator on every row of a small grid."""
    nx, ny, H = 11, 8, 0.1
    rng = np.random.default_rng(3)
    k = rng.uniform(1.0, 4.0, nx * ny)
    x = rng.standard_normal(nx * ny) + 1j * rng.standard_normal(nx * ny)
    A = op.five_point(nx, ny, H, k, 1.0 + 0.5j, bc=bc)
    got = op.five_point_rows(nx, ny, H, k, 1.0 + 0.5j, np.arange(nx * ny), x, bc=bc)
    assert np.allclose(got, A @ x, rtol=0, atol=1e-12 * np.abs(A @ x).max())


def _flip_x(v, nx, ny):
    return np.asarray(v).reshape(ny, nx)[:, ::-1].ravel()


def _flip_y(v, nx, ny):
    return np.asarray(v).reshape(ny, nx)[::-1, :].ravel()


def _swap_xy(v, nx, ny):
    return np.asarray(v).reshape(ny, nx).T.ravel()


@pytest.mark.parametrize("bc", [op.SOMMERFELD, op.DIRICHLET])
@pytest.mark.parametrize("level", [1, 2, 3, 4, 5, 6])
def test_level_operators_commute_with_grid_symmetries(level, bc):
    """The boundary band of the coarse operators (readings R7, R8, R24) has no
    printed values, but the discretisation must treat the four sides and the two
    axes alike: the operator built from a reflected (or transposed) medium,
    applied to the reflected (transposed) vector, gives the reflected
    (transposed) result.  A ghost rule slipped on one side, a mirror index off by
    one, or x and y exchanged in a tap breaks this on the rows next to that side.
    Oblong grid, random medium and vector; the two sides differ only in the
    order of each row's sum."""
    nx, ny, h, sigma = 15, 19, 1.0 / 32, 1.0 + 0.5j
    rng = np.random.default_rng(40 + level)
    k = rng.uniform(2.0, 6.0, nx * ny)
    u = rng.standard_normal(nx * ny) + 1j * rng.standard_normal(nx * ny)
    Au = op.level_operator(nx, ny, h, level, k, sigma, bc=bc) @ u
    scale = np.max(np.abs(Au))
    for flip in (_flip_x, _flip_y):
        got = op.level_operator(nx, ny, h, level, flip(k, nx, ny), sigma, bc=bc) @ flip(u, nx, ny)
        assert np.max(np.abs(got - flip(Au, nx, ny))) <= 1e-12 * scale, flip.__name__
    # transposition maps an nx x ny grid to an ny x nx one
    got = op.level_operator(ny, nx, h, level, _swap_xy(k, nx, ny), sigma, bc=bc) @ _swap_xy(u, nx, ny)
    assert np.max(np.abs(got - _swap_xy(Au, nx, ny))) <= 1e-12 * scale
