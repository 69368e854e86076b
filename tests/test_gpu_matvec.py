"""GPU parity of the matrix-free and stored-matrix (CSR) forms of the finest
operator (Appendix B of the paper; the matvec comparison table).

  * hm_csr_assemble against the oracle's assembled 5-point Sommerfeld matrix:
    row pointers and column pattern bit-exact, values to rounding (the ghost
    elimination is written independently on the two sides);
  * hm_matfree_apply and hm_csr_spmv of that matrix against the oracle's
    A @ x on every row, for dyadic, ragged and minimal grids;
  * hm_csr_spmv of a general CSR matrix (variable row lengths, empty rows)
    against a host product;
  * at the largest benchmarked workload (4097 x 4097) the two GPU forms against
    the oracle's A @ x on every row;
  * at the largest grid of the matvec sweep (16385 x 16385) the two forms
    against each other on every row and against the oracle's per-row
    evaluation on sampled rows.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import paper_2412_04980_amd as hm
from oracle import operators as op

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def host(t):
    return t.cpu().numpy()


def relerr(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def medium(nx, ny, seed):
    rng = np.random.default_rng(seed)
    k = rng.uniform(20.0, 60.0, nx * ny)
    x = rng.standard_normal(nx * ny) + 1j * rng.standard_normal(nx * ny)
    return k, x


GRIDS = [(3, 3), (17, 17), (33, 65), (37, 29), (129, 129), (300, 7)]


@pytest.mark.parametrize("nx,ny", GRIDS)
def test_csr_assembly_matches_oracle_matrix(nx, ny):
    h = 1.0 / (max(nx, ny) - 1)
    k, _ = medium(nx, ny, nx * 7 + ny)
    rp, ci, va = hm.csr_assemble(nx, ny, h, gpu(k))
    torch.cuda.synchronize()
    rp, ci, va = host(rp), host(ci), host(va)
    n = nx * ny
    assert np.array_equal(rp, 5 * np.arange(n + 1, dtype=np.int32))
    assert ci.min() >= 0 and ci.max() < n
    G = sp.csr_matrix((va, ci, rp), shape=(n, n))
    G.sum_duplicates()
    G.eliminate_zeros()
    A = op.five_point(nx, ny, h, k, 1.0).tocsr()
    A.sum_duplicates()
    A.eliminate_zeros()
    G.sort_indices()
    A.sort_indices()
    assert np.array_equal(G.indptr, A.indptr)
    assert np.array_equal(G.indices, A.indices)
    assert relerr(G.data, A.data) <= 1e-15


@pytest.mark.parametrize("nx,ny", GRIDS)
def test_matfree_and_csr_spmv_match_oracle(nx, ny):
    h = 1.0 / (max(nx, ny) - 1)
    k, x = medium(nx, ny, nx * 11 + ny)
    A = op.five_point(nx, ny, h, k, 1.0)
    ref = A @ x
    kd, xd = gpu(k), gpu(x)
    v = hm.matfree_apply(nx, ny, h, kd, xd)
    rp, ci, va = hm.csr_assemble(nx, ny, h, kd)
    y = hm.csr_spmv(rp, ci, va, xd)
    torch.cuda.synchronize()
    assert relerr(host(v), ref) <= 1e-13
    assert relerr(host(y), ref) <= 1e-13


def test_csr_spmv_general_matrix():
    rng = np.random.default_rng(21)
    nrows, ncols = 1000, 700
    lens = rng.integers(0, 12, nrows)
    lens[::97] = 0                                     # empty rows
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    nnz = int(rp[-1])
    ci = rng.integers(0, ncols, nnz).astype(np.int32)
    va = rng.standard_normal(nnz) + 1j * rng.standard_normal(nnz)
    x = rng.standard_normal(ncols) + 1j * rng.standard_normal(ncols)
    ref = sp.csr_matrix((va, ci, rp), shape=(nrows, ncols)) @ x
    y = hm.csr_spmv(gpu(rp), gpu(ci), gpu(va), gpu(x), ncols=ncols)
    torch.cuda.synchronize()
    y = host(y)
    assert np.all(y[lens == 0] == 0)
    assert relerr(y, ref) <= 1e-14


def test_csr_spmv_column_outside_gives_nan_row():
    """An entry whose column lies outside [0, ncols) is not read from x: its row
    becomes NaN and every other row is the product."""
    rng = np.random.default_rng(22)
    nrows, ncols = 300, 200
    rp = np.arange(0, 3 * nrows + 1, 3, dtype=np.int32)
    ci = rng.integers(0, ncols, 3 * nrows).astype(np.int32)
    bad = [5, 123, 299]
    for r in bad:
        ci[3 * r + 1] = ncols + 7 * r          # past the end of x
    va = rng.standard_normal(3 * nrows) + 1j * rng.standard_normal(3 * nrows)
    x = rng.standard_normal(ncols) + 1j * rng.standard_normal(ncols)
    good = np.setdiff1d(np.arange(nrows), bad)
    ci_ok = ci.copy()
    for r in bad:
        ci_ok[3 * r + 1] = 0
    ref = sp.csr_matrix((va, ci_ok, rp), shape=(nrows, ncols)) @ x
    y = host(hm.csr_spmv(gpu(rp), gpu(ci), gpu(va), gpu(x), ncols=ncols))
    assert np.all(np.isnan(y[bad]))
    assert relerr(y[good], ref[good]) <= 1e-14


def test_matvec_forms_at_4097():
    nx = ny = 4097
    h = 1.0 / 4096
    k, x = medium(nx, ny, 5)
    A = op.five_point(nx, ny, h, k, 1.0)
    ref = A @ x
    del A
    kd, xd = gpu(k), gpu(x)
    v = hm.matfree_apply(nx, ny, h, kd, xd)
    rp, ci, va = hm.csr_assemble(nx, ny, h, kd)
    y = hm.csr_spmv(rp, ci, va, xd)
    torch.cuda.synchronize()
    assert relerr(host(v), ref) <= 1e-13
    assert relerr(host(y), ref) <= 1e-13


def test_matvec_forms_at_16385_sampled():
    """The largest grid of the matvec sweep (268,468,225 rows): both GPU forms
    agree with each other on every row and with the oracle's per-row
    evaluation on 4096 sampled rows plus the four corners and edge midpoints."""
    nx = ny = 16385
    n = nx * ny
    h = 1.0 / (nx - 1)
    rng = np.random.default_rng(11)
    k = rng.uniform(20.0, 60.0, n)
    x = np.empty(n, dtype=np.complex128)
    x.real = rng.standard_normal(n)
    x.imag = rng.standard_normal(n)
    kd, xd = gpu(k), gpu(x)
    v = hm.matfree_apply(nx, ny, h, kd, xd)
    rp, ci, va = hm.csr_assemble(nx, ny, h, kd)
    y = hm.csr_spmv(rp, ci, va, xd)
    del rp, ci, va
    torch.cuda.synchronize()
    scale = float(v.abs().max())
    assert float((v - y).abs().max()) <= 1e-13 * scale
    rows = np.concatenate([rng.integers(0, n, 4096),
                           [0, nx - 1, n - nx, n - 1, nx // 2, n - nx // 2 - 1,
                            (ny // 2) * nx, (ny // 2) * nx + nx - 1]])
    ref = op.five_point_rows(nx, ny, h, k, 1.0, rows, x)
    idx = torch.from_numpy(rows).to(DEV)
    assert np.max(np.abs(host(v[idx]) - ref)) <= 1e-13 * scale
    assert np.max(np.abs(host(y[idx]) - ref)) <= 1e-13 * scale


@pytest.mark.parametrize("bc", [hm.HM_BC_SOMMERFELD, hm.HM_BC_DIRICHLET])
@pytest.mark.parametrize("nx,ny", [(3, 3), (67, 45), (513, 257)])
def test_true_residual_matches_oracle(bc, nx, ny):
    """hm_residual: r = b - A u on every row and its norm against the oracle's
    assembled operator (both boundary conditions), with and without r."""
    h = 1.0 / (max(nx, ny) - 1)
    k, u = medium(nx, ny, 3 * nx + ny)
    rng = np.random.default_rng(nx + 7 * ny)
    b = rng.standard_normal(nx * ny) + 1j * rng.standard_normal(nx * ny)
    bcname = op.DIRICHLET if bc == hm.HM_BC_DIRICHLET else op.SOMMERFELD
    A = op.five_point(nx, ny, h, k, 1.0, bc=bcname)
    ref = b - A @ u
    kd, bd, ud = gpu(k), gpu(b), gpu(u)
    r = torch.empty_like(bd)
    norms = host(hm.residual(nx, ny, h, kd, bd, ud, bc=bc, r=r))
    assert relerr(host(r), ref) <= 1e-13
    assert abs(norms[0] - np.linalg.norm(ref)) <= 1e-12 * np.linalg.norm(ref)
    assert abs(norms[1] - np.linalg.norm(b)) <= 1e-12 * np.linalg.norm(b)
    again = host(hm.residual(nx, ny, h, kd, bd, ud, bc=bc))
    assert np.array_equal(again, norms)

