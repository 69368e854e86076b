"""Assembled (CSR) operators of the MADP hierarchy (oracle; test infrastructure).

Grid convention: a level holds nx*ny vertex-centred nodes including the
boundary nodes (Sec. 2.1); node (i, j) has index j*nx + i (x fastest).
All matrices are scipy.sparse CSR in complex128.

Readings of the paper this module fixes:
  * Sommerfeld ghost point (Sec. 2.1, eq. ghost_sommerfeld): the ghost behind a
    boundary node b, mirrored from the interior neighbour m, is
    u_ghost = u_m + 2 i H k_b u_b, with H the spacing of the grid concerned.
    Boundary rows are not rescaled (reading R2).
  * CSLP (Sec. 3.1, eq. CSLP def): sigma = beta1 + i beta2 multiplies only the
    k^2 term; the Sommerfeld ghost keeps the unshifted k (reading R9).
  * Coarse levels l >= 2 (Sec. 3.3): interior and near-boundary rows use the
    Galerkin-derived stencils with the wavenumber read at each stencil point,
    (K u)_I = sum K[a,b] k^2_{I+(a,b)} u_{I+(a,b)} (reading R6).  A stencil
    point one step outside the grid in exactly one direction is a ghost point
    with the Sommerfeld value above at spacing h_l and zero wavenumber; points
    further out, or outside in both directions, are zero (reading R8).
    Boundary-node rows are s_l times the standard 5-point operator at spacing
    h_l (reading R7), s_l = 4^(l-1).
  * Deflation vectors: Z = p (x) p, p = [1,4,6,4,1]/8, truncated at the
    boundary; Z^T is its exact transpose (readings R3, R4).
  * Multigrid transfers: full weighting (1/16)[1 2 1; 2 4 2; 1 2 1] with
    out-of-grid fine values zero, bilinear interpolation, wavenumber by
    injection (reading R10).

Dirichlet boundaries (Sec. 2.1, eq. ghost_Dirichlt; Sec. 3.3 boundary paragraph),
reading R24: homogeneous, u = 0 on every boundary node.  The boundary nodes stay
in the grid but are decoupled: a boundary row is d_b u_b with d_b = s_l 4 / h_l^2,
and no other row reads a boundary value (it is zero).  A stencil point one step
outside the grid in exactly one direction is the ghost 2 u_b - u_m = -u_m with
wavenumber k_g = 2 k_b - k_m (b the boundary node, m its interior neighbour);
points further out are zero.  Every transfer is masked to the interior:
Z_D = D_f Z D_c, R_D = D_c R D_f, P_D = D_f P D_c with D the 0/1 interior masks,
so vectors that vanish on the boundary keep vanishing at every level.
"""
import numpy as np
import scipy.sparse as sp

from . import stencils

_NEIGHBOURS = ((-1, 0), (1, 0), (0, -1), (0, 1))


SOMMERFELD, DIRICHLET = "sommerfeld", "dirichlet"


def interior_mask(nx, ny):
    """1.0 on nodes off the boundary, 0.0 on boundary nodes (row-major)."""
    m = np.zeros((ny, nx))
    m[1:-1, 1:-1] = 1.0
    return m.ravel()


def _mask_rows_cols(M, rows_mask, cols_mask):
    return (sp.diags(rows_mask) @ M @ sp.diags(cols_mask)).tocsr()


def coarse_size(n, factor):
    """Nodes of a grid with (n-1) intervals coarsened by `factor` (must divide)."""
    assert (n - 1) % factor == 0
    return (n - 1) // factor + 1


def inject(field, nx, ny):
    """Injection of a nodal field onto the next coarser grid: f_c(J) = f(2J)."""
    f = np.asarray(field).reshape(ny, nx)
    return np.ascontiguousarray(f[::2, ::2]).ravel()


def five_point(nx, ny, H, k, sigma, scale=1.0, bc=SOMMERFELD):
    """scale * ( H^-2 (4u - sum of 4 neighbours) - sigma k^2 u ) with a Sommerfeld
    ghost point behind every boundary side (Sec. 2.1, eqs. helm operator h and
    ghost_sommerfeld; with sigma = beta1 + i beta2 it is the CSLP, Sec. 3.1).

    `k` is the nodal wavenumber (not squared).  Rows of corner nodes receive a
    ghost from both directions.  bc = "dirichlet": reading R24 (module docstring).
    """
    if bc == DIRICHLET:
        return _five_point_dirichlet(nx, ny, H, k, sigma, scale)
    k = np.asarray(k, dtype=np.float64).reshape(ny, nx)
    jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    idx = jj * nx + ii
    rows, cols, vals = [], [], []
    off = -scale / H**2
    diag = scale * (4.0 / H**2 - sigma * k**2) + 0j
    for di, dj in _NEIGHBOURS:
        ni, nj = ii + di, jj + dj
        inside = (ni >= 0) & (ni < nx) & (nj >= 0) & (nj < ny)
        rows.append(idx[inside]); cols.append((nj * nx + ni)[inside])
        vals.append(np.full(inside.sum(), off, dtype=np.complex128))
        out = ~inside
        # ghost u_g = u_mirror + 2 i H k_b u_b ; mirror is the opposite neighbour
        mi, mj = ii - di, jj - dj
        rows.append(idx[out]); cols.append((mj * nx + mi)[out])
        vals.append(np.full(out.sum(), off, dtype=np.complex128))
        diag = diag + np.where(out, off * 2j * H * k, 0.0)
    rows.append(idx.ravel()); cols.append(idx.ravel()); vals.append(diag.ravel())
    N = nx * ny
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(N, N)).tocsr()


def five_point_rows(nx, ny, H, k, sigma, rows, x, scale=1.0, bc=SOMMERFELD):
    """Selected rows of five_point(...) @ x, each computed from its definition
    (the stencil with the ghost of eq. ghost_sommerfeld, or the Dirichlet rule
    of reading R24) without assembling the matrix: for grids too large to
    assemble, where outputs are checked at sampled nodes."""
    rows = np.asarray(rows, dtype=np.int64)
    k = np.asarray(k).ravel()
    x = np.asarray(x).ravel()
    i, j = rows % nx, rows // nx
    def val(ii, jj):
        ok = (ii >= 0) & (ii < nx) & (jj >= 0) & (jj < ny)
        out = np.zeros(len(rows), dtype=np.complex128)
        out[ok] = x[(jj * nx + ii)[ok]]
        return out, ok
    uc = x[rows]
    if bc == DIRICHLET:
        bnd = (i == 0) | (j == 0) | (i == nx - 1) | (j == ny - 1)
        s = 4.0 * uc
        for di, dj in _NEIGHBOURS:
            ii, jj = i + di, j + dj
            v, _ = val(ii, jj)
            nb = (ii == 0) | (jj == 0) | (ii == nx - 1) | (jj == ny - 1)
            s = s - np.where(nb, 0.0, v)
        inner = scale * (s / H**2 - sigma * k[rows] ** 2 * uc)
        return np.where(bnd, scale * 4.0 / H**2 * uc, inner)
    s = 4.0 * uc
    for di, dj in _NEIGHBOURS:
        v, ok = val(i + di, j + dj)
        mirror, _ = val(i - di, j - dj)
        ghost = mirror + 2j * H * k[rows] * uc          # u_g = u_m + 2 i H k_b u_b
        s = s - np.where(ok, v, ghost)
    return scale * (s / H**2 - sigma * k[rows] ** 2 * uc)


def _five_point_dirichlet(nx, ny, H, k, sigma, scale):
    k = np.asarray(k, dtype=np.float64).ravel()
    m = interior_mask(nx, ny).astype(bool)
    N = nx * ny
    rows, cols, vals = [], [], []
    idx = np.arange(N)
    ii, jj = idx % nx, idx // nx
    # interior rows: centre and the interior neighbours (boundary values are zero)
    rows.append(idx[m]); cols.append(idx[m])
    vals.append(scale * (4.0 / H**2 - sigma * k[m] ** 2) + 0j)
    for di, dj in _NEIGHBOURS:
        ni, nj = ii + di, jj + dj
        ok = m.copy()
        ok[m] = m[(nj * nx + ni)[m]]
        rows.append(idx[ok]); cols.append((nj * nx + ni)[ok])
        vals.append(np.full(ok.sum(), -scale / H**2, dtype=np.complex128))
    # boundary rows: d_b u_b
    rows.append(idx[~m]); cols.append(idx[~m])
    vals.append(np.full((~m).sum(), scale * 4.0 / H**2, dtype=np.complex128))
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(N, N)).tocsr()


def _wide_dirichlet(nx, ny, h, level, k, sigma):
    L, K = stencils.stencils_2d_float(level)
    r = L.shape[0] // 2
    hl = h * 2 ** (level - 1)
    sl = float(stencils.level_scale(level))
    k2d = np.asarray(k, dtype=np.float64).reshape(ny, nx)
    N = nx * ny
    interior = interior_mask(nx, ny).reshape(ny, nx).astype(bool)
    rows, cols, vals = [], [], []
    for j in range(1, ny - 1):
        for i in range(1, nx - 1):
            I = j * nx + i
            for b in range(-r, r + 1):
                for a in range(-r, r + 1):
                    lap, wav = L[b + r, a + r] / h**2, K[b + r, a + r]
                    x, y = i + a, j + b
                    xin, yin = 0 <= x < nx, 0 <= y < ny
                    if xin and yin:
                        if interior[y, x]:
                            rows.append(I); cols.append(y * nx + x)
                            vals.append(lap - sigma * wav * k2d[y, x] ** 2)
                        continue
                    if yin and x in (-1, nx):          # ghost in x: -u_m, k_g = 2k_b - k_m
                        xb, xm = (0, 1) if x < 0 else (nx - 1, nx - 2)
                        if interior[y, xm]:
                            kg = 2 * k2d[y, xb] - k2d[y, xm]
                            rows.append(I); cols.append(y * nx + xm)
                            vals.append(-(lap - sigma * wav * kg**2))
                    elif xin and y in (-1, ny):        # ghost in y
                        yb, ym = (0, 1) if y < 0 else (ny - 1, ny - 2)
                        if interior[ym, x]:
                            kg = 2 * k2d[yb, x] - k2d[ym, x]
                            rows.append(I); cols.append(ym * nx + x)
                            vals.append(-(lap - sigma * wav * kg**2))
    bnd = np.flatnonzero(~interior.ravel())
    rows.extend(bnd.tolist()); cols.extend(bnd.tolist())
    vals.extend([sl * 4.0 / hl**2] * len(bnd))
    return sp.coo_matrix((np.asarray(vals, dtype=np.complex128), (rows, cols)),
                         shape=(N, N)).tocsr()


def wide_stencil(nx, ny, h, level, k, sigma, bc=SOMMERFELD):
    """Re-discretised coarse operator of deflation level `level` >= 2 (Sec. 3.3).

    h is the FINEST spacing (the printed stencils are in units of h^-2); the
    level spacing is h_l = 2^(l-1) h.  Interior/near-boundary rows:
        sum_{a,b} ( h^-2 L[b,a] - sigma K[b,a] k^2_{I+(a,b)} ) u_{I+(a,b)}
    with the ghost/zero rule for points outside the grid; boundary rows are
    s_l * five_point at spacing h_l.  bc = "dirichlet": reading R24.

    Parity: interior rows are pinned (rows of the assembled Galerkin triple
    product, plane-wave consistency).  The values of the boundary band (rows
    whose taps leave the grid) are parity unpinned: the paper prints none.  Its
    consistency across the four sides and the two axes is pinned by the grid
    symmetries (reflections and transposition of medium and vector).
    """
    if bc == DIRICHLET:
        return _wide_dirichlet(nx, ny, h, level, k, sigma)
    L, K = stencils.stencils_2d_float(level)
    r = L.shape[0] // 2
    hl = h * 2 ** (level - 1)
    sl = float(stencils.level_scale(level))
    k2d = np.asarray(k, dtype=np.float64).reshape(ny, nx)
    N = nx * ny
    jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    interior = (ii > 0) & (ii < nx - 1) & (jj > 0) & (jj < ny - 1)
    ii_in, jj_in = ii[interior], jj[interior]
    I_in = jj_in * nx + ii_in
    rows, cols, vals = [], [], []
    for b in range(-r, r + 1):
        for a in range(-r, r + 1):
            lap = L[b + r, a + r] / h**2
            wav = K[b + r, a + r]
            if lap == 0.0 and wav == 0.0:
                continue
            pi, pj = ii_in + a, jj_in + b
            xin = (pi >= 0) & (pi < nx)
            yin = (pj >= 0) & (pj < ny)
            inside = xin & yin
            P = pj * nx + pi
            kp = np.where(inside, k2d[np.clip(pj, 0, ny - 1), np.clip(pi, 0, nx - 1)], 0.0)
            rows.append(I_in[inside]); cols.append(P[inside])
            vals.append((lap - sigma * wav * kp[inside] ** 2).astype(np.complex128))
            # ghost: one step outside in x only
            for side_x, bnd_i, mir_i in ((-1, 0, 1), (nx, nx - 1, nx - 2)):
                g = (pi == side_x) & yin
                if g.any():
                    pjg = pj[g]
                    kb = k2d[pjg, bnd_i]
                    rows.append(I_in[g]); cols.append(pjg * nx + mir_i)
                    vals.append(np.full(g.sum(), lap, dtype=np.complex128))
                    rows.append(I_in[g]); cols.append(pjg * nx + bnd_i)
                    vals.append(lap * 2j * hl * kb)
            # ghost: one step outside in y only
            for side_y, bnd_j, mir_j in ((-1, 0, 1), (ny, ny - 1, ny - 2)):
                g = (pj == side_y) & xin
                if g.any():
                    pig = pi[g]
                    kb = k2d[bnd_j, pig]
                    rows.append(I_in[g]); cols.append(mir_j * nx + pig)
                    vals.append(np.full(g.sum(), lap, dtype=np.complex128))
                    rows.append(I_in[g]); cols.append(bnd_j * nx + pig)
                    vals.append(lap * 2j * hl * kb)
    W = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N)).tocsr()
    B = five_point(nx, ny, hl, k, sigma, scale=sl)
    bmask = (~interior).ravel()
    D = sp.diags(bmask.astype(np.float64))
    Dc = sp.diags((~bmask).astype(np.float64))
    return (Dc @ W + D @ B).tocsr()


def level_operator(nx, ny, h, level, k, sigma, bc=SOMMERFELD):
    """Operator of deflation level `level`: the 5-point operator on the finest
    level, the Galerkin-derived wide stencil on coarser levels."""
    if level == 1:
        return five_point(nx, ny, h, k, sigma, 1.0, bc=bc)
    return wide_stencil(nx, ny, h, level, k, sigma, bc=bc)


def _bezier_1d(nc):
    """1-D quadratic-Bezier deflation interpolation, fine (2nc-1) x coarse nc."""
    nf = 2 * (nc - 1) + 1
    p = [1 / 8, 4 / 8, 6 / 8, 4 / 8, 1 / 8]
    rows, cols, vals = [], [], []
    for J in range(nc):
        for s in range(-2, 3):
            i = 2 * J + s
            if 0 <= i < nf:
                rows.append(i); cols.append(J); vals.append(p[s + 2])
    return sp.csr_matrix((vals, (rows, cols)), shape=(nf, nc))


def deflation_z(nxc, nyc, bc=SOMMERFELD):
    """Z from the coarse grid (nxc x nyc) to the fine grid: p (x) p, truncated;
    masked to the interior for Dirichlet boundaries (reading R24)."""
    Z = sp.kron(_bezier_1d(nyc), _bezier_1d(nxc)).tocsr().astype(np.complex128)
    if bc == DIRICHLET:
        nxf, nyf = 2 * (nxc - 1) + 1, 2 * (nyc - 1) + 1
        Z = _mask_rows_cols(Z, interior_mask(nxf, nyf), interior_mask(nxc, nyc))
    return Z


def _bilinear_1d(nc):
    nf = 2 * (nc - 1) + 1
    rows, cols, vals = [], [], []
    for J in range(nc):
        rows.append(2 * J); cols.append(J); vals.append(1.0)
        if 2 * J - 1 >= 0:
            rows.append(2 * J - 1); cols.append(J); vals.append(0.5)
        if 2 * J + 1 < nf:
            rows.append(2 * J + 1); cols.append(J); vals.append(0.5)
    return sp.csr_matrix((vals, (rows, cols)), shape=(nf, nc))


def bilinear_prolongation(nxc, nyc, bc=SOMMERFELD):
    """Bilinear interpolation coarse -> fine (multigrid prolongation); masked to
    the interior for Dirichlet boundaries."""
    P = sp.kron(_bilinear_1d(nyc), _bilinear_1d(nxc)).tocsr().astype(np.complex128)
    if bc == DIRICHLET:
        nxf, nyf = 2 * (nxc - 1) + 1, 2 * (nyc - 1) + 1
        P = _mask_rows_cols(P, interior_mask(nxf, nyf), interior_mask(nxc, nyc))
    return P


def _full_weighting_1d(nf):
    nc = coarse_size(nf, 2)
    rows, cols, vals = [], [], []
    for J in range(nc):
        for a, w in ((-1, 0.25), (0, 0.5), (1, 0.25)):
            if 0 <= 2 * J + a < nf:
                rows.append(J); cols.append(2 * J + a); vals.append(w)
    return sp.csr_matrix((vals, (rows, cols)), shape=(nc, nf))


def full_weighting(nxf, nyf, bc=SOMMERFELD):
    """Full-weighting restriction fine -> coarse with weights (1/16)[1 2 1;2 4 2;1 2 1]
    centred at fine node 2J; fine nodes outside the grid contribute zero.  The
    2-D weights are the outer product of the 1-D weights [1, 2, 1]/4.  Masked to
    the interior for Dirichlet boundaries."""
    R = sp.kron(_full_weighting_1d(nyf), _full_weighting_1d(nxf)).tocsr().astype(np.complex128)
    if bc == DIRICHLET:
        nxc, nyc = coarse_size(nxf, 2), coarse_size(nyf, 2)
        R = _mask_rows_cols(R, interior_mask(nxc, nyc), interior_mask(nxf, nyf))
    return R
