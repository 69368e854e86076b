"""Multigrid V-cycle approximating the CSLP inverse (oracle; test infrastructure).

Sec. 3.2 and Sec. 4.4 of the paper replace the Krylov approximation of the CSLP
inverse on the first and second levels by one multigrid V-cycle with complex
shift beta2 = 0.5 and defer the settings to the authors' earlier matrix-free
multigrid.  Those settings are not printed, so this module fixes a reading
(reading R10):

  * V(1,1) cycle, damped Jacobi x <- x + omega D^-1 (b - M x), first sweep from
    x = 0; omega_q = 0.8 where k_max^2 H_q^2 <= 1 and 0.5 otherwise (H_q the
    spacing of multigrid level q);
  * full-weighting restriction of the residual, bilinear prolongation of the
    correction;
  * the top operator is the CSLP of the deflation level (5-point on the finest
    level, Galerkin-derived 5x5 on the second); every coarser multigrid level
    uses s_l times the 5-point CSLP at its spacing with the wavenumber injected;
  * coarsen while (nx-1) and (ny-1) are both even and the coarse grid keeps at
    least 3 nodes per direction;
  * coarsest level: dense LU when it has at most DENSE_MAX unknowns, otherwise
    unpreconditioned GMRES to relative tolerance 0.1 with at most
    floor(6 N^(1/4)) steps (the Krylov CSLP rule of Sec. 4.2).

Pins: fixed point = exact solve (iterating x <- x + V(b - Mx) converges to the
direct solution), single-level case = dense solve, transfer identities
(R = P^T / 4, bilinear exactness on linear functions).  The multigrid settings
themselves are "parity unpinned" by the paper (only GPU-vs-oracle).
"""
import math

import numpy as np
import scipy.linalg as sla

from . import operators as op
from .krylov import fgmres

DENSE_MAX = 512


def smoothing_weight(kmax, H):
    """omega_q of reading R10."""
    return 0.8 if kmax * kmax * H * H <= 1.0 else 0.5


def krylov_maxit(N, coef=6.0):
    """Maximum Krylov steps for a CSLP solve on N unknowns: floor(coef N^(1/4))."""
    return max(1, int(math.floor(coef * N ** 0.25)))


def can_coarsen(nx, ny):
    return (nx - 1) % 2 == 0 and (ny - 1) % 2 == 0 and (nx - 1) // 2 + 1 >= 3 \
        and (ny - 1) // 2 + 1 >= 3


class MGLevel:
    def __init__(self, nx, ny, H, k, M, omega):
        self.nx, self.ny, self.H, self.k = nx, ny, H, k
        self.M = M
        self.diag = M.diagonal()
        self.omega = omega


class VCycle:
    """Multigrid hierarchy for one CSLP operator.

    top_operator: CSR of the CSLP at the top level (nx x ny, spacing H0);
    scale: s_l applied to the re-discretised coarse multigrid operators.
    """

    def __init__(self, nx, ny, H0, k, top_operator, sigma, scale, kmax=None,
                 nu_pre=1, nu_post=1, tol_cslp=0.1, maxit_coef=6.0, log=None,
                 bc=op.SOMMERFELD):
        kmax = float(np.max(k)) if kmax is None else kmax
        self.nu_pre, self.nu_post = nu_pre, nu_post
        self.tol_cslp, self.maxit_coef = tol_cslp, maxit_coef
        self.log = log
        self.levels = [MGLevel(nx, ny, H0, k, top_operator, smoothing_weight(kmax, H0))]
        self.R, self.P = [], []
        while can_coarsen(nx, ny):
            nxc, nyc = op.coarse_size(nx, 2), op.coarse_size(ny, 2)
            kc = op.inject(k, nx, ny)
            Hc = 2 * self.levels[-1].H
            Mc = op.five_point(nxc, nyc, Hc, kc, sigma, scale, bc=bc)
            self.R.append(op.full_weighting(nx, ny, bc=bc))
            self.P.append(op.bilinear_prolongation(nxc, nyc, bc=bc))
            self.levels.append(MGLevel(nxc, nyc, Hc, kc, Mc, smoothing_weight(kmax, Hc)))
            nx, ny, k = nxc, nyc, kc
        last = self.levels[-1]
        N = last.nx * last.ny
        self.dense = N <= DENSE_MAX
        if self.dense:
            self.lu = sla.lu_factor(last.M.toarray())
        self.coarse_maxit = krylov_maxit(N, maxit_coef)

    def coarse_solve(self, b):
        last = self.levels[-1]
        if self.dense:
            return sla.lu_solve(self.lu, b)
        x, _, _ = fgmres(lambda v: last.M @ v, b, None, tol=self.tol_cslp,
                         maxit=self.coarse_maxit, log=self.log, kind="mg_coarse")
        return x

    def _cycle(self, q, b):
        lev = self.levels[q]
        if q == len(self.levels) - 1:
            return self.coarse_solve(b)
        x = lev.omega * b / lev.diag                      # first sweep from x = 0
        for _ in range(self.nu_pre - 1):
            x = x + lev.omega * (b - lev.M @ x) / lev.diag
        r = b - lev.M @ x
        ec = self._cycle(q + 1, self.R[q] @ r)
        x = x + self.P[q] @ ec
        for _ in range(self.nu_post):
            x = x + lev.omega * (b - lev.M @ x) / lev.diag
        return x

    def __call__(self, b):
        return self._cycle(0, np.asarray(b, dtype=np.complex128))
