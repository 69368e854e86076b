"""MADP: matrix-free multilevel adapted deflation preconditioner (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Operators are assembled
CSR matrices; the steps follow Algorithm 1 of the paper (recursive two-level
deflated FGMRES) with the MADP configuration of Sec. 4.4:

  level l preconditioner  Prec_l(v):
      v_hat = Z_l^T v                                   (restriction)
      if l+1 is the coarsest level L:
          v_t = m FGMRES steps on E_{l+1} v_t = v_hat, preconditioned by the
                CSLP of level l+1 approximated by GMRES (tol 0.1,
                at most floor(6 N^(1/4)) steps)
      else:
          v_t = FGMRES on E_{l+1} v_t = v_hat preconditioned by Prec_{l+1},
                to relative tolerance 0.3 on level 2, m steps on levels >= 3
      t  = Z_l v_t                                      (interpolation)
      r~ = v - A_l t
      r  = CSLP_l^-1 r~   (one multigrid V-cycle on levels 1-2, GMRES below)
      return r + t                                      (x = r + t)

  outer solve: FGMRES on A_1 u = b with Prec_1, zero initial guess, stop at
  ||b - A u|| / ||b|| <= 1e-6 (Sec. 4), restart 30, at most 300 steps.

A_1 is the 5-point Helmholtz operator; E_l (l >= 2) and the CSLP operators M_l
are the re-discretised Galerkin-derived stencils (Sec. 3.3).  The optional
`galerkin_coarse=True` replaces E_{l+1} by the exact Z^T A Z product and the
coarsest solve by a dense direct solve, and `cslp_override` replaces the CSLP
approximation of a level by a given map; both exist only for the deflation
identities of Sec. 3.1 (tests).

Variants of the same algorithm (Sec. 3.2, the cycle type, and Sec. 4.4-4.5):
`coarse_steps` is m, the fixed number of FGMRES steps on every coarse level
that has no tolerance (1: V-cycle, the MADP setting; 2: W-cycle);
`tol_levels` is the deepest level that iterates to `tol_level2` instead (2: MADP;
1: every coarse level takes m steps; 3 or 4: the tolerance also on the third
and fourth levels, the variant of the per-level tolerance table of Sec. 4.5).
The coarsest level always takes m steps.  MADP-v3 is tol_level2 = 0.1.
`bc` selects Sommerfeld (default) or homogeneous Dirichlet boundaries on every
level (reading R24, oracle.operators).
"""
import time

import numpy as np
import scipy.linalg as sla

from . import operators as op
from . import stencils
from .krylov import CountLog, fgmres, fgmres_restarted
from .multigrid import VCycle, krylov_maxit


class Level:
    def __init__(self, l, nx, ny, h, k, beta, bc=op.SOMMERFELD):
        self.l, self.nx, self.ny = l, nx, ny
        self.N = nx * ny
        self.h_l = h * 2 ** (l - 1)
        self.s_l = float(stencils.level_scale(l))
        self.k = k
        sigma = complex(beta[0], beta[1])
        self.A = op.level_operator(nx, ny, h, l, k, 1.0, bc=bc)     # A_1 or E_l
        self.M = op.level_operator(nx, ny, h, l, k, sigma, bc=bc)   # CSLP of the level
        self.Z = None                                         # to level l+1


class MADP:
    def __init__(self, nx, ny, h, k, levels=3, beta=(1.0, 0.5), tol_level2=0.3,
                 tol_cslp=0.1, maxit_coef=6.0, level2_maxit=100, nu_pre=1, nu_post=1,
                 log=None, galerkin_coarse=False, cslp_override=None, coarse_steps=1,
                 tol_levels=2, bc=op.SOMMERFELD):
        assert levels >= 2 and coarse_steps >= 1 and tol_levels >= 1
        f = 2 ** (levels - 1)
        if (nx - 1) % f or (ny - 1) % f:
            raise ValueError("(n-1) must be divisible by 2^(levels-1)")
        self.L = levels
        self.beta = beta
        self.tol_level2, self.tol_cslp = tol_level2, tol_cslp
        self.maxit_coef, self.level2_maxit = maxit_coef, level2_maxit
        self.coarse_steps, self.tol_levels = coarse_steps, tol_levels
        self.log = log if log is not None else CountLog("record")
        self.galerkin_coarse = galerkin_coarse
        self.cslp_override = dict(cslp_override or {})
        sigma = complex(beta[0], beta[1])
        t0 = time.perf_counter()
        self.levels = [None]                                  # 1-based
        k = np.asarray(k, dtype=np.float64).ravel()
        for l in range(1, levels + 1):
            self.levels.append(Level(l, nx, ny, h, k, beta, bc))
            if l < levels:
                nxc, nyc = op.coarse_size(nx, 2), op.coarse_size(ny, 2)
                self.levels[l].Z = op.deflation_z(nxc, nyc, bc)
                k = op.inject(k, nx, ny)
                nx, ny = nxc, nyc
        if galerkin_coarse:
            for l in range(2, levels + 1):
                Zp = self.levels[l - 1].Z
                self.levels[l].A = (Zp.conj().T @ self.levels[l - 1].A @ Zp).tocsr()
        # CSLP approximations: V-cycles on levels 1-2
        self.mg = {}
        for l in range(1, min(2, levels) + 1):
            lev = self.levels[l]
            self.mg[l] = VCycle(lev.nx, lev.ny, lev.h_l, lev.k, lev.M, sigma, lev.s_l,
                                nu_pre=nu_pre, nu_post=nu_post, tol_cslp=tol_cslp,
                                maxit_coef=maxit_coef, log=self.log, bc=bc)
        self.setup_seconds = time.perf_counter() - t0

    # -- CSLP^-1 on level l ------------------------------------------------
    def cslp(self, l, r):
        if l in self.cslp_override:
            return self.cslp_override[l](r)
        if l in self.mg:
            return self.mg[l](r)
        lev = self.levels[l]
        x, _, _ = fgmres(lambda v: lev.M @ v, r, None, tol=self.tol_cslp,
                         maxit=krylov_maxit(lev.N, self.maxit_coef), log=self.log,
                         kind="cslp_l%d" % l)
        return x

    # -- coarse problem E_{l+1} v_t = v_hat -----------------------------------
    def coarse(self, l, v_hat):
        c = l + 1
        lev = self.levels[c]
        if self.galerkin_coarse and c == self.L:
            return sla.solve(lev.A.toarray(), v_hat)
        if c == self.L:
            x, _, _ = fgmres(lambda v: lev.A @ v, v_hat, lambda v: self.cslp(c, v),
                             tol=None, maxit=self.coarse_steps)
            return x
        if c <= self.tol_levels:
            tol, maxit = self.tol_level2, self.level2_maxit
        else:
            tol, maxit = None, self.coarse_steps
        x, _, _ = fgmres(lambda v: lev.A @ v, v_hat, lambda v: self.precond(c, v),
                         tol=tol, maxit=maxit, log=self.log, kind="level%d" % c)
        return x

    def precond(self, l, v):
        """Prec_l(v) = M_l^-1 (v - A_l Z v_t) + Z v_t, v_t ~ E^-1 Z^T v."""
        lev = self.levels[l]
        v_hat = lev.Z.conj().T @ v
        v_t = self.coarse(l, v_hat)
        t = lev.Z @ v_t
        r_t = v - lev.A @ t
        r = self.cslp(l, r_t)
        return r + t

    def apply(self, v):
        """One application of the finest-level preconditioner."""
        return self.precond(1, np.asarray(v, dtype=np.complex128))

    def solve(self, b, tol=1e-6, restart=30, maxit=300):
        A = self.levels[1].A
        t0 = time.perf_counter()
        u, its, rel = fgmres_restarted(lambda v: A @ v, b, self.apply, tol=tol,
                                       restart=restart, maxit=maxit, log=self.log)
        info = {"outer_iters": its, "rel_res_true": rel,
                "seconds": time.perf_counter() - t0,
                "level2_iters_total": sum(self.log.data.get("level2", [])),
                "cslp_iters_total": sum(self.log.data.get("cslp_l%d" % self.L, []))}
        return u, info

