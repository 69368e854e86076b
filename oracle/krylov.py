"""(F)GMRES with modified Gram-Schmidt (oracle; test infrastructure).

Follows Algorithm 1 of the paper: zero initial guess, Arnoldi with modified
Gram-Schmidt, h_ij = (w, v_i) = v_i^H w (reading R13), Hessenberg least
squares y = argmin || beta e1 - H y || and u = u0 + X y with X the flexible
basis of preconditioned vectors (Z = V when there is no preconditioner, i.e.
plain GMRES).

Stopping rule (reading R11): after Arnoldi step j stop when the least-squares
residual estimate |g_{j+1}| <= tol * ||rhs|| (<=, computed by Givens
rotations), or when j = maxit, or on happy breakdown h_{j+1,j} <= 1e-14 ||rhs||.
At least one step is always taken.  `tol=None` means "run exactly maxit steps".

Count logging: a CountLog in "record" mode appends the number of steps every
solve took under a kind label; in "replay" mode each solve of that kind takes
exactly the recorded number of steps (tolerance test off).  This makes the
nonlinear, tolerance-driven preconditioner a fixed linear map for parity tests.

Pins: agreement with a dense direct solve (tol 1e-12), the estimate |g_{j+1}|
equalling the true residual norm, and exact termination in n steps on an n x n
system (tests/test_oracle_krylov.py).
"""
import numpy as np


class CountLog:
    """Per-kind iteration counts of inner solves, recorded or replayed."""

    def __init__(self, mode="record", data=None):
        assert mode in ("record", "replay", "off")
        self.mode = mode
        self.data = {k: list(v) for k, v in (data or {}).items()}
        self._pos = {k: 0 for k in self.data}

    def forced(self, kind):
        if self.mode != "replay":
            return None
        pos = self._pos.get(kind, 0)
        self._pos[kind] = pos + 1
        return self.data[kind][pos]

    def record(self, kind, n):
        if self.mode == "record":
            self.data.setdefault(kind, []).append(int(n))


def givens(a, b):
    """Unitary rotation (c real, s complex) with [c s; -conj(s) c] [a; b] = [r; 0]."""
    if b == 0:
        return 1.0, 0j
    if a == 0:
        return 0.0, 1.0 + 0j
    aa = abs(a)
    nrm = np.hypot(aa, abs(b))
    c = aa / nrm
    s = (a / aa) * np.conj(b) / nrm
    return c, s


def fgmres(apply_a, rhs, precond=None, tol=None, maxit=1, log=None, kind=None,
           breakdown=1e-14):
    """One cycle of (F)GMRES from a zero initial guess.

    Returns (x, steps, estimate) where estimate = |g_{steps+1}| / ||rhs||.
    """
    rhs = np.asarray(rhs, dtype=np.complex128)
    beta = np.linalg.norm(rhs)
    if beta == 0.0:
        if log is not None and kind is not None:
            log.record(kind, 0)
        return np.zeros_like(rhs), 0, 0.0
    forced = log.forced(kind) if (log is not None and kind is not None) else None
    if forced is not None:
        maxit, tol = forced, None
    V = [rhs / beta]
    Zs = []
    H = np.zeros((maxit + 1, maxit), dtype=np.complex128)
    R = np.zeros((maxit + 1, maxit), dtype=np.complex128)   # rotated copy
    cs, sn = [], []
    g = np.zeros(maxit + 1, dtype=np.complex128)
    g[0] = beta
    steps = 0
    for j in range(maxit):
        z = precond(V[j]) if precond is not None else V[j]
        Zs.append(z)
        w = apply_a(z)
        for i in range(j + 1):                      # modified Gram-Schmidt
            H[i, j] = np.vdot(V[i], w)
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        # least-squares residual estimate via Givens rotations
        col = H[: j + 2, j].copy()
        for i in range(j):
            t = cs[i] * col[i] + sn[i] * col[i + 1]
            col[i + 1] = -np.conj(sn[i]) * col[i] + cs[i] * col[i + 1]
            col[i] = t
        c, s = givens(col[j], col[j + 1])
        cs.append(c); sn.append(s)
        col[j] = c * col[j] + s * col[j + 1]
        col[j + 1] = 0.0
        R[: j + 2, j] = col
        g[j + 1] = -np.conj(s) * g[j]
        g[j] = c * g[j]
        steps = j + 1
        broke = H[j + 1, j].real <= breakdown * beta
        if not broke:
            V.append(w / H[j + 1, j])
        if broke:
            break
        if tol is not None and abs(g[j + 1]) <= tol * beta:
            break
    # y = argmin || beta e1 - Hbar y ||  (Algorithm 1, final step)
    Hbar = H[: steps + 1, :steps]
    e1 = np.zeros(steps + 1, dtype=np.complex128)
    e1[0] = beta
    y = np.linalg.lstsq(Hbar, e1, rcond=None)[0]
    x = np.zeros_like(rhs)
    for i in range(steps):
        x = x + y[i] * Zs[i]
    if log is not None and kind is not None:
        log.record(kind, steps)
    return x, steps, abs(g[steps]) / beta


def fgmres_restarted(apply_a, b, precond, tol=1e-6, restart=30, maxit=300, log=None,
                     kind="outer"):
    """Outer FGMRES (reading R12): cycles of at most `restart` steps from the
    current iterate, each stopping when the estimate reaches tol*||b||; the
    true residual is recomputed after every cycle and the solve ends when it is
    within tolerance or `maxit` steps have been taken."""
    b = np.asarray(b, dtype=np.complex128)
    bnorm = np.linalg.norm(b)
    u = np.zeros_like(b)
    total = 0
    history = []
    while True:
        r = b - apply_a(u)
        rnorm = np.linalg.norm(r)
        history.append(rnorm / bnorm if bnorm else 0.0)
        if bnorm == 0.0 or rnorm <= tol * bnorm or total >= maxit:
            break
        m = min(restart, maxit - total)
        # the cycle tolerance is relative to ||r||; scale so it means tol*||b||
        du, steps, _ = fgmres(apply_a, r, precond, tol=tol * bnorm / rnorm, maxit=m,
                              log=log, kind=kind)
        u = u + du
        total += steps
    return u, total, history[-1]
