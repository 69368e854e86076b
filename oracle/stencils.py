"""Coarse-level stencils by exact Galerkin coarsening (oracle; test infrastructure).

Sec. 3.3 of the paper derives the third-level Laplace and wavenumber stencils by
applying Galerkin coarsening with the higher-order deflation vectors to the
5-point stencils (equations "Glk Laplace 4h" and "ReD-Glk K 4h"), and lists the
fourth- to sixth-level ones in Appendix A.  The deflation vectors are not
printed; they are the quadratic-Bezier interpolation of Dwarka & Vuik, whose
1-D weights at fine offsets -2..2 around the coarse node are p = [1,4,6,4,1]/8
(reading R3).  With Z = p (x) p the 2-D Galerkin product separates:

    Laplace_l   = h^-2 (t_l (x) m_l + m_l (x) t_l)
    wavenumber_l = k^2 (m_l (x) m_l)

where t_1 = [-1, 2, -1], m_1 = [1] and every further level is the 1-D Galerkin
product  s_{l+1}[D] = sum_{a,b} p_a p_b s_l[2D + b - a].

Everything here is exact (fractions.Fraction).  Pins: the printed stencils of
Sec. 3.3 and Appendix A (tests/golden), and an assembled sparse triple product
Z^T A Z on a finite grid whose interior rows must equal these tables.
"""
from fractions import Fraction

import numpy as np

# 1-D quadratic-Bezier interpolation weights, fine offsets -2..2 (reading R3).
P_WEIGHTS = (Fraction(1, 8), Fraction(4, 8), Fraction(6, 8), Fraction(4, 8), Fraction(1, 8))


def galerkin_1d(s):
    """One Galerkin coarsening step of a symmetric 1-D stencil (list of Fractions,
    odd length, centred).  Returns the coarse stencil c[D] = sum p_a p_b s[2D+b-a]."""
    r = len(s) // 2
    rc = (r + 4) // 2                      # largest |D| with a nonzero term
    out = []
    for D in range(-rc, rc + 1):
        acc = Fraction(0)
        for a in range(-2, 3):
            for b in range(-2, 3):
                idx = 2 * D + b - a
                if -r <= idx <= r:
                    acc += P_WEIGHTS[a + 2] * P_WEIGHTS[b + 2] * s[idx + r]
        out.append(acc)
    # strip zero ends (keeps tables minimal; they are symmetric)
    while len(out) > 1 and out[0] == 0 and out[-1] == 0:
        out = out[1:-1]
    return out


def one_d_tables(level):
    """(t_l, m_l) for deflation level `level` >= 1, exact."""
    t = [Fraction(-1), Fraction(2), Fraction(-1)]
    m = [Fraction(1)]
    for _ in range(level - 1):
        t = galerkin_1d(t)
        m = galerkin_1d(m)
    return t, m


def _pad(v, n):
    r = (n - len(v)) // 2
    return [Fraction(0)] * r + list(v) + [Fraction(0)] * r


def stencils_2d(level):
    """Exact 2-D stencils (Laplace in units of h^-2, wavenumber in units of k^2)
    of deflation level `level` as square lists of Fractions, indexed [b][a] with
    b the y offset and a the x offset (both centred)."""
    t, m = one_d_tables(level)
    n = max(len(t), len(m))
    t, m = _pad(t, n), _pad(m, n)
    lap = [[t[a] * m[b] + m[a] * t[b] for a in range(n)] for b in range(n)]
    wav = [[m[a] * m[b] for a in range(n)] for b in range(n)]
    return lap, wav


def stencils_2d_float(level):
    """The same tables as float64 numpy arrays (Laplace / h^-2, wavenumber / k^2)."""
    lap, wav = stencils_2d(level)
    return (np.array([[float(x) for x in row] for row in lap]),
            np.array([[float(x) for x in row] for row in wav]))


def level_scale(level):
    """s_l = 4^(l-1): the sum of the level-l wavenumber stencil (Galerkin scale)."""
    return 4 ** (level - 1)
