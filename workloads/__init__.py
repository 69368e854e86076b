"""Seeded synthetic inputs: wavenumber fields, right-hand sides, request streams.

This module holds no arithmetic of the solver: it only builds inputs (grids,
velocity models, k = 2 pi f / c, point sources) that both the GPU library's
tests/benchmark and the CPU oracle consume.  The paper's wedge and Marmousi
models are not available as data (the wedge exists only in a figure, the
Marmousi model is a public dataset that is not shipped), so synthetic
stand-ins with the same sizes and structure are generated here:

  constant   constant k on the unit square, Sommerfeld on all sides (MP-1b,
             Sec. 2.2), point source at the centre
  wedge      three-layer wedge on 600 m x 1000 m (Sec. 2.3): interfaces
             z1 = 400 - x/3, z2 = 600 + x/3; c = 2000 / 1500 / 3000 m/s
  layered    30 folded layers, velocities increasing with depth in
             [1500, 5500] m/s, 3 dipping faults, Gaussian smoothing
             (stand-in for the Marmousi model of Sec. 2.4)
  serving    Poisson request stream of Gaussian-random-field media

Grid convention everywhere: nx*ny nodes including the boundary, node (i, j)
at index j*nx + i, x fastest; for the geophysical models j counts depth.
"""
import math
from dataclasses import dataclass, field

import numpy as np
from scipy import ndimage


@dataclass
class Problem:
    name: str
    nx: int
    ny: int
    h: float
    k: np.ndarray                     # float64, nx*ny nodal wavenumber
    sources: list = field(default_factory=list)   # list of (i, j) nodes

    def rhs(self, s=0):
        """Discrete point source (Dirac delta) 1/h^2 at source s."""
        b = np.zeros(self.nx * self.ny, dtype=np.complex128)
        i, j = self.sources[s]
        b[j * self.nx + i] = 1.0 / self.h**2
        return b


def point_source(nx, ny, h, i, j):
    b = np.zeros(nx * ny, dtype=np.complex128)
    b[j * nx + i] = 1.0 / h**2
    return b


def constant(n_interior, k, name=None):
    """Unit square, (n_interior+2)^2 nodes, h = 1/(n_interior+1), source at the centre."""
    n = n_interior + 2
    h = 1.0 / (n - 1)
    return Problem(name or "constant_k%g_n%d" % (k, n), n, n, h,
                   np.full(n * n, float(k)), [((n - 1) // 2, (n - 1) // 2)])


def wedge_velocity(nx, ny, h):
    x = np.arange(nx) * h
    z = np.arange(ny) * h
    Z, X = np.meshgrid(z, x, indexing="ij")
    z1 = 400.0 - X / 3.0
    z2 = 600.0 + X / 3.0
    c = np.full((ny, nx), 1500.0)
    c[Z < z1] = 2000.0
    c[Z >= z2] = 3000.0
    return c.ravel()


def wedge(f=40.0, h=1.0):
    """Wedge stand-in: 600 m x 1000 m, node on an interface takes the deeper layer."""
    nx, ny = int(round(600 / h)) + 1, int(round(1000 / h)) + 1
    c = wedge_velocity(nx, ny, h)
    k = 2 * math.pi * f / c
    return Problem("wedge_f%g" % f, nx, ny, h, k, [(int(round(300 / h)), int(round(1 / h)))])


def layered_velocity(nx, ny, h, seed=3, n_layers=30, n_faults=3):
    rng = np.random.default_rng(seed)
    Lx, Lz = (nx - 1) * h, (ny - 1) * h
    x = np.arange(nx) * h
    z = np.arange(ny) * h
    amp = rng.uniform(20, 120, n_layers - 1)
    lam = rng.uniform(2000, 6000, n_layers - 1)
    phi = rng.uniform(0, 2 * np.pi, n_layers - 1)
    vel = np.sort(rng.uniform(1500, 5500, n_layers))
    base = Lz * np.arange(1, n_layers) / n_layers
    iface = base[:, None] + amp[:, None] * np.sin(2 * np.pi * x[None, :] / lam[:, None] + phi[:, None])
    iface = np.maximum.accumulate(iface, axis=0)            # keep the order with depth
    x0 = rng.uniform(1000, 8000, n_faults)
    dip = np.deg2rad(rng.uniform(55, 75, n_faults))
    throw = rng.uniform(50, 250, n_faults)
    Z, X = np.meshgrid(z, x, indexing="ij")
    zq = Z.copy()
    for f in range(n_faults):
        # fault line x = x0 + z / tan(dip); hanging wall (x beyond the line) shifted up
        hanging = X > x0[f] + Z / np.tan(dip[f])
        zq = np.where(hanging, zq - throw[f], zq)
    layer = np.zeros_like(Z, dtype=np.int64)
    for i in range(n_layers - 1):
        layer += (zq >= iface[i][None, :]).astype(np.int64)
    c = vel[layer]
    c = ndimage.gaussian_filter(c, sigma=20.0 / h, mode="reflect")
    return c.ravel()


def layered(f=20.0, h=2.0, seed=3, n_rhs=8):
    """Layered-and-faulted stand-in for the Marmousi model: 9192 m x 2904 m."""
    nx, ny = int(round(9192 / h)) + 1, int(round(2904 / h)) + 1
    c = layered_velocity(nx, ny, h, seed)
    k = 2 * math.pi * f / c
    src = [(int(round(9192 * (s + 0.5) / n_rhs / h)), 1) for s in range(n_rhs)]
    return Problem("layered_f%g" % f, nx, ny, h, k, src)


def gaussian_random_velocity(n, rng, mean=2500.0, std=500.0, corr=0.05):
    """Gaussian random field on n x n nodes of the unit square, Gaussian covariance
    with correlation length `corr`, renormalised to the exact mean/std, clipped."""
    w = rng.standard_normal((n, n))
    fx = np.fft.fftfreq(n, d=1.0 / (n - 1))
    KX, KY = np.meshgrid(fx, fx, indexing="ij")
    filt = np.exp(-(np.pi * corr) ** 2 * (KX**2 + KY**2) / 2.0)
    g = np.real(np.fft.ifft2(np.fft.fft2(w) * filt))
    g = (g - g.mean()) / g.std()
    return np.clip(mean + std * g, 1000.0, 4000.0).ravel()


def smooth_field(nx, ny, seed, sigma=2.0):
    """Complex Gaussian noise on nx x ny nodes smoothed by a Gaussian of width
    sigma nodes (reflecting edges): a smooth seeded test vector, the kind of
    input a coarse level receives from the deflation restriction."""
    rng = np.random.default_rng(seed)
    re = ndimage.gaussian_filter(rng.standard_normal((ny, nx)), sigma, mode="reflect")
    im = ndimage.gaussian_filter(rng.standard_normal((ny, nx)), sigma, mode="reflect")
    return (re + 1j * im).ravel()


@dataclass
class Request:
    rid: int
    arrival: float
    problem: Problem


def serving_stream(n_requests=500, rate=50.0, seed=4, sizes=(255, 511, 1023, 2047)):
    """Poisson arrivals; each request draws a grid class, a random medium and 1-4
    interior point sources at least 8 nodes from the boundary; k chosen so that
    k0^3 h^2 = 0.5 and k = k0 * 2500 / c."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for r in range(n_requests):
        t += rng.exponential(1.0 / rate)
        n_int = int(rng.choice(sizes))
        n = n_int + 2
        h = 1.0 / (n - 1)
        k0 = (0.5 / h**2) ** (1.0 / 3.0)
        c = gaussian_random_velocity(n, rng)
        k = k0 * 2500.0 / c
        ns = int(rng.integers(1, 5))
        src = [(int(rng.integers(8, n - 8)), int(rng.integers(8, n - 8))) for _ in range(ns)]
        out.append(Request(r, t, Problem("serve_n%d" % n, n, n, h, k, src)))
    return out


def config(index):
    """The five benchmark workloads by index (see module docstring)."""
    if index == 0:
        return constant(127, 20.0, "constant_k20_129")
    if index == 1:
        return constant(4095, 200.0, "constant_k200_4097")
    if index == 2:
        return wedge(40.0, 1.0)
    if index == 3:
        return layered(20.0, 2.0)
    raise ValueError("config 4 is a request stream: use serving_stream()")
