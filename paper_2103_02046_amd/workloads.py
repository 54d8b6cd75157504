"""Seeded synthetic bunches shaped like the beam workloads of the paper.

This module only draws inputs and fixes run parameters (mesh spacing, cutoff,
Ewald split, time step). It holds none of the P3M arithmetic, so both the
CPU oracle and the GPU library can be fed from it without sharing any part of
the method.

Units are SI. A bunch carries a total charge of -1 nC split equally over N
macro-particles; every macro-particle has the charge-to-mass ratio of an
electron, so a macro-particle of charge q has mass m = q * m_e / (-e).

The time step is a fixed fraction of the plasma period of the initial peak
number density n0: omega_p^2 = n0 q^2 / (eps0 m), dt = (2 pi / omega_p) / 200.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

E_CHARGE = 1.602176634e-19       # C
M_ELECTRON = 9.1093837015e-31    # kg
EPS0 = 8.8541878128e-12          # F/m
K_E = 8.9875517923e9             # 1/(4 pi eps0), N m^2 / C^2
C_LIGHT = 299792458.0            # m/s
BUNCH_CHARGE = -1e-9             # C

# Mesh order: 1 = cloud-in-cell (linear B-spline), 2 = triangular-shaped cloud
# (quadratic B-spline).
CIC = 1
TSC = 2


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    n: int
    grid: tuple          # mesh nodes per dimension (N_x, N_y, N_z)
    h: tuple             # mesh spacing at zoom 1 [m]
    r_cut: float         # PP cutoff at zoom 1 [m]
    split: float         # Ewald split parameter alpha [1/m]
    order: int           # CIC or TSC
    dt: float            # time step [s]
    steps: int           # leapfrog steps of the run
    q: float             # macro-particle charge [C]
    m: float             # macro-particle mass [kg]
    n0: float            # initial peak number density [1/m^3]
    seed: int = 0
    pp_cell_div: int = 1  # PP cells per cutoff along each axis (2: half-size cells, for dense cores)

    @property
    def ke_q2(self) -> float:
        return K_E * self.q * self.q

    def draw(self):
        """Return (x, p) as float64 arrays of shape (n, 3); p is zero (cold beam)."""
        x = _DRAWS[self.name](self.n, self.seed)
        return x, np.zeros_like(x)


def _macro(n):
    q = BUNCH_CHARGE / n
    m = q * M_ELECTRON / (-E_CHARGE)
    return q, m


def _dt(n0, q, m):
    omega_p = math.sqrt(n0 * q * q / (EPS0 * m))
    return (2.0 * math.pi / omega_p) / 200.0


def _usable(order, nodes):
    # Nodes the bunch may span so that every assignment stencil stays on the mesh.
    return nodes - 1 if order == CIC else nodes - 2


# ---- draws (fixed draw order, numpy PCG64) --------------------------------

def _draw_gauss_iso(n, seed, sigma=1e-3):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, 3)) * sigma


def _draw_gauss_aniso(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, 3)) * np.array([1e-3, 1e-3, 3e-3])


def _draw_sphere(n, seed, radius=1e-3):
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = radius * rng.random(n) ** (1.0 / 3.0)
    return d * r[:, None]


def halo_split(n):
    n_core = int(round(0.9 * n))
    return n_core, n - n_core


def _draw_halo(n, seed, sigma_core=5e-4, r_halo=5e-3):
    # Halo: number density proportional to r^-2 between the core's sigma and
    # r_halo, i.e. radii uniform on [sigma_core, r_halo], isotropic. (Down to
    # r = 0 the r^-2 law would put a cusp at the centre whose closest pairs,
    # a nanometre apart, a fixed-step leapfrog throws out of the bunch.)
    rng = np.random.default_rng(seed)
    n_core, n_halo = halo_split(n)
    core = rng.standard_normal((n_core, 3)) * sigma_core
    r = sigma_core + rng.random(n_halo) * (r_halo - sigma_core)
    d = rng.standard_normal((n_halo, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return np.concatenate([core, d * r[:, None]], axis=0)


_DRAWS = {
    "gauss": _draw_gauss_iso,
    "aniso": _draw_gauss_aniso,
    "sphere": _draw_sphere,
    "halo": _draw_halo,
}


# ---- the five configurations ----------------------------------------------

def gauss_cic(n=4096, grid=32, steps=10, seed=0):
    """Isotropic Gaussian (sigma 1 mm), +-4 sigma over the usable node span, CIC, r_c = 2h."""
    sigma = 1e-3
    h = 8 * sigma / _usable(CIC, grid)
    rc = 2 * h
    q, m = _macro(n)
    n0 = n / ((2 * math.pi) ** 1.5 * sigma ** 3)
    return Workload("gauss", n, (grid,) * 3, (h,) * 3, rc, 3.0 / rc, CIC,
                    _dt(n0, q, m), steps, q, m, n0, seed)


def aniso_tsc(n=1 << 20, grid=128, steps=100, seed=0):
    """Gaussian sigma = (1, 1, 3) mm, +-4 sigma per axis, TSC, r_c = 2 h_x."""
    sig = (1e-3, 1e-3, 3e-3)
    h = tuple(8 * s / _usable(TSC, grid) for s in sig)
    rc = 2 * h[0]
    q, m = _macro(n)
    n0 = n / ((2 * math.pi) ** 1.5 * sig[0] * sig[1] * sig[2])
    return Workload("aniso", n, (grid,) * 3, h, rc, 3.0 / rc, TSC,
                    _dt(n0, q, m), steps, q, m, n0, seed)


def sphere_tsc(n=1 << 23, grid=256, steps=200, seed=0):
    """Uniform ball of radius 1 mm at rest, diameter over the usable span, TSC, r_c = 2.5h."""
    radius = 1e-3
    h = 2 * radius / _usable(TSC, grid)
    rc = 2.5 * h
    q, m = _macro(n)
    n0 = n / (4.0 / 3.0 * math.pi * radius ** 3)
    return Workload("sphere", n, (grid,) * 3, (h,) * 3, rc, 3.0 / rc, TSC,
                    _dt(n0, q, m), steps, q, m, n0, seed)


def halo_tsc(n=1 << 25, grid=512, steps=50, seed=0):
    """90% Gaussian core (sigma 0.5 mm) + 10% 1/r^2 halo from sigma to 10 sigma, TSC, r_c = 2h."""
    sigma_c, r_halo = 5e-4, 5e-3
    h = 2 * r_halo / _usable(TSC, grid)
    rc = 2 * h
    q, m = _macro(n)
    n_core, _ = halo_split(n)
    n0 = n_core / ((2 * math.pi) ** 1.5 * sigma_c ** 3)
    # the core holds ~10^3 particles per cutoff cube: half-size PP cells
    # (about 10^2 each) still fill the pair kernel's groups of 16
    return Workload("halo", n, (grid,) * 3, (h,) * 3, rc, 3.0 / rc, TSC,
                    _dt(n0, q, m), steps, q, m, n0, seed, pp_cell_div=2)


CONFIGS = {
    "gauss4k": gauss_cic,       # 4096 particles, 32^3 mesh, CIC, 10 steps, FP64
    "aniso1m": aniso_tsc,       # 2^20 particles, 128^3 mesh, TSC, 100 steps
    "sphere8m": sphere_tsc,     # 2^23 particles, 256^3 mesh, TSC, 200 steps
    "halo32m": halo_tsc,        # 2^25 particles, 512^3 mesh, TSC, 50 steps
}


def get(name, **kw):
    return CONFIGS[name](**kw)
