"""FP64 CPU oracle of the P3M force evaluation, leapfrog step and its adjoint.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this module; the product path never does. It
shares no code with the GPU library and imports nothing from it.

Paper: Wyssling & Adelmann, arXiv 2103.02046. Each function cites the
passage it follows. Where the paper is silent the readings are:

  * placement: the mesh is centred on the bunch's bounding box each
    evaluation and zoomed by s >= 1 so every assignment stencil fits
    (h' = s h, r_c' = s r_c, a' = a / s);
  * the mesh kernel is the erf part of the Ewald split sampled on the mesh,
    with the Gaussian screening folded into the kernel rather than into the
    assignment (Sec. 2.2 shows the two are the same convolution); no
    deconvolution of the assignment function;
  * the open boundary is realised by zero padding to a doubled mesh (the
    aperiodic convolution of N nodes needs offsets up to N-1 only);
  * the force is the variational one of eq. eom_p3m_coord: minus the weight
    gradient against the mesh potential;
  * leapfrog is kick-drift-kick with p = m v.

The C part (p3m_oracle.c) holds the particle loops; FFTs are numpy's.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np
from scipy.special import erf, erfc, ive

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "p3m_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, ENOMEM, EDOMAIN, ENONFINITE = 0, -1, -2, -5, -6


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: status {code}")
        self.code = code


def build(force=False):
    """Compile the C part with gcc (plain -O2, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC",
                               "-shared", "-std=c11", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None
_lib_path = None


def build_native(out_path):
    """Compile the C part for the host it runs on (-O3 -march=native, OpenMP,
    still no FMA contraction) into out_path, for timing the oracle as a
    CPU baseline; the arithmetic is the same as build()'s."""
    tmp = out_path + ".tmp"
    subprocess.check_call(["gcc", "-O3", "-march=native", "-fopenmp", "-ffp-contract=off", "-fPIC",
                           "-shared", "-std=c11", _SRC, "-o", tmp, "-lm"])
    os.replace(tmp, out_path)
    return out_path


def use_library(path):
    """Load the C part from path (a build_native output) instead of the default build."""
    global _lib, _lib_path
    _lib, _lib_path = None, path
    return lib()


def lib():
    global _lib
    if _lib is None:
        path = _lib_path
        if path is None:
            build()
            path = _LIB
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i64, dbl, i32 = ctypes.c_int64, ctypes.c_double, ctypes.c_int
        sig = {
            "oracle_placement": (i32, [i64, P, P, P, i32, i32, i32, P]),
            "oracle_pp_brute": (None, [i64, P, P, dbl, dbl, dbl, P]),
            "oracle_pp_cells": (i32, [i64, P, P, dbl, dbl, dbl, P]),
            "oracle_pp_sample": (i32, [i64, P, P, dbl, dbl, dbl, i64, P, P]),
            "oracle_pp_energy": (dbl, [i64, P, P, dbl, dbl, dbl]),
            "oracle_deposit": (i32, [i64, P, P, P, P, P, i32, P]),
            "oracle_green": (dbl, [i64, i64, i64, P, dbl]),
            "oracle_conv_direct": (None, [P, P, dbl, P, P]),
            "oracle_phi_image_point": (dbl, [P, P, P, dbl, dbl, P, P]),
            "oracle_conv_direct_image": (None, [P, P, P, dbl, dbl, P, P]),
            "oracle_phi_at": (None, [P, P, dbl, P, i64, P, P]),
            "oracle_stencil_nodes": (i32, [P, P, P, P, i32, P]),
            "oracle_gather": (i32, [i64, P, P, P, P, P, i32, P, dbl, P]),
            "oracle_gather_momentum": (i32, [i64, P, P, P, P, P, i32, P, dbl, P]),
            "oracle_pp_hvp": (None, [i64, P, P, dbl, dbl, dbl, P, P]),
            "oracle_deposit_grad": (i32, [i64, P, P, P, P, P, i32, P, P]),
            "oracle_gather_hvp": (i32, [i64, P, P, P, P, P, i32, P, P, P, dbl, P]),
            "oracle_threads": (i32, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(code, what):
    if code != OK:
        raise OracleError(code, what)


class Params:
    """Run parameters of one P3M configuration (SI units)."""

    def __init__(self, grid, h, r_cut, split, order, ke_q2, m=1.0, dt=0.0, zoom=True, qw=None,
                 gather="variational", cathode_z=None, influence="sampled"):
        self.grid = np.asarray(grid, dtype=np.int32)
        self.h = np.asarray(h, dtype=np.float64)
        self.r_cut = float(r_cut)
        self.split = float(split)
        self.order = int(order)
        self.ke_q2 = float(ke_q2)
        self.m = float(m)
        self.dt = float(dt)
        self.zoom = bool(zoom)
        self.qw = None if qw is None else _f64(qw)
        if gather not in ("variational", "momentum"):
            raise ValueError(gather)
        self.gather = gather
        self.cathode_z = None if cathode_z is None else float(cathode_z)
        if influence not in ("sampled", "optimal", "principal", "lattice"):
            raise ValueError(influence)
        self.influence = influence

    @classmethod
    def from_workload(cls, wl, **kw):
        return cls(wl.grid, wl.h, wl.r_cut, wl.split, wl.order, wl.ke_q2, wl.m, wl.dt, **kw)


def threads():
    """OpenMP threads used by the C loops."""
    return int(lib().oracle_threads())


# ---- placement --------------------------------------------------------------

def placement(x, prm):
    """Mesh origin, zoom and zoomed spacing for positions x (reading of Sec. 2.4.2).
    The momentum-conserving gather keeps every stencil one node inside the mesh."""
    x = _f64(x)
    out = np.zeros(8)
    margin = 1 if prm.gather == "momentum" else 0
    _check(lib().oracle_placement(len(x), _p(x), _p(prm.grid), _p(prm.h), prm.order,
                                  int(prm.zoom), margin, _p(out)), "placement")
    s = out[3]
    return {"x0": out[0:3].copy(), "s": s, "hp": out[4:7].copy(),
            "rc": prm.r_cut * s, "a": prm.split / s}


# ---- short range (PP) ---------------------------------------------------------

def pp_brute(x, prm, rc, a):
    """O(N^2) erfc pair force inside rc (Sec. 1 eq. summation_short; Sec. 2.2)."""
    x = _f64(x)
    f = np.zeros_like(x)
    lib().oracle_pp_brute(len(x), _p(x), _p(prm.qw), rc, a, prm.ke_q2, _p(f))
    return f


def pp_cells(x, prm, rc, a):
    """Same pair force through linked cells (exact equivalent of pp_brute)."""
    x = _f64(x)
    f = np.zeros_like(x)
    _check(lib().oracle_pp_cells(len(x), _p(x), _p(prm.qw), rc, a, prm.ke_q2, _p(f)), "pp_cells")
    return f


def pp_sample(x, prm, rc, a, idx):
    x = _f64(x)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    f = np.zeros((len(idx), 3))
    _check(lib().oracle_pp_sample(len(x), _p(x), _p(prm.qw), rc, a, prm.ke_q2, len(idx),
                                  _p(idx), _p(f)), "pp_sample")
    return f


def pp_energy(x, prm, rc, a):
    x = _f64(x)
    return lib().oracle_pp_energy(len(x), _p(x), _p(prm.qw), rc, a, prm.ke_q2)


# ---- mesh (PM) --------------------------------------------------------------

def deposit(x, prm, pl):
    """Mesh charge Q[z, y, x] (Sec. 2.5 eq. eom_p3m_poiss_L; Sec. 2.4.2 B-splines)."""
    x = _f64(x)
    g = prm.grid
    Q = np.zeros((g[2], g[1], g[0]))
    _check(lib().oracle_deposit(len(x), _p(x), _p(prm.qw), _p(g), _p(pl["x0"]), _p(pl["hp"]),
                                prm.order, _p(Q)), "deposit")
    return Q


def green_padded(grid, hp, a):
    """erf(a r)/r sampled on the doubled mesh, offsets k in [-N, N-1] per axis
    (stored at k mod 2N), value 2a/sqrt(pi) at r = 0 (Sec. 2.2 charge screening
    with the free-space Green's function of Sec. 2.1, eq. free_gf)."""
    axes = []
    for d in range(3):
        n = int(grid[d])
        k = np.arange(2 * n)
        k = np.where(k < n, k, k - 2 * n)
        axes.append(k * hp[d])
    rz, ry, rx = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    r = np.sqrt(rx * rx + ry * ry + rz * rz)
    with np.errstate(invalid="ignore", divide="ignore"):
        g = erf(a * r) / r
    g[r == 0] = 2.0 * a / math.sqrt(math.pi)
    return g


def lattice_cell_weights(h, a, tol=1e-18):
    """Charge of the Gaussian screening cloud (density (a/sqrt(pi)) exp(-a^2 x^2)
    along one axis, the gamma of Sec. 2.2) inside each mesh cell of edge h
    centred on a node: g(m) = [erf(a (m + 1/2) h) - erf(a (m - 1/2) h)] / 2,
    m = 0, 1, ... until below tol (g is even in m), the tail through erfc.
    a = None: no screening, g = delta."""
    if a is None:
        return np.array([1.0])
    out = []
    m = 0
    while True:
        if m == 0:
            g = erf(0.5 * a * h)
        else:
            g = 0.5 * (erfc(a * (m - 0.5) * h) - erfc(a * (m + 0.5) * h))
        out.append(g)
        if m > 0 and g < tol:
            return np.array(out)
        m += 1


def _gauss_legendre_panels(lo, hi, width=1.0, q=16):
    x, w = np.polynomial.legendre.leggauss(q)
    n = int(math.ceil((hi - lo) / width))
    edges = np.linspace(lo, hi, n + 1)
    u = np.concatenate([0.5 * (b - a) * x + 0.5 * (a + b) for a, b in zip(edges[:-1], edges[1:])])
    wu = np.concatenate([0.5 * (b - a) * w for a, b in zip(edges[:-1], edges[1:])])
    return u, wu


def lattice_kernel(nmax, hp, a):
    """Mesh kernel of the lattice form on the octant 0 <= n_d <= nmax_d:
    K = 4 pi G_L (x) g, where G_L solves the 7-point discrete Poisson equation
    of the free (unbounded) lattice, -sum_d D_d G_L / h_d^2 = delta / (h_x h_y h_z)
    (D_d the second difference of Sec. 2.4.2 eq. 1d_ddiff, summed as in eq.
    3dim_second_order_fin_diff_tensor; the Green's function of Sec. 3 eq.
    def_G_L), and g = prod_d g_d the Gaussian screening integrated over cells
    (lattice_cell_weights). K -> 1/r far away, like the sampled erf(a r)/r.

    Evaluated through 1/L = int_0^inf exp(-t L) dt for the operator L: the
    heat kernel of the second difference along one axis is
    exp(-2 s) I_k(2 s) = ive(k, 2 s), s = t / h_d^2, so
      K(n) = (4 pi / V) int_0^inf prod_d F_d(n_d, t) dt,
      F_d(n, t) = sum_m g_d(m) ive(n - m, 2 t / h_d^2).
    The t integral is Gauss-Legendre over panels of ln t from 1e-14 h_min^2
    to T = 5e7 h_min^2 (scipy's ive is accurate there); beyond T the heat
    kernel is Gaussian to O(h^2 / T) and the rest is erf(r / (2 sqrt(T))) / r.
    Returned as K[z, y, x]."""
    hp = np.asarray(hp, dtype=np.float64)
    V = float(np.prod(hp))
    T = 5e7 * hp.min() ** 2
    u, wu = _gauss_legendre_panels(math.log(1e-14 * hp.min() ** 2), math.log(T))
    t = np.exp(u)
    F = []
    for d in range(3):
        g = lattice_cell_weights(hp[d], a)
        n = np.arange(int(nmax[d]) + 1)
        z = 2.0 * t / hp[d] ** 2
        Fd = np.zeros((len(n), len(t)))
        for m in range(-(len(g) - 1), len(g)):
            Fd += g[abs(m)] * ive(np.abs(n - m)[:, None], z[None, :])
        F.append(Fd)
    K = np.einsum("t,it,jt,kt->kji", wu * t, F[0], F[1], F[2]) * (4.0 * math.pi / V)
    ax = [np.arange(int(nmax[d]) + 1) * hp[d] for d in range(3)]
    rz, ry, rx = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    r = np.sqrt(rx * rx + ry * ry + rz * rz)
    with np.errstate(invalid="ignore", divide="ignore"):
        tail = np.where(r > 0, erf(r / (2.0 * math.sqrt(T))) / r, 1.0 / math.sqrt(math.pi * T))
    return K + tail


def green_padded_lattice(grid, hp, a):
    """The lattice kernel on the doubled mesh, laid out like green_padded."""
    K = lattice_kernel(grid, hp, a)
    idx = []
    for d in range(3):
        n = int(grid[d])
        k = np.arange(2 * n)
        idx.append(np.abs(np.where(k < n, k, k - 2 * n)))
    return K[np.ix_(idx[2], idx[1], idx[0])]


def bspline_ft(kh, order):
    """Fourier transform of the cardinal B-spline of the assignment along one
    axis at k h: sinc(k h / 2)^(p+1), sinc(x) = sin(x)/x (b1 CIC p = 1, b2 TSC p = 2)."""
    x = 0.5 * np.asarray(kh, dtype=np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        s = np.where(x == 0.0, 1.0, np.sin(x) / x)
    return s ** (order + 1)


def alias_sum_u2(kh, order, M):
    """sum_{m=-M..M} U^2(k h - 2 pi m) along one axis."""
    return sum(bspline_ft(kh - 2 * math.pi * m, order) ** 2 for m in range(-M, M + 1))


def influence_correction(grid, hp, a, order, mode, M=2):
    """Table correction of the optimal influence function (Sec. 3.1.2, eq.
    Ghfinal), on numpy's rfftn layout of the doubled mesh. For point particles,
    with the Gaussian screening folded into the reference kernel
    (R gamma)^(k) = 4 pi exp(-k^2/(4 a^2)) / k^2 and the assignment U = prod sinc^(p+1):
      optimal:   G = sum_m U^2(k_m) (R gamma)(k_m) / [sum_m U^2(k_m)]^2, |m_d| <= M;
      principal: the m = 0 term alone, (R gamma)(k) / U^2(k).
    Returned is (G - (R gamma)(k)) / (h_x h_y h_z): added to the transform of the
    sampled kernel it makes the mesh kernel the optimal one near the origin
    while leaving its long-range part, and with it the open boundary, as the
    exact sampled erf(a r)/r (the difference is finite at k = 0 and short-ranged).
    The k = 0 entry is the limit along k_x."""
    shp = [2 * int(grid[2]), 2 * int(grid[1]), int(grid[0]) + 1]
    kz = 2 * math.pi * np.fft.fftfreq(shp[0], d=hp[2])
    ky = 2 * math.pi * np.fft.fftfreq(shp[1], d=hp[1])
    kx = 2 * math.pi * np.fft.rfftfreq(2 * int(grid[0]), d=hp[0])
    KZ, KY, KX = np.meshgrid(kz, ky, kx, indexing="ij")
    KX = KX.copy()
    KX[0, 0, 0] = 1e-3 * math.pi / (int(grid[0]) * hp[0])     # limit k -> 0 along k_x
    ks = (KX, KY, KZ)

    def rg(kx_, ky_, kz_):
        k2 = kx_ * kx_ + ky_ * ky_ + kz_ * kz_
        return 4 * math.pi * np.exp(-k2 / (4 * a * a)) / k2

    if mode == "principal":
        u2 = np.ones_like(KX)
        for d in range(3):
            u2 = u2 * bspline_ft(ks[d] * hp[d], order) ** 2
        G = rg(KX, KY, KZ) / u2
    else:
        num = np.zeros_like(KX)
        for mz in range(-M, M + 1):
            for my in range(-M, M + 1):
                for mx in range(-M, M + 1):
                    q = [KX - 2 * math.pi * mx / hp[0], KY - 2 * math.pi * my / hp[1],
                         KZ - 2 * math.pi * mz / hp[2]]
                    u2 = np.ones_like(KX)
                    for d in range(3):
                        u2 = u2 * bspline_ft(q[d] * hp[d], order) ** 2
                    num += u2 * rg(*q)
        den = np.ones_like(KX)
        for d in range(3):
            den = den * alias_sum_u2(ks[d] * hp[d], order, M)
        G = num / den ** 2
    return (G - rg(KX, KY, KZ)) / (hp[0] * hp[1] * hp[2])


def conv_fft(Q, grid, hp, a, influence=None):
    """phi = G (x) Q, aperiodic, by zero padding to 2N and numpy's FFT
    (Sec. 3 eq. phi_L as a finite convolution; Hockney's doubling). With
    influence = (order, mode) the kernel carries the optimal-influence
    correction (Sec. 3.1.2), or, for mode "lattice", is the lattice kernel."""
    nz, ny, nx = Q.shape
    Qp = np.zeros((2 * nz, 2 * ny, 2 * nx))
    Qp[:nz, :ny, :nx] = Q
    if influence is not None and influence[1] == "lattice":
        Gk = np.fft.rfftn(green_padded_lattice(grid, hp, a))
        influence = None
    else:
        Gk = np.fft.rfftn(green_padded(grid, hp, a))
    if influence is not None:
        Gk = Gk + influence_correction(grid, hp, a, influence[0], influence[1])
    phi = np.fft.irfftn(np.fft.rfftn(Qp) * Gk, s=Qp.shape, axes=(0, 1, 2))
    return np.ascontiguousarray(phi[:nz, :ny, :nx])


def conv_direct(Q, grid, hp, a):
    """phi by the plain O(M^2) aperiodic sum (tiny meshes only)."""
    Q = _f64(Q)
    phi = np.zeros_like(Q)
    lib().oracle_conv_direct(_p(np.asarray(grid, np.int32)), _p(_f64(hp)), a, _p(Q), _p(phi))
    return phi


def image_shifted_kernel(grid, hp, a, x0, zc):
    """Kernel of the image term on the doubled mesh: with the charge reflected
    in z (node k -> N_z - 1 - k) the mirror images sit at z-offset
    delta_z h_z + D from the field nodes, D = (N_z - 1) h_z + 2 (z0 - zc), so the
    image potential is an aperiodic convolution with G shifted by D (the
    shifted Green's function of Sec. 3.1)."""
    D = (int(grid[2]) - 1) * hp[2] + 2.0 * (x0[2] - zc)
    axes = []
    for d in range(3):
        n = int(grid[d])
        k = np.arange(2 * n)
        k = np.where(k < n, k, k - 2 * n)
        axes.append(k * hp[d] + (D if d == 2 else 0.0))
    rz, ry, rx = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    r = np.sqrt(rx * rx + ry * ry + rz * rz)
    with np.errstate(invalid="ignore", divide="ignore"):
        g = erf(a * r) / r
    g[r == 0] = 2.0 * a / math.sqrt(math.pi)
    return g


def conv_fft_image(Q, grid, hp, a, x0, zc):
    """phi with a grounded plane z = zc: free-space convolution minus the image
    term, both by zero padding and numpy's FFT."""
    nz, ny, nx = Q.shape
    Qr = np.zeros((2 * nz, 2 * ny, 2 * nx))
    Qr[:nz, :ny, :nx] = Q[::-1, :, :]
    Gs = np.fft.rfftn(image_shifted_kernel(grid, hp, a, x0, zc))
    img = np.fft.irfftn(np.fft.rfftn(Qr) * Gs, s=Qr.shape, axes=(0, 1, 2))[:nz, :ny, :nx]
    return conv_fft(Q, grid, hp, a) - img


def conv_direct_image(Q, grid, x0, hp, a, zc):
    """phi with images by the plain O(M^2) sum (tiny meshes only)."""
    Q = _f64(Q)
    phi = np.zeros_like(Q)
    lib().oracle_conv_direct_image(_p(np.asarray(grid, np.int32)), _p(_f64(x0)), _p(_f64(hp)), a,
                                   float(zc), _p(Q), _p(phi))
    return phi


def phi_image_point(Q, grid, x0, hp, a, zc, y):
    """Potential of the mesh charge and its images at the point y."""
    return lib().oracle_phi_image_point(_p(np.asarray(grid, np.int32)), _p(_f64(x0)), _p(_f64(hp)), a,
                                        float(zc), _p(_f64(Q)), _p(_f64(y)))


def mesh_potential(Q, prm, pl, direct=False):
    """The long-range potential on the mesh: free space, or with the grounded
    plane when prm.cathode_z is set."""
    if prm.influence != "sampled":
        if direct or prm.cathode_z is not None:
            raise ValueError("the alternative mesh kernels are applied in the FFT route, free space")
        return conv_fft(Q, prm.grid, pl["hp"], pl["a"], influence=(prm.order, prm.influence))
    if prm.cathode_z is None:
        return (conv_direct if direct else conv_fft)(Q, prm.grid, pl["hp"], pl["a"])
    if direct:
        return conv_direct_image(Q, prm.grid, pl["x0"], pl["hp"], pl["a"], prm.cathode_z)
    return conv_fft_image(Q, prm.grid, pl["hp"], pl["a"], pl["x0"], prm.cathode_z)


def phi_at(Q, grid, hp, a, nodes):
    Q = _f64(Q)
    nodes = np.ascontiguousarray(nodes, dtype=np.int64)
    out = np.zeros(len(nodes))
    lib().oracle_phi_at(_p(np.asarray(grid, np.int32)), _p(_f64(hp)), a, _p(Q), len(nodes),
                        _p(nodes), _p(out))
    return out


def stencil_nodes(xi, prm, pl):
    nodes = np.zeros(27, dtype=np.int64)
    k = lib().oracle_stencil_nodes(_p(_f64(xi)), _p(prm.grid), _p(pl["x0"]), _p(pl["hp"]),
                                   prm.order, _p(nodes))
    return nodes[:k]


def gather(x, prm, pl, phi):
    """Mesh force at the particles from the mesh potential phi.
    variational: -k_e q^2 qw_i sum_m phi_m grad W_m(x_i) (Sec. 2.5 eq. eom_p3m_coord);
    momentum: k_e q^2 qw_i sum_m W_m(x_i) E_m with E the central difference of -phi."""
    x = _f64(x)
    phi = _f64(phi)
    f = np.zeros_like(x)
    fn = lib().oracle_gather_momentum if prm.gather == "momentum" else lib().oracle_gather
    _check(fn(len(x), _p(x), _p(prm.qw), _p(prm.grid), _p(pl["x0"]), _p(pl["hp"]), prm.order,
              _p(phi), prm.ke_q2, _p(f)), "gather")
    return f


# ---- whole force evaluation and step ----------------------------------------

def forces(x, prm, parts=False, brute=False, direct=False, pl=None):
    """Total P3M force F = F_PP + F_PM at positions x (Sec. 2.5 eq. eom_p3m_coord)."""
    if pl is None:
        pl = placement(x, prm)
    fpp = (pp_brute if brute else pp_cells)(x, prm, pl["rc"], pl["a"])
    Q = deposit(x, prm, pl)
    phi = mesh_potential(Q, prm, pl, direct=direct)
    fpm = gather(x, prm, pl, phi)
    if parts:
        return fpp + fpm, {"pp": fpp, "pm": fpm, "Q": Q, "phi": phi, "pl": pl}
    return fpp + fpm


def pp_image(x, prm, rc, a, zc):
    """Short-range force of the mirror images of a grounded plane z = zc
    (Sec. 3.1.1, the term eq. short_range_error measures): every particle j
    has an image of charge -q_j at S(x_j) = (x_j, y_j, 2 zc - z_j) (eq.
    symmetry_planar_cathode), and particle i feels the erfc pair force of
    every image closer than rc, its own image included:
      F_i = sum_j k_e q_i (-q_j) [erfc(a r)/r + (2a/sqrt(pi)) e^{-a^2 r^2}] (x_i - S(x_j)) / r^2,
    r = |x_i - S(x_j)| < rc. This is the part of the image interaction that the
    scheme of Sec. 3.1 (free-space pair sum, images on the mesh) leaves out.
    Plain O(N^2) sum."""
    x = _f64(x)
    n = len(x)
    qw = np.ones(n) if prm.qw is None else prm.qw
    img = x.copy()
    img[:, 2] = 2.0 * zc - x[:, 2]
    f = np.zeros_like(x)
    for i0 in range(0, n, 1024):
        xi = x[i0:i0 + 1024]
        d = xi[:, None, :] - img[None, :, :]
        r = np.sqrt((d * d).sum(-1))
        inside = r < rc
        rr = np.where(inside, r, 1.0)
        g = (erfc(a * rr) / rr + 2.0 * a / math.sqrt(math.pi) * np.exp(-(a * rr) ** 2)) / (rr * rr)
        g = np.where(inside, g, 0.0) * (-qw[None, :])
        f[i0:i0 + 1024] = prm.ke_q2 * qw[i0:i0 + 1024, None] * (g[:, :, None] * d).sum(1)
    return f


def coulomb_image_brute(x, ke_q2, zc, qw=None):
    """Unsplit Coulomb force with a grounded plane z = zc: every other particle
    directly, and every particle's image -q at S(x_j), own image included
    (the free-space Green's function minus its mirror, eq.
    GreenFunc_planar_cathode). Plain O(N^2) sum."""
    x = _f64(x)
    n = len(x)
    qw = np.ones(n) if qw is None else _f64(qw)
    img = x.copy()
    img[:, 2] = 2.0 * zc - x[:, 2]
    f = coulomb_brute(x, ke_q2, qw)
    for i0 in range(0, n, 1024):
        d = x[i0:i0 + 1024, None, :] - img[None, :, :]
        r2 = (d * d).sum(-1)
        f[i0:i0 + 1024] -= ke_q2 * qw[i0:i0 + 1024, None] * ((qw[None, :] / (r2 * np.sqrt(r2)))[:, :, None]
                                                           * d).sum(1)
    return f


def coulomb_brute(x, ke_q2, qw=None):
    """Unsplit O(N^2) Coulomb force, the physics the split approximates (Sec. 1)."""
    prm = Params((4, 4, 4), (1, 1, 1), np.inf, 0.0, 1, ke_q2, qw=qw)
    return pp_brute(x, prm, np.inf, 0.0)


def step(x, p, prm, nsteps, f=None):
    """Kick-drift-kick leapfrog (Sec. 2.4.3 eq. leapfrog; Sec. 2.5 eq. eom_p3m_coord):
    p += dt/2 F(x); x += dt p/m; p += dt/2 F(x)."""
    x = _f64(x).copy()
    p = _f64(p).copy()
    if f is None:
        f = forces(x, prm)
    dt, m = prm.dt, prm.m
    for _ in range(nsteps):
        p += 0.5 * dt * f
        x += dt * p / m
        f = forces(x, prm)
        p += 0.5 * dt * f
    return x, p, f


# ---- diagnostics ------------------------------------------------------------

C_LIGHT = 299792458.0


def emittance(x, p, m, axis):
    """Normalised rms emittance sqrt(<dx^2><dp^2> - <dx dp>^2)/(m c), centred."""
    dx = x[:, axis] - x[:, axis].mean()
    dp = p[:, axis] - p[:, axis].mean()
    val = (dx * dx).mean() * (dp * dp).mean() - (dx * dp).mean() ** 2
    return math.sqrt(max(val, 0.0)) / (m * C_LIGHT)


def diagnostics(x, p, prm, brute_pp=False):
    pl = placement(x, prm)
    Q = deposit(x, prm, pl)
    phi = mesh_potential(Q, prm, pl)
    if brute_pp:
        upp = pp_energy(x, prm, pl["rc"], pl["a"])
    else:
        upp = float("nan")
    qw = np.ones(len(x)) if prm.qw is None else prm.qw
    return {
        "momentum": p.sum(axis=0),
        "kinetic": float((p * p).sum() / (2 * prm.m)),
        "u_pp": upp,
        "u_pm": float(0.5 * prm.ke_q2 * (Q * phi).sum()),
        "mean": x.mean(axis=0),
        "rms": x.std(axis=0),
        "emit_x": emittance(x, p, prm.m, 0),
        "emit_y": emittance(x, p, prm.m, 1),
        "charge": float(qw.sum()),
    }


# ---- adjoint ----------------------------------------------------------------

def hvp(x, v, prm, pl, brute=True):
    """H v with H = dF/dx (symmetric, F = -grad U), placement frozen at pl.
    PP part: sum_j K_ij (v_i - v_j); PM part: gather of psi = G (x) R plus the
    second derivative of the weights against phi (derivatives of Sec. 2.5
    eq. eom_p3m_coord)."""
    if prm.gather != "variational":
        raise ValueError("the Hessian is that of the variational force")
    x = _f64(x)
    v = _f64(v)
    out_pp = np.zeros_like(x)
    lib().oracle_pp_hvp(len(x), _p(x), _p(prm.qw), pl["rc"], pl["a"], prm.ke_q2, _p(v), _p(out_pp))
    g = prm.grid
    Q = deposit(x, prm, pl)
    phi = mesh_potential(Q, prm, pl)
    R = np.zeros_like(Q)
    _check(lib().oracle_deposit_grad(len(x), _p(x), _p(prm.qw), _p(g), _p(pl["x0"]), _p(pl["hp"]),
                                     prm.order, _p(v), _p(R)), "deposit_grad")
    psi = mesh_potential(R, prm, pl)
    out_pm = np.zeros_like(x)
    _check(lib().oracle_gather_hvp(len(x), _p(x), _p(prm.qw), _p(g), _p(pl["x0"]), _p(pl["hp"]),
                                   prm.order, _p(phi), _p(psi), _p(v), prm.ke_q2, _p(out_pm)),
           "gather_hvp")
    return out_pp + out_pm


def rollout(x, p, prm, nsteps, record=True):
    """Forward KDK that also records every step's positions and placement."""
    xs, pls = [_f64(x).copy()], [placement(x, prm)]
    f = forces(xs[0], prm, pl=pls[0])
    x = xs[0].copy()
    p = _f64(p).copy()
    for _ in range(nsteps):
        p += 0.5 * prm.dt * f
        x += prm.dt * p / prm.m
        pl = placement(x, prm)
        f = forces(x, prm, pl=pl)
        p += 0.5 * prm.dt * f
        xs.append(x.copy())
        pls.append(pl)
    return x, p, xs, pls


def step_backward(x_n, x_np1, pl_n, pl_np1, xbar, pbar, prm):
    """Reverse of one KDK step (placements frozen at the recorded values):
    with H = dF/dx symmetric,
      pbar <- pbar_{n+1};  xbar <- xbar_{n+1} + dt/2 H(x_{n+1}) pbar;
      pbar <- pbar + dt/m xbar;  xbar_n <- xbar + dt/2 H(x_n) pbar."""
    dt, m = prm.dt, prm.m
    xb = xbar + 0.5 * dt * hvp(x_np1, pbar, prm, pl_np1)
    pb = pbar + dt / m * xb
    xb = xb + 0.5 * dt * hvp(x_n, pb, prm, pl_n)
    return xb, pb


def forward_frozen(x, p, prm, pls):
    """KDK with the placement of each evaluation taken from pls (for FD checks)."""
    x = _f64(x).copy()
    p = _f64(p).copy()
    f = forces(x, prm, pl=pls[0])
    for n in range(len(pls) - 1):
        p += 0.5 * prm.dt * f
        x += prm.dt * p / prm.m
        f = forces(x, prm, pl=pls[n + 1])
        p += 0.5 * prm.dt * f
    return x, p


def objective(x, p, prm):
    """J = (eps_x + eps_y)/2, the transverse normalised rms emittance."""
    return 0.5 * (emittance(x, p, prm.m, 0) + emittance(x, p, prm.m, 1))


def objective_grad(x, p, prm):
    """Closed-form dJ/dx, dJ/dp of the transverse emittance."""
    gx = np.zeros_like(x)
    gp = np.zeros_like(p)
    n = len(x)
    mc = prm.m * C_LIGHT
    for ax in (0, 1):
        dx = x[:, ax] - x[:, ax].mean()
        dp = p[:, ax] - p[:, ax].mean()
        sxx, spp, sxp = (dx * dx).mean(), (dp * dp).mean(), (dx * dp).mean()
        e2 = sxx * spp - sxp * sxp
        if e2 <= 0:
            continue
        eps = math.sqrt(e2)
        # d e2 / d x_i = 2 dx_i spp / n - 2 sxp dp_i / n  (centring terms sum to zero)
        gx[:, ax] += 0.5 * (2 * dx * spp / n - 2 * sxp * dp / n) / (2 * eps) / mc
        gp[:, ax] += 0.5 * (2 * dp * sxx / n - 2 * sxp * dx / n) / (2 * eps) / mc
    return gx, gp


def gradient(x0, p0, prm, nsteps):
    """dJ/d(x0, p0) through the reverse KDK, placements frozen as recorded."""
    xN, pN, xs, pls = rollout(x0, p0, prm, nsteps)
    xb, pb = objective_grad(xN, pN, prm)
    for n in range(nsteps - 1, -1, -1):
        xb, pb = step_backward(xs[n], xs[n + 1], pls[n], pls[n + 1], xb, pb, prm)
    return xb, pb, (xN, pN, pls)
