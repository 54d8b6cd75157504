"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each checks a closed form, an
invariant, a special case that reduces to a textbook result, brute force on a
tiny input, or an exact value from the B-spline definition.
"""
import math
import os

import numpy as np
import pytest
from scipy.optimize import brentq

from oracle import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_bunch(n, seed, scale=1.0, aniso=(1, 1, 1)):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, 3)) * scale * np.asarray(aniso, float)


def _prm(grid=(16, 16, 16), h=(0.25, 0.25, 0.25), rc=0.5, kappa=3.0, order=2, **kw):
    return O.Params(grid, h, rc, kappa / rc, order, kw.pop("ke_q2", 1.0), **kw)


# ---- split identity and PP kernel (Sec. 2.2, eq. ewald_split) -------------------------

def test_split_kernels_sum_to_coulomb():
    """erfc(a r)/r (PP energy) + erf(a r)/r (mesh kernel) = 1/r at every offset."""
    h = np.array([0.3, 0.5, 0.7])
    a = 2.3
    for off in [(1, 0, 0), (0, 2, 1), (3, 1, 2), (1, 1, 1), (4, 0, 3)]:
        r = math.sqrt(sum((o * hh) ** 2 for o, hh in zip(off, h)))
        x = np.array([[0.0, 0.0, 0.0], [off[0] * h[0], off[1] * h[1], off[2] * h[2]]])
        prm = O.Params((4, 4, 4), h, 10.0, a, 1, 1.0)
        u_pp = O.pp_energy(x, prm, 10.0, a)
        g = O.lib().oracle_green(off[0], off[1], off[2], h.ctypes.data, a)
        assert abs(u_pp + g - 1.0 / r) < 1e-14 / r


def test_mesh_kernel_limit_at_origin():
    """erf(a r)/r -> 2a/sqrt(pi) as r -> 0 (Taylor series of erf)."""
    a = 1.7
    h = np.array([1e-7, 1e-7, 1e-7])
    g0 = O.lib().oracle_green(0, 0, 0, h.ctypes.data, a)
    g1 = O.lib().oracle_green(1, 0, 0, h.ctypes.data, a)
    assert g0 == pytest.approx(2 * a / math.sqrt(math.pi), rel=1e-15)
    assert g1 == pytest.approx(g0, rel=1e-12)


def test_alpha_zero_pp_is_coulomb_two_particles():
    """a = 0: the PP force is Coulomb's k q1 q2 / r^2 along the separation."""
    x = np.array([[0.1, -0.2, 0.3], [0.4, 0.2, -0.1]])
    qw = np.array([1.5, -0.5])
    prm = O.Params((4, 4, 4), (1, 1, 1), 10.0, 0.0, 1, 2.0, qw=qw)
    f = O.pp_brute(x, prm, 10.0, 0.0)
    d = x[0] - x[1]
    r = np.linalg.norm(d)
    expect = 2.0 * 1.5 * -0.5 / r ** 2 * d / r
    np.testing.assert_allclose(f[0], expect, rtol=1e-14)
    np.testing.assert_allclose(f[1], -expect, rtol=1e-14)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_pp_cells_equal_brute(seed):
    """Linked cells find exactly the pairs of the O(N^2) sum (strict r < r_c)."""
    rng = np.random.default_rng(seed)
    x = _rand_bunch(700, seed, aniso=(1, 0.5, 3))
    x[5] = x[6]                      # coincident pair contributes nothing
    d = rng.standard_normal(3)
    x[11] = x[10] + 0.4 * d / np.linalg.norm(d)   # a pair near the cutoff
    qw = rng.random(len(x)) + 0.5
    prm = O.Params((8, 8, 8), (1, 1, 1), 0.4, 3.0 / 0.4, 1, 1.0, qw=qw)
    fb = O.pp_brute(x, prm, 0.4, 7.5)
    fc = O.pp_cells(x, prm, 0.4, 7.5)
    scale = np.abs(fb).max()
    assert np.abs(fb - fc).max() <= 1e-13 * scale


def test_pp_newton_third_law():
    x = _rand_bunch(2000, 3)
    prm = _prm(rc=0.3)
    f = O.pp_cells(x, prm, 0.3, 10.0)
    assert np.abs(f.sum(axis=0)).max() <= 1e-13 * np.abs(f).sum()


def test_pp_force_is_minus_energy_gradient():
    """Central differences of the erfc pair energy give the PP force."""
    x = _rand_bunch(60, 4, scale=0.3)
    rc, a = 0.6, 3.0 / 0.6
    prm = _prm(rc=rc)
    f = O.pp_brute(x, prm, rc, a)
    eps = 1e-6
    for i, d in [(0, 0), (7, 1), (33, 2), (59, 0)]:
        xp, xm = x.copy(), x.copy()
        xp[i, d] += eps
        xm[i, d] -= eps
        fd = -(O.pp_energy(xp, prm, rc, a) - O.pp_energy(xm, prm, rc, a)) / (2 * eps)
        assert fd == pytest.approx(f[i, d], rel=2e-6, abs=1e-6 * np.abs(f).max())


# ---- assignment (Sec. 2.4.2, eq. interpolation_splines_b0) ----------------------------

def _golden_weights():
    rows = []
    with open(os.path.join(GOLDEN, "bspline_weights.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                rows.append([float(t) for t in line.split()])
    return rows


def test_bspline_weights_golden():
    """One particle at fractional node offsets deposits the exact B-spline weights."""
    for order, frac, w0, w1, w2 in _golden_weights():
        order = int(order)
        grid = (8, 8, 8)
        prm = O.Params(grid, (1, 1, 1), 1.0, 1.0, order, 1.0, zoom=False)
        pl = {"x0": np.zeros(3), "hp": np.ones(3)}
        u = 3.0 + frac
        x = np.array([[u, 3.0, 3.0]])
        Q = O.deposit(x, prm, pl)
        line = Q.sum(axis=(0, 1))
        if order == 1:
            base = int(math.floor(u))
            got = [line[base], line[base + 1], 0.0]
        else:
            c = int(math.floor(u + 0.5))
            got = [line[c - 1], line[c], line[c + 1]]
        np.testing.assert_allclose(got, [w0, w1, w2], atol=1e-15)
        # the transverse axes sit on a node
        prof = Q.sum(axis=(0, 2))
        expect = [1.0] if order == 1 else [0.125, 0.75, 0.125]
        lo = 3 if order == 1 else 2
        np.testing.assert_allclose(prof[lo:lo + len(expect)], expect, atol=1e-15)


@pytest.mark.parametrize("order", [1, 2])
def test_deposit_conserves_charge_and_dipole(order):
    """sum Q = sum q and sum x_m Q_m = sum q_i xi_i (B-splines reproduce linears)."""
    x = _rand_bunch(3000, 5, aniso=(1, 2, 0.5))
    rng = np.random.default_rng(9)
    qw = rng.random(len(x)) + 0.1
    prm = O.Params((20, 24, 12), (0.4, 0.7, 0.3), 0.8, 3.0, order, 1.0, qw=qw)
    pl = O.placement(x, prm)
    Q = O.deposit(x, prm, pl)
    assert Q.sum() == pytest.approx(qw.sum(), rel=1e-13)
    nz, ny, nx = Q.shape
    gz, gy, gx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    for d, g in enumerate((gx, gy, gz)):
        xm = pl["x0"][d] + g * pl["hp"][d]
        assert (xm * Q).sum() == pytest.approx((qw * x[:, d]).sum(), rel=1e-12, abs=1e-12)


# ---- convolution (Sec. 3, eq. phi_L; Hockney doubling) --------------------------------

@pytest.mark.parametrize("grid", [(2, 2, 2), (3, 4, 5), (6, 6, 6), (5, 2, 3)])
def test_fft_convolution_equals_direct(grid):
    rng = np.random.default_rng(sum(grid))
    Q = rng.standard_normal((grid[2], grid[1], grid[0]))
    hp = np.array([0.5, 0.3, 0.9])
    a = 1.3
    np.testing.assert_allclose(O.conv_fft(Q, grid, hp, a), O.conv_direct(Q, grid, hp, a),
                               rtol=1e-12, atol=1e-12 * np.abs(Q).sum())


def test_single_charge_gives_kernel():
    """A unit charge on node m0 gives phi(m) = G(m - m0), with no wrap-around."""
    grid = (8, 6, 7)
    hp = np.array([0.2, 0.35, 0.5])
    a = 2.0
    Q = np.zeros((7, 6, 8))
    Q[6, 0, 7] = 1.0                 # a corner: offsets reach N-1 in every axis
    phi = O.conv_fft(Q, grid, hp, a)
    for (z, y, x) in [(0, 5, 0), (6, 0, 7), (3, 2, 1), (0, 0, 0)]:
        g = O.lib().oracle_green(x - 7, y - 0, z - 6, hp.ctypes.data, a)
        assert phi[z, y, x] == pytest.approx(g, rel=1e-12)


# ---- gather (Sec. 2.5, eq. eom_p3m_coord first term) ----------------------------------

@pytest.mark.parametrize("order", [1, 2])
def test_gather_linear_potential_exact_gradient(order):
    """For phi linear in the node position the weight gradient returns it exactly."""
    grid = (10, 12, 9)
    x = _rand_bunch(200, 6, scale=0.3)
    qw = np.random.default_rng(1).random(len(x)) + 0.5
    prm = O.Params(grid, (0.3, 0.25, 0.4), 0.5, 1.0, order, 2.0, qw=qw)
    pl = O.placement(x, prm)
    c = np.array([1.5, -0.7, 0.4])
    nz, ny, nx = grid[2], grid[1], grid[0]
    gz, gy, gx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    phi = 3.0 + c[0] * (pl["x0"][0] + gx * pl["hp"][0]) + c[1] * (pl["x0"][1] + gy * pl["hp"][1]) \
        + c[2] * (pl["x0"][2] + gz * pl["hp"][2])
    f = O.gather(x, prm, pl, phi)
    np.testing.assert_allclose(f, -2.0 * qw[:, None] * c[None, :], rtol=1e-11)


@pytest.mark.parametrize("order", [1, 2])
def test_pm_force_is_minus_energy_gradient(order):
    """F_PM = -dU_PM/dxi with U_PM = k q^2 sum_m Q_m phi_m / 2 (placement frozen)."""
    x = _rand_bunch(40, 7, scale=0.5)
    prm = O.Params((12, 12, 12), (0.4, 0.4, 0.4), 0.8, 3.0 / 0.8, order, 1.0)
    pl = O.placement(x, prm)
    pl["x0"] = pl["x0"] - 0.013        # keep every particle well away from a knot
    F, parts = O.forces(x, prm, parts=True, pl=pl)

    def upm(xx):
        Q = O.deposit(xx, prm, pl)
        return 0.5 * (Q * O.conv_fft(Q, prm.grid, pl["hp"], pl["a"])).sum()

    eps = 1e-7
    for i, d in [(0, 0), (3, 1), (17, 2), (39, 1)]:
        u = (x[i, d] - pl["x0"][d]) / pl["hp"][d]
        knot = u - math.floor(u) if order == 1 else u + 0.5 - math.floor(u + 0.5)
        if min(knot, 1 - knot) < 1e-3:
            continue
        xp, xm = x.copy(), x.copy()
        xp[i, d] += eps
        xm[i, d] -= eps
        fd = -(upm(xp) - upm(xm)) / (2 * eps)
        assert fd == pytest.approx(parts["pm"][i, d], rel=1e-5, abs=1e-6 * np.abs(parts["pm"]).max())


def test_pm_two_particles_far_limit():
    """TSC, smooth kernel (a h = 0.25): at 8h the mesh force approaches the
    closed-form force of the erf(a r)/r pair potential."""
    from scipy.special import erf
    rng = np.random.default_rng(11)
    h, a = 1.0, 0.25
    errs = []
    for _ in range(10):
        c = rng.random(3)
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        x = np.array([c, c + 8 * h * d])
        prm = O.Params((32, 32, 32), (h, h, h), 1e-9, a, 2, 1.0)
        pl = O.placement(x, prm)
        Q = O.deposit(x, prm, pl)
        f = O.gather(x, prm, pl, O.conv_fft(Q, prm.grid, pl["hp"], pl["a"]))
        r = 8.0 * h
        g = (erf(a * r) / r - 2 * a / math.sqrt(math.pi) * math.exp(-(a * r) ** 2)) / r ** 2
        exact = g * (x[0] - x[1])
        errs.append(np.linalg.norm(f[0] - exact) / np.linalg.norm(exact))
    assert max(errs) < 0.03


# ---- momentum-conserving gather (mesh E by central differences) -------------------

def _pm_momentum(x, prm):
    pl = O.placement(x, prm)
    Q = O.deposit(x, prm, pl)
    phi = O.conv_fft(Q, prm.grid, pl["hp"], pl["a"])
    return O.gather(x, prm, pl, phi), pl


@pytest.mark.parametrize("order", [1, 2])
def test_momentum_gather_total_force_vanishes(order):
    """With E = -D phi, D the antisymmetric central difference, and phi = G (x) Q
    for a symmetric G, sum_i F_i = sum_m Q_m E_m = 0 (the variational force has
    no such property, which the second assertion confirms on the same bunch)."""
    x = _rand_bunch(300, 21, scale=0.6, aniso=(1, 1, 2))
    qw = np.random.default_rng(22).random(len(x)) + 0.5
    prm = O.Params((14, 12, 16), (0.3, 0.35, 0.4), 0.6, 3.0 / 0.6, order, 1.0, qw=qw, gather="momentum")
    f, _ = _pm_momentum(x, prm)
    scale = np.abs(f).sum(axis=0)
    assert np.all(np.abs(f.sum(axis=0)) <= 1e-13 * scale)
    prm_v = O.Params((14, 12, 16), (0.3, 0.35, 0.4), 0.6, 3.0 / 0.6, order, 1.0, qw=qw)
    fv, _ = _pm_momentum(x, prm_v)
    assert np.abs(fv.sum(axis=0)).max() > 1e-8 * np.abs(fv).sum(axis=0).max()


@pytest.mark.parametrize("order", [1, 2])
def test_momentum_gather_no_self_force(order):
    """A lone particle feels no mesh force from its own charge (the single-particle
    case of the vanishing total), wherever it sits between nodes."""
    rng = np.random.default_rng(23)
    for _ in range(8):
        x = rng.random((1, 3)) * 0.3
        x2 = np.vstack([x, x + 0.9])       # a second particle sets the placement scale only
        prm = O.Params((12, 12, 12), (0.25, 0.25, 0.25), 0.5, 3.0 / 0.5, order, 1.0, gather="momentum")
        pl = O.placement(x2, prm)
        Q = O.deposit(x, prm, pl)
        phi = O.conv_fft(Q, prm.grid, pl["hp"], pl["a"])
        f = O.gather(x, prm, pl, phi)
        prm_v = O.Params((12, 12, 12), (0.25, 0.25, 0.25), 0.5, 3.0 / 0.5, order, 1.0)
        fv = O.gather(x, prm_v, pl, phi)
        ref = max(np.abs(fv).max(), np.abs(phi).max() / pl["hp"][0])
        assert np.abs(f).max() <= 1e-13 * ref


@pytest.mark.parametrize("order", [1, 2])
def test_momentum_gather_linear_potential(order):
    """Central differences of a linear potential are exact and the weights sum
    to one: F = -k q^2 qw grad(phi) exactly."""
    grid = (10, 12, 9)
    x = _rand_bunch(200, 24, scale=0.3)
    qw = np.random.default_rng(25).random(len(x)) + 0.5
    prm = O.Params(grid, (0.3, 0.25, 0.4), 0.5, 1.0, order, 2.0, qw=qw, gather="momentum")
    pl = O.placement(x, prm)
    c = np.array([1.5, -0.7, 0.4])
    nz, ny, nx = grid[2], grid[1], grid[0]
    gz, gy, gx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    phi = 3.0 + c[0] * (pl["x0"][0] + gx * pl["hp"][0]) + c[1] * (pl["x0"][1] + gy * pl["hp"][1]) \
        + c[2] * (pl["x0"][2] + gz * pl["hp"][2])
    f = O.gather(x, prm, pl, phi)
    np.testing.assert_allclose(f, -2.0 * qw[:, None] * c[None, :], rtol=1e-11)


def test_momentum_placement_keeps_stencils_off_the_edge():
    """The momentum form needs phi one node beyond every stencil node: the zoom
    leaves the outer node layer free."""
    x = _rand_bunch(400, 26, scale=5.0)
    for order in (1, 2):
        prm = O.Params((16, 16, 16), (0.2, 0.2, 0.2), 0.4, 7.5, order, 1.0, gather="momentum")
        pl = O.placement(x, prm)
        nodes = np.concatenate([O.stencil_nodes(xi, prm, pl) for xi in x])
        nz = nodes // 256
        ny = (nodes // 16) % 16
        nx = nodes % 16
        for v in (nx, ny, nz):
            assert v.min() >= 1 and v.max() <= 14


def test_momentum_two_particles_far_limit():
    """Far apart (8h, a h = 0.25) the momentum-conserving mesh force also
    approaches the closed-form erf(a r)/r pair force, and the pair is exactly
    action-reaction."""
    from scipy.special import erf
    rng = np.random.default_rng(27)
    h, a = 1.0, 0.25
    errs = []
    for _ in range(10):
        c = rng.random(3)
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        x = np.array([c, c + 8 * h * d])
        prm = O.Params((32, 32, 32), (h, h, h), 1e-9, a, 2, 1.0, gather="momentum")
        f, _ = _pm_momentum(x, prm)
        assert np.abs(f[0] + f[1]).max() <= 1e-13 * np.abs(f).max()
        r = 8.0 * h
        g = (erf(a * r) / r - 2 * a / math.sqrt(math.pi) * math.exp(-(a * r) ** 2)) / r ** 2
        exact = g * (x[0] - x[1])
        errs.append(np.linalg.norm(f[0] - exact) / np.linalg.norm(exact))
    assert max(errs) < 0.03


# ---- grounded planar cathode (image charges, shifted Green's function) -------------

@pytest.mark.parametrize("grid,zc_off", [((4, 5, 6), -3.7), ((6, 6, 6), -0.45), ((5, 3, 4), 1.6)])
def test_image_fft_route_equals_direct_sum(grid, zc_off):
    """Reflected charge convolved with the shifted kernel (the FFT route) equals
    the plain sum over every node charge and its mirror image, for a plane
    below the mesh, just below it, and through it."""
    rng = np.random.default_rng(31)
    Q = rng.standard_normal(grid[::-1])
    hp = np.array([0.3, 0.45, 0.25])
    x0 = np.array([0.1, -0.2, 0.7])
    zc = x0[2] + zc_off * hp[2]
    a = 1.3
    f = O.conv_fft_image(Q, grid, hp, a, x0, zc)
    d = O.conv_direct_image(Q, grid, x0, hp, a, zc)
    assert np.abs(f - d).max() <= 1e-12 * np.abs(d).max()


def test_image_potential_vanishes_on_the_plane():
    """Every point of the grounded plane is equidistant from a charge and its
    image: the potential is zero there (direct sum at arbitrary points, and the
    FFT route at mesh nodes lying on the plane)."""
    rng = np.random.default_rng(32)
    grid = (6, 5, 7)
    Q = rng.random(grid[::-1])
    Q[:3] = 0.0                         # charges only above the plane
    hp = np.array([0.3, 0.3, 0.2])
    x0 = np.array([0.0, 0.0, 0.0])
    zc = x0[2] + 2 * hp[2]              # the plane through node layer z = 2
    a = 2.0
    scale = np.abs(Q).sum() * 2 * a / math.sqrt(math.pi)
    for _ in range(10):
        y = np.array([rng.random() * 2, rng.random() * 2, zc])
        assert abs(O.phi_image_point(Q, grid, x0, hp, a, zc, y)) <= 1e-14 * scale
    phi = O.conv_fft_image(Q, grid, hp, a, x0, zc)
    assert np.abs(phi[2]).max() <= 1e-13 * scale


def test_image_force_on_a_lone_charge():
    """A charge at height d attracts to the plane like its mirror image -q at
    distance 2d: with a smooth kernel (a h = 0.25) and 2d = 8h the mesh force
    with the plane, less the same mesh force without it, matches the
    closed-form erf(a r)/r pair force at r = 2d."""
    from scipy.special import erf
    rng = np.random.default_rng(33)
    h, a = 1.0, 0.25
    errs = []
    for _ in range(6):
        x = np.array([rng.random(3) * 0.7 + 8.0])
        zc = x[0, 2] - 4.0 * h
        kw = dict(grid=(24, 24, 24), h=(h, h, h), r_cut=1e-9, split=a, order=2, ke_q2=1.0)
        prm_i = O.Params(kw["grid"], kw["h"], kw["r_cut"], a, 2, 1.0, cathode_z=zc)
        prm_f = O.Params(kw["grid"], kw["h"], kw["r_cut"], a, 2, 1.0)
        x2 = np.vstack([x, x + 3.0 + rng.random(3)])   # a second particle only moves the mesh
        pl = O.placement(x2, prm_f)
        Q = O.deposit(x, prm_f, pl)
        f_i = O.gather(x, prm_i, pl, O.mesh_potential(Q, prm_i, pl))
        f_f = O.gather(x, prm_f, pl, O.mesh_potential(Q, prm_f, pl))
        r = 2 * (x[0, 2] - zc)
        g = erf(a * r) / r ** 2 - 2 * a / math.sqrt(math.pi) * math.exp(-(a * r) ** 2) / r
        exact = np.array([0.0, 0.0, -g])       # toward the plane
        errs.append(np.linalg.norm((f_i - f_f)[0] - exact) / g)
    assert max(errs) < 0.03


@pytest.mark.parametrize("order", [1, 2])
def test_image_pm_force_is_minus_energy_gradient(order):
    """With the plane the mesh energy is still a symmetric quadratic form of the
    node charges (|x - S(y)| = |y - S(x)|), so F_PM = -dU_PM/dxi."""
    x = _rand_bunch(40, 34, scale=0.5)
    zc = x[:, 2].min() - 0.9
    prm = O.Params((12, 12, 12), (0.4, 0.4, 0.4), 0.8, 3.0 / 0.8, order, 1.0, cathode_z=zc)
    pl = O.placement(x, prm)
    pl["x0"] = pl["x0"] - 0.013
    F, parts = O.forces(x, prm, parts=True, pl=pl)

    def upm(xx):
        Q = O.deposit(xx, prm, pl)
        return 0.5 * (Q * O.mesh_potential(Q, prm, pl)).sum()

    eps = 1e-7
    for i, d in [(0, 0), (3, 1), (17, 2), (39, 2)]:
        u = (x[i, d] - pl["x0"][d]) / pl["hp"][d]
        knot = u - math.floor(u) if order == 1 else u + 0.5 - math.floor(u + 0.5)
        if min(knot, 1 - knot) < 1e-3:
            continue
        xp, xm = x.copy(), x.copy()
        xp[i, d] += eps
        xm[i, d] -= eps
        fd = -(upm(xp) - upm(xm)) / (2 * eps)
        assert fd == pytest.approx(parts["pm"][i, d], rel=1e-5, abs=1e-6 * np.abs(parts["pm"]).max())


# ---- optimal influence function (Sec. 3.1.2, eq. Ghfinal) --------------------------

@pytest.mark.parametrize("order", [1, 2])
def test_bspline_alias_sums_closed_form(order):
    """sum_m sinc^4(x + pi m) = 1 - (2/3) sin^2 x and sum_m sinc^6(x + pi m) =
    1 - sin^2 x + (2/15) sin^4 x (x = k h / 2): the aliasing sums of the CIC and
    TSC assignment functions in closed form."""
    kh = np.linspace(-math.pi, math.pi, 37)
    s2 = np.sin(0.5 * kh) ** 2
    closed = 1 - (2.0 / 3.0) * s2 if order == 1 else 1 - s2 + (2.0 / 15.0) * s2 ** 2
    np.testing.assert_allclose(O.alias_sum_u2(kh, order, 400), closed, rtol=1e-9)
    np.testing.assert_allclose(O.alias_sum_u2(kh, order, 2), closed, rtol=3e-3)


def _lr_potential_error(order, mode):
    """rms error of the mesh's long-range potential at the particles against
    the exact sum of erf(a r)/r over all particles (self term 2a/sqrt(pi)),
    the quantity the optimal influence function minimises."""
    from scipy.special import erf
    x = _rand_bunch(600, 35)
    prm = O.Params((24, 24, 24), (0.35, 0.35, 0.35), 0.7, 3.0 / 0.7, order, 1.0, influence=mode)
    pl = O.placement(x, prm)
    Q = O.deposit(x, prm, pl)
    phi = O.mesh_potential(Q, prm, pl).ravel()
    est = np.array([(O.deposit(x[i:i + 1], prm, pl).ravel() * phi).sum() for i in range(len(x))])
    a = pl["a"]
    d = np.sqrt(((x[:, None, :] - x[None, :, :]) ** 2).sum(-1))
    with np.errstate(divide="ignore", invalid="ignore"):
        G = erf(a * d) / d
    G[d == 0] = 2 * a / math.sqrt(math.pi)
    ref = G.sum(1)
    return math.sqrt(((est - ref) ** 2).mean() / (ref ** 2).mean())


@pytest.mark.parametrize("order", [1, 2])
def test_optimal_influence_lowers_the_potential_error(order):
    e_s = _lr_potential_error(order, "sampled")
    e_o = _lr_potential_error(order, "optimal")
    e_p = _lr_potential_error(order, "principal")
    assert e_o < 0.5 * e_s and e_p < 0.7 * e_s


def test_optimal_influence_lowers_tsc_force_error_vs_coulomb():
    """Total P3M force against the unsplit O(N^2) Coulomb sum, TSC at r_c = 2h:
    the optimal table lowers the rms error well below the sampled kernel's."""
    x = _rand_bunch(2000, 36)
    e = {}
    for mode in ("sampled", "optimal"):
        prm = O.Params((32, 32, 32), (8 / 30,) * 3, 16 / 30, 3.0 / (16 / 30), 2, 1.0, influence=mode)
        f = O.forces(x, prm)
        fc = O.coulomb_brute(x, 1.0)
        e[mode] = math.sqrt(((f - fc) ** 2).sum() / (fc ** 2).sum())
    assert e["optimal"] < 0.6 * e["sampled"]


def test_optimal_influence_correction_is_short_ranged():
    """The table correction, taken back to real space on the doubled mesh, is
    concentrated near the origin: off the axes it is below 1e-6 of its peak at
    half the mesh, along the axes (where the separable sinc^(p+1) of the
    assignment leaves slower tails) below 1e-3. The mesh kernel keeps the
    erf(a r)/r tail and the zero-padded open boundary."""
    grid = (32, 32, 32)
    hp = np.array([0.25, 0.25, 0.25])
    a = 3.0 / 0.5
    for order in (1, 2):
        C = O.influence_correction(grid, hp, a, order, "optimal")
        D = np.fft.irfftn(C, s=(64, 64, 64), axes=(0, 1, 2))
        d0 = abs(D[0, 0, 0])
        for off in [(16, 0, 0), (0, 16, 0), (0, 0, 31)]:
            assert abs(D[off[2], off[1], off[0]]) < 1e-3 * d0
        for off in [(12, 12, 12), (16, 16, 0), (31, 31, 31)]:
            assert abs(D[off[2], off[1], off[0]]) < 1e-6 * d0


def test_optimal_influence_force_is_minus_energy_gradient():
    """The corrected table is still real and even: the mesh energy stays a
    symmetric quadratic form and F_PM = -dU_PM/dxi."""
    x = _rand_bunch(40, 37, scale=0.5)
    prm = O.Params((12, 12, 12), (0.4, 0.4, 0.4), 0.8, 3.0 / 0.8, 2, 1.0, influence="optimal")
    pl = O.placement(x, prm)
    pl["x0"] = pl["x0"] - 0.013
    F, parts = O.forces(x, prm, parts=True, pl=pl)

    def upm(xx):
        Q = O.deposit(xx, prm, pl)
        return 0.5 * (Q * O.mesh_potential(Q, prm, pl)).sum()

    eps = 1e-7
    for i, d in [(0, 0), (3, 1), (17, 2), (39, 1)]:
        u = (x[i, d] - pl["x0"][d]) / pl["hp"][d]
        knot = u + 0.5 - math.floor(u + 0.5)
        if min(knot, 1 - knot) < 1e-3:
            continue
        xp, xm = x.copy(), x.copy()
        xp[i, d] += eps
        xm[i, d] -= eps
        fd = -(upm(xp) - upm(xm)) / (2 * eps)
        assert fd == pytest.approx(parts["pm"][i, d], rel=1e-5, abs=1e-6 * np.abs(parts["pm"]).max())


# ---- lattice Green's function of the discrete Laplacian (Sec. 2.4.2, Sec. 3) -----------

def _watson_sc():
    """Watson's simple-cubic integral (1/pi^3) int_[0,pi]^3 dx dy dz / (1 - (cos x +
    cos y + cos z)/3) in the closed form of Glasser and Zucker (1977):
    sqrt(6)/(32 pi^3) Gamma(1/24) Gamma(5/24) Gamma(7/24) Gamma(11/24)."""
    from scipy.special import gamma
    return (math.sqrt(6) / (32 * math.pi ** 3) * gamma(1 / 24) * gamma(5 / 24) * gamma(7 / 24)
            * gamma(11 / 24))


def test_lattice_green_origin_is_watsons_integral():
    """Unscreened, cubic spacing h: the 7-point Green's function at the origin is
    (1/h) int d^3theta/(2 pi)^3 / (6 - 2 sum cos) = W / (6 h), so K(0) = 4 pi W / (6 h);
    its neighbour follows from the lattice equation at the origin, K(e) = K(0) - 4 pi / (6 h)."""
    W = _watson_sc()
    assert W == pytest.approx(1.516386059151978, rel=1e-14)
    for h in (1.0, 0.37):
        K = O.lattice_kernel((3, 3, 3), (h, h, h), None)
        assert K[0, 0, 0] == pytest.approx(4 * math.pi * W / (6 * h), rel=1e-12)
        assert K[0, 0, 1] == pytest.approx(K[0, 0, 0] - 4 * math.pi / (6 * h), rel=1e-12)
        assert K[1, 0, 0] == pytest.approx(K[0, 0, 1], rel=1e-13)
        assert K[0, 1, 0] == pytest.approx(K[0, 0, 1], rel=1e-13)


def test_lattice_cell_weights_are_the_screening_charge_per_cell():
    """The Gaussian cloud's charge per cell: positive, decreasing, summing to 1
    over the whole axis; a -> infinity leaves the unit charge on its node."""
    for h, a in [(0.5, 1.9), (1.3, 1.9), (0.25, 6.0), (1.0, 0.3)]:
        g = O.lattice_cell_weights(h, a)
        assert g[0] + 2 * g[1:].sum() == pytest.approx(1.0, abs=1e-15)
        assert np.all(g > 0) and np.all(np.diff(g) < 0)
    g = O.lattice_cell_weights(1.0, 40.0)
    assert g[0] == pytest.approx(1.0, abs=1e-15)


@pytest.mark.parametrize("h,a", [((0.5, 0.7, 1.3), 1.9), ((0.4, 0.4, 0.4), None), ((0.25, 0.25, 0.75), 6.0)])
def test_lattice_kernel_solves_the_discrete_poisson_equation(h, a):
    """Minus the 7-point Laplacian with spacings h_d (second differences D_d / h_d^2
    of Sec. 2.4.2, eq. 1d_ddiff) of K is the screening charge per cell over the
    cell volume times 4 pi: prod_d g_d(n_d), g_d(m) = [erf(a (m+1/2) h_d) -
    erf(a (m-1/2) h_d)]/2, or the unit charge at the origin unscreened."""
    from scipy.special import erf
    nm = (10, 9, 8)
    K = O.lattice_kernel(nm, h, a)
    V = float(np.prod(h))

    def k(i, j, l):
        return K[abs(l), abs(j), abs(i)]

    def gd(m, hd):
        if a is None:
            return 1.0 if m == 0 else 0.0
        return 0.5 * (erf(a * (m + 0.5) * hd) - erf(a * (m - 0.5) * hd))

    scale = 4 * math.pi / V
    for n in [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 3, 1), (1, 1, 1), (5, 5, 5),
              (9, 1, 3), (0, 8, 0), (3, 0, 7)]:
        lap = 0.0
        for d in range(3):
            e = [0, 0, 0]
            e[d] = 1
            lap -= (k(n[0] + e[0], n[1] + e[1], n[2] + e[2]) + k(n[0] - e[0], n[1] - e[1], n[2] - e[2])
                    - 2 * k(*n)) / h[d] ** 2
        rhs = scale * gd(n[0], h[0]) * gd(n[1], h[1]) * gd(n[2], h[2])
        assert lap == pytest.approx(rhs, abs=1e-11 * scale)


def test_lattice_green_far_field_asymptote():
    """Unscreened cubic lattice: r K(n) = 1 + (h^2 / (8 r^2)) (5 sum_d x_d^4 / r^4 - 3)
    + O(h^4 / r^4), the leading anisotropic correction of the simple-cubic
    lattice Green's function to the Coulomb potential."""
    K = O.lattice_kernel((12, 12, 12), (1.0, 1.0, 1.0), None)
    for n in [(12, 0, 0), (12, 12, 12), (6, 9, 12), (3, 0, 12), (8, 8, 0), (10, 4, 2)]:
        r2 = float(sum(v * v for v in n))
        r = math.sqrt(r2)
        pred = (5 * sum(v ** 4 for v in n) / r2 ** 2 - 3) / (8 * r2)
        assert K[n[2], n[1], n[0]] * r - 1 == pytest.approx(pred, abs=2.0 / r2 ** 2)


def test_lattice_kernel_tends_to_the_sampled_kernel():
    """When the screening spans many cells (a h -> 0) the lattice kernel tends
    to erf(a r)/r at second order in a h."""
    from scipy.special import erf
    err = []
    for ah in (0.4, 0.2, 0.1):
        K = O.lattice_kernel((12, 12, 12), (1.0, 1.0, 1.0), ah)
        ax = np.arange(13.0)
        rz, ry, rx = np.meshgrid(ax, ax, ax, indexing="ij")
        r = np.sqrt(rx * rx + ry * ry + rz * rz)
        with np.errstate(invalid="ignore", divide="ignore"):
            ref = np.where(r > 0, erf(ah * r) / r, 2 * ah / math.sqrt(math.pi))
        err.append(np.abs(K - ref).max() / ref.max())
    assert err[0] < 3e-3
    assert 3.5 < err[0] / err[1] < 4.5 and 3.5 < err[1] / err[2] < 4.5


def test_lattice_fft_route_equals_direct_sum():
    """The zero-padded FFT convolution with the lattice kernel equals the plain
    aperiodic sum over node pairs."""
    grid, hp, a = (4, 5, 3), (0.3, 0.25, 0.4), 2.0
    Q = np.random.default_rng(3).standard_normal((3, 5, 4))
    prm = O.Params(grid, hp, 0.5, a, 2, 1.0, influence="lattice")
    pl = {"hp": np.array(hp), "a": a, "x0": np.zeros(3)}
    phi = O.mesh_potential(Q, prm, pl)
    K = O.lattice_kernel(grid, hp, a)
    ref = np.zeros_like(Q)
    for iz, iy, ix in np.ndindex(*Q.shape):
        for jz, jy, jx in np.ndindex(*Q.shape):
            ref[iz, iy, ix] += Q[jz, jy, jx] * K[abs(iz - jz), abs(iy - jy), abs(ix - jx)]
    assert np.abs(phi - ref).max() <= 1e-13 * np.abs(ref).max()


def test_lattice_force_is_minus_energy_gradient():
    """The lattice kernel is real and even, so the variational mesh force stays
    the exact gradient of the mesh energy."""
    x = _rand_bunch(40, 38, scale=0.5)
    prm = O.Params((12, 12, 12), (0.4, 0.4, 0.4), 0.8, 3.0 / 0.8, 2, 1.0, influence="lattice")
    pl = O.placement(x, prm)
    pl["x0"] = pl["x0"] - 0.013
    F, parts = O.forces(x, prm, parts=True, pl=pl)

    def upm(xx):
        Q = O.deposit(xx, prm, pl)
        return 0.5 * (Q * O.mesh_potential(Q, prm, pl)).sum()

    eps = 1e-7
    for i, d in [(0, 0), (3, 1), (17, 2), (39, 1)]:
        u = (x[i, d] - pl["x0"][d]) / pl["hp"][d]
        knot = u + 0.5 - math.floor(u + 0.5)
        if min(knot, 1 - knot) < 1e-3:
            continue
        xp, xm = x.copy(), x.copy()
        xp[i, d] += eps
        xm[i, d] -= eps
        fd = -(upm(xp) - upm(xm)) / (2 * eps)
        assert fd == pytest.approx(parts["pm"][i, d], rel=1e-5, abs=1e-6 * np.abs(parts["pm"]).max())


# ---- whole force ----------------------------------------------------------------

def test_alpha_zero_large_cutoff_equals_coulomb():
    """a = 0 and r_c wider than the bunch: P3M is the O(N^2) Coulomb sum."""
    x = _rand_bunch(500, 8)
    prm = O.Params((8, 8, 8), (1.0, 1.0, 1.0), 100.0, 0.0, 2, 3.0)
    f = O.forces(x, prm)
    fc = O.coulomb_brute(x, 3.0)
    assert np.abs(f - fc).max() <= 1e-13 * np.abs(fc).max()


def test_zoom_keeps_stencils_on_mesh_and_scales():
    x = _rand_bunch(400, 9, scale=5.0)
    prm = O.Params((16, 16, 16), (0.2, 0.2, 0.2), 0.4, 7.5, 2, 1.0)
    pl = O.placement(x, prm)
    assert pl["s"] > 1
    u = (x - pl["x0"]) / pl["hp"]
    assert u.min() > 0.5 and u.max() < 16 - 1.5
    assert pl["rc"] == pytest.approx(0.4 * pl["s"]) and pl["a"] == pytest.approx(7.5 / pl["s"])


def test_error_paths():
    x = _rand_bunch(50, 10)
    prm = O.Params((16, 16, 16), (0.01, 0.01, 0.01), 0.02, 150.0, 2, 1.0, zoom=False)
    with pytest.raises(O.OracleError) as e:
        O.placement(x, prm)
    assert e.value.code == O.EDOMAIN
    x[3, 1] = np.nan
    prm.zoom = True
    with pytest.raises(O.OracleError) as e:
        O.placement(x, prm)
    assert e.value.code == O.ENONFINITE
    prm.order = 3
    with pytest.raises(O.OracleError) as e:
        O.placement(x[:2] * 0, prm)
    assert e.value.code == O.EINVAL


# ---- integrator (Sec. 2.4.3, eq. leapfrog; Sec. 2.5, eq. eom_p3m_coord) --------------

def _small_run_prm(n=300, seed=12):
    x = _rand_bunch(n, seed, scale=1e-3)
    ke_q2 = 8.9875517923e9 * (1e-9 / n) ** 2
    m = (1e-9 / n) * 9.1093837015e-31 / 1.602176634e-19
    prm = O.Params((16, 16, 16), (8e-3 / 14,) * 3, 2 * 8e-3 / 14, 3.0 / (2 * 8e-3 / 14), 2,
                   ke_q2, m=m, dt=2e-12)
    return x, prm


def test_leapfrog_discrete_euler_lagrange():
    """KDK positions obey m (xi^{n+1} - 2 xi^n + xi^{n-1}) = dt^2 F(xi^n)."""
    x, prm = _small_run_prm()
    p = np.zeros_like(x)
    xs = [x]
    f = None
    for _ in range(3):
        x, p, f = O.step(x, p, prm, 1, f)
        xs.append(x)
    for n in (1, 2):
        lhs = prm.m * (xs[n + 1] - 2 * xs[n] + xs[n - 1])
        rhs = prm.dt ** 2 * O.forces(xs[n], prm)
        assert np.abs(lhs - rhs).max() <= 1e-9 * np.abs(rhs).max()


def test_leapfrog_time_reversible():
    x0, prm = _small_run_prm()
    p0 = np.zeros_like(x0)
    x1, p1, _ = O.step(x0, p0, prm, 5)
    x2, p2, _ = O.step(x1, -p1, prm, 5)
    assert np.abs(x2 - x0).max() <= 1e-9 * np.abs(x1 - x0).max()
    assert np.abs(p2).max() <= 1e-8 * np.abs(p1).max()


def test_two_particles_from_rest_closed_form():
    """Pure Coulomb pair (a = 0) released at r0: s = r/r0 obeys s'' = A/s^2,
    A = 2 k q^2/(m r0^3); t sqrt(2A) = sqrt(s(s-1)) + ln(sqrt(s) + sqrt(s-1)).
    Leapfrog converges to it at second order."""
    ke_q2, m, r0 = 1.0, 1.0, 1.0
    A = 2 * ke_q2 / (m * r0 ** 3)
    T = 1.5
    s_exact = brentq(lambda s: math.sqrt(s * (s - 1)) + math.log(math.sqrt(s) + math.sqrt(s - 1))
                     - T * math.sqrt(2 * A), 1.0 + 1e-12, 100.0)
    errs = []
    for nsteps in (100, 200):
        prm = O.Params((4, 4, 4), (1.0, 1.0, 1.0), 1e6, 0.0, 1, ke_q2, m=m, dt=T / nsteps)
        x = np.array([[0.0, 0.0, -0.5], [0.0, 0.0, 0.5]])
        xn, _, _ = O.step(x, np.zeros_like(x), prm, nsteps)
        errs.append(abs((xn[1, 2] - xn[0, 2]) / r0 - s_exact))
    assert errs[0] < 1e-3
    assert 3.5 < errs[0] / errs[1] < 4.5


def test_energy_bounded():
    x, prm = _small_run_prm(n=200)
    prm.dt = 5e-12
    p = np.zeros_like(x)

    def energy(x, p):
        pl = O.placement(x, prm)
        d = O.diagnostics(x, p, prm, brute_pp=True)
        return d["kinetic"] + d["u_pp"] + d["u_pm"]

    e0 = energy(x, p)
    es = []
    f = None
    for _ in range(6):
        x, p, f = O.step(x, p, prm, 5, f)
        es.append(energy(x, p))
    ke = O.diagnostics(x, p, prm)["kinetic"]
    assert max(abs(e - e0) for e in es) < 0.05 * ke


@pytest.mark.slow
def test_uniform_sphere_expansion_closed_form():
    """Cold uniform ball: r_rms(t) = sqrt(3/5) R s(t) with
    t w_p sqrt(2/3) = sqrt(s(s-1)) + ln(sqrt(s) + sqrt(s-1))."""
    from paper_2103_02046_amd import workloads as W
    wl = W.sphere_tsc(n=20000, grid=32, steps=50)
    x, p = wl.draw()
    prm = O.Params.from_workload(wl)
    xn, pn, _ = O.step(x, p, prm, 50)        # 0.25 plasma periods
    t = 50 * wl.dt
    wp = 2 * math.pi / (200 * wl.dt)
    s = brentq(lambda s: math.sqrt(s * (s - 1)) + math.log(math.sqrt(s) + math.sqrt(s - 1))
               - t * wp * math.sqrt(2 / 3), 1 + 1e-12, 50)
    rrms = math.sqrt(((xn - xn.mean(0)) ** 2).sum(1).mean())
    rrms0 = math.sqrt(((x - x.mean(0)) ** 2).sum(1).mean())
    assert rrms / rrms0 == pytest.approx(s, rel=2e-2)


# ---- adjoint pieces -------------------------------------------------------------

def _adj_setup(order=2, n=80, seed=13):
    x = _rand_bunch(n, seed, scale=0.5)
    prm = O.Params((12, 12, 12), (0.35, 0.35, 0.35), 0.7, 3.0 / 0.7, order, 1.0, m=1.0, dt=0.01)
    pl = O.placement(x, prm)
    pl["x0"] = pl["x0"] - 0.011
    return x, prm, pl


@pytest.mark.parametrize("order", [1, 2])
def test_hvp_symmetric(order):
    x, prm, pl = _adj_setup(order)
    rng = np.random.default_rng(3)
    v, w = rng.standard_normal(x.shape), rng.standard_normal(x.shape)
    a = (O.hvp(x, v, prm, pl) * w).sum()
    b = (v * O.hvp(x, w, prm, pl)).sum()
    assert a == pytest.approx(b, rel=1e-11)


@pytest.mark.parametrize("order", [1, 2])
def test_hvp_matches_force_differences(order):
    x, prm, pl = _adj_setup(order)
    rng = np.random.default_rng(4)
    v = rng.standard_normal(x.shape)
    eps = 1e-7
    fd = (O.forces(x + eps * v, prm, brute=True, pl=pl) - O.forces(x - eps * v, prm, brute=True, pl=pl)) / (2 * eps)
    hv = O.hvp(x, v, prm, pl)
    assert np.abs(fd - hv).max() <= 1e-5 * np.abs(hv).max()


def test_gradient_drift_only_closed_form():
    """k_e = 0: x_N = x_0 + N dt p_0/m, so dJ/dx0 = g_x, dJ/dp0 = g_p + N dt/m g_x."""
    x, prm, _ = _adj_setup()
    prm.ke_q2 = 0.0
    rng = np.random.default_rng(5)
    p = rng.standard_normal(x.shape)
    N = 4
    gx, gp, (xN, pN, _) = O.gradient(x, p, prm, N)
    ex, ep = O.objective_grad(xN, pN, prm)
    np.testing.assert_allclose(gx, ex, rtol=1e-12, atol=1e-14 * np.abs(ex).max())
    np.testing.assert_allclose(gp, ep + N * prm.dt / prm.m * ex, rtol=1e-12,
                               atol=1e-14 * np.abs(ep + ex).max())


def test_gradient_matches_central_differences():
    x, prm, _ = _adj_setup(n=60)
    prm.dt = 0.02
    rng = np.random.default_rng(6)
    p = 0.1 * rng.standard_normal(x.shape)
    N = 3
    gx, gp, (_, _, pls) = O.gradient(x, p, prm, N)
    for _ in range(4):
        dx, dp = rng.standard_normal(x.shape), rng.standard_normal(p.shape)
        eps = 1e-6
        jp = O.objective(*O.forward_frozen(x + eps * dx, p + eps * dp, prm, pls), prm)
        jm = O.objective(*O.forward_frozen(x - eps * dx, p - eps * dp, prm, pls), prm)
        fd = (jp - jm) / (2 * eps)
        an = (gx * dx).sum() + (gp * dp).sum()
        assert an == pytest.approx(fd, rel=1e-5)


# ---- emittance (the adjoint's objective) ------------------------------------------

def test_emittance_closed_form_phase_space():
    """A discrete phase space with exactly known centred moments: points
    (x, p) = (mu_x + a u_k, mu_p + b u_k + c v_k) with u = (1, 1, -1, -1) and
    v = (1, -1, 1, -1) repeated, so <u> = <v> = <uv> = 0 and <u^2> = <v^2> = 1:
    <dx^2> = a^2, <dp^2> = b^2 + c^2, <dx dp> = a b and the normalised rms
    emittance is |a c| / (m c_light). Nonzero means test the centring, the
    shear b the correlation term."""
    u = np.tile([1.0, 1.0, -1.0, -1.0], 25)
    v = np.tile([1.0, -1.0, 1.0, -1.0], 25)
    m = 2.7e-3
    for a, b, c, mx, mp in [(1e-3, 4e-24, 3e-24, 0.37, -8e-22), (2.5e-4, -1e-23, 7e-25, -1.2e-3, 5e-23)]:
        x = np.zeros((len(u), 3))
        p = np.zeros((len(u), 3))
        for ax in range(3):
            x[:, ax] = mx + a * u
            p[:, ax] = mp + b * u + c * v
        for ax in range(3):
            assert O.emittance(x, p, m, ax) == pytest.approx(abs(a * c) / (m * O.C_LIGHT), rel=1e-9)
        J = O.objective(x, p, O.Params((4, 4, 4), (1, 1, 1), 1.0, 0.0, 1, 1.0, m=m))
        assert J == pytest.approx(abs(a * c) / (m * O.C_LIGHT), rel=1e-9)


def test_emittance_invariant_under_drift_and_zero_for_a_line():
    """A drift x -> x + t p / m is a shear of phase space: the covariance
    determinant, hence the emittance, is unchanged. A beam on a straight line
    p = k x in phase space has zero emittance."""
    rng = np.random.default_rng(40)
    x = rng.standard_normal((500, 3)) * 1e-3 + 0.2
    p = rng.standard_normal((500, 3)) * 1e-24 - 3e-24
    m = 1e-30
    for ax in range(3):
        e0 = O.emittance(x, p, m, ax)
        e1 = O.emittance(x + 3e-9 * p / m, p, m, ax)
        assert e1 == pytest.approx(e0, rel=1e-9)
        assert O.emittance(x, 2e-21 * x + 5e-24, m, ax) < 1e-7 * e0


def test_objective_gradient_closed_form_on_the_four_point_beam():
    """dJ/dp for the four-point phase space of the closed-form test: with
    eps = sqrt(a^2 (b^2 + c^2) - a^2 b^2) / (m c) and n points,
    d eps / d p_k = (a^2 dp_k - a b dx_k) / (n eps (m c)^2), d eps / d x_k =
    ((b^2 + c^2) dx_k - a b dp_k) / (n eps (m c)^2); J averages x and y."""
    u = np.tile([1.0, 1.0, -1.0, -1.0], 5)
    v = np.tile([1.0, -1.0, 1.0, -1.0], 5)
    n = len(u)
    a, b, c, m = 2e-3, 3e-24, 5e-24, 1e-30
    x = np.zeros((n, 3))
    p = np.zeros((n, 3))
    for ax in range(3):
        x[:, ax] = 0.1 + a * u
        p[:, ax] = -2e-24 + b * u + c * v
    prm = O.Params((4, 4, 4), (1, 1, 1), 1.0, 0.0, 1, 1.0, m=m)
    gx, gp = O.objective_grad(x, p, prm)
    mc = m * O.C_LIGHT
    eps = abs(a * c) / mc
    dx, dp = a * u, b * u + c * v
    ex = ((b * b + c * c) * dx - a * b * dp) / (n * eps * mc * mc)
    ep = (a * a * dp - a * b * dx) / (n * eps * mc * mc)
    for ax in (0, 1):
        np.testing.assert_allclose(gx[:, ax], 0.5 * ex, rtol=1e-9)
        np.testing.assert_allclose(gp[:, ax], 0.5 * ep, rtol=1e-9)
    assert np.all(gx[:, 2] == 0) and np.all(gp[:, 2] == 0)


def test_optimal_influence_small_screening_limit():
    """When the screening is wide against the mesh (a h = 0.2), the screened
    reference (R gamma)(k) = 4 pi exp(-k^2/4a^2)/k^2 vanishes at every alias
    k - 2 pi m / h (m != 0) of a wavevector in the inner half of the zone, to
    exp(-pi^2/(2 a^2 h^2)) = e^-123. There the numerator of eq. Ghfinal reduces
    to its m = 0 term U^2(k) (R gamma)(k), whatever the alias loops do, and the
    optimal table times the squared aliasing sums of the denominator (the
    table's |m_d| <= 2, pinned to the closed forms above) must return exactly
    that term; the principal table is (R gamma)(k) / U^2(k)."""
    grid = (16, 16, 16)
    hp = np.array([0.3, 0.3, 0.3])
    a = 0.2 / 0.3
    kz = 2 * math.pi * np.fft.fftfreq(32, d=hp[2])
    ky = 2 * math.pi * np.fft.fftfreq(32, d=hp[1])
    kx = 2 * math.pi * np.fft.rfftfreq(32, d=hp[0])
    KZ, KY, KX = np.meshgrid(kz, ky, kx, indexing="ij")
    k2 = KX ** 2 + KY ** 2 + KZ ** 2
    inner = (np.abs(KX) * hp[0] < 0.5 * math.pi) & (np.abs(KY) * hp[1] < 0.5 * math.pi) & \
            (np.abs(KZ) * hp[2] < 0.5 * math.pi) & (k2 > 0)
    rg = np.zeros_like(k2)
    rg[k2 > 0] = 4 * math.pi * np.exp(-k2[k2 > 0] / (4 * a * a)) / k2[k2 > 0]
    V = hp.prod()
    for order in (1, 2):
        u2 = np.ones_like(k2)
        A = np.ones_like(k2)
        for K, h in ((KX, hp[0]), (KY, hp[1]), (KZ, hp[2])):
            s = np.sin(0.5 * K * h)
            with np.errstate(invalid="ignore", divide="ignore"):
                sinc = np.where(K == 0, 1.0, s / (0.5 * K * h))
            u2 = u2 * sinc ** (2 * (order + 1))
            A = A * O.alias_sum_u2(K * h, order, 2)
        G_opt = O.influence_correction(grid, hp, a, order, "optimal", M=2) * V + rg
        G_pri = O.influence_correction(grid, hp, a, order, "principal") * V + rg
        np.testing.assert_allclose((G_opt * A ** 2)[inner], (u2 * rg)[inner], rtol=1e-10)
        np.testing.assert_allclose(G_pri[inner], (rg / u2)[inner], rtol=1e-10)
        # the optimal table is not the principal one here: the assignment's own
        # aliases (not screened) enter the denominator
        assert np.abs(G_opt[inner] / G_pri[inner] - 1).max() > 1e-3


# ---- short-range image term of the grounded plane (Sec. 3.1.1) ----------------------

def test_image_pair_term_lone_charge_closed_form():
    """One charge at height d above the plane meets its own image -q at 2d:
    F_z = -k_e q^2 [erfc(2ad)/(2d) + (2a/sqrt(pi)) e^{-4a^2 d^2}] / (2d) while
    2d < r_c, and nothing from 2d = r_c on: only a particle within r_c/2 of the
    plane feels its image's short-range part (Sec. 3.1.1, Fig. ShortError)."""
    from scipy.special import erfc
    rc, a, zc = 0.8, 3.0 / 0.8, -0.3
    prm = O.Params((8, 8, 8), (0.2, 0.2, 0.2), rc, a, 2, 2.5)
    for d in (0.01, 0.1, 0.25, 0.399, 0.4, 0.41, 0.9):
        x = np.array([[0.2, -0.1, zc + d]])
        f = O.pp_image(x, prm, rc, a, zc)
        r = 2 * d
        exact = 0.0 if r >= rc else -2.5 * (erfc(a * r) / r + 2 * a / math.sqrt(math.pi)
                                            * math.exp(-(a * r) ** 2)) / r
        assert f[0, 2] == pytest.approx(exact, rel=1e-13, abs=1e-300)
        assert f[0, 0] == 0.0 and f[0, 1] == 0.0


def test_image_pair_term_unscreened_is_image_coulomb():
    """a = 0 and a cutoff beyond the bunch: the short-range image term is the
    whole Coulomb force of the images, i.e. the image Coulomb sum minus the
    free-space one (two independent plain sums)."""
    rng = np.random.default_rng(51)
    x = rng.standard_normal((60, 3))
    zc = x[:, 2].min() - 0.2
    prm = O.Params((8, 8, 8), (1, 1, 1), 1e9, 0.0, 2, 1.7)
    f = O.pp_image(x, prm, 1e9, 0.0, zc)
    ref = O.coulomb_image_brute(x, 1.7, zc) - O.coulomb_brute(x, 1.7)
    np.testing.assert_allclose(f, ref, rtol=1e-11, atol=1e-12 * np.abs(ref).max())


def test_image_pair_term_mirror_symmetry():
    """|x_i - S(x_j)| = |x_j - S(x_i)|, and the two separations have equal z
    and opposite transverse components: in a two-particle system the cross
    image forces agree in z and are opposite across."""
    rng = np.random.default_rng(52)
    rc, a, zc = 1.0, 3.0, 0.0
    prm = O.Params((8, 8, 8), (0.2, 0.2, 0.2), rc, a, 2, 1.0)
    for _ in range(5):
        x = np.array([[0.0, 0.0, 0.3], [0.0, 0.0, 0.3]]) + rng.random((2, 3)) * [0.4, 0.4, 0.1]
        own = np.array([O.pp_image(x[k:k + 1], prm, rc, a, zc)[0] for k in range(2)])
        cross = O.pp_image(x, prm, rc, a, zc) - own
        assert cross[0, 2] == pytest.approx(cross[1, 2], rel=1e-12)
        np.testing.assert_allclose(cross[0, :2], -cross[1, :2], rtol=1e-12, atol=1e-15)
