"""GPU path at the workloads' full sizes, against the FP64 oracle.

* 2^20-particle anisotropic Gaussian, 128^3 mesh: every particle's force
  compared with the oracle's full force (cell-list PP + numpy FFT PM).
* 2^23-particle uniform sphere, 256^3 mesh: PP forces of sampled particles
  (oracle cell list) and their mesh forces (oracle deposit + FFT potential);
  then a run of one plasma period against the closed-form self-similar
  expansion of a cold uniform ball.
* 2^25-particle core/halo bunch, 512^3 mesh: sampled PP forces, and the mesh
  force of two sampled particles from the oracle's direct potential sums at
  their stencil nodes.
* adjoint: gradients of the transverse emittance after 30 steps of 2^16
  particles and of the bunch's second moments after 20 steps of 2^20
  (checkpoints every 10) against central differences along random
  directions (momenta only at 2^20), and symmetry of the Hessian-vector product at 2^20.

Tolerances as in test_gpu_parity: float64 1e-11 relative rms, float32
(compensated) 1e-5, both relative to the rms of the total force; the PP and
mesh parts are checked against the same denominator (their share of the
total error), and their errors relative to their own rms are printed.
"""
import dataclasses
import math

import numpy as np
import pytest
import torch
from scipy.optimize import brentq

from oracle import oracle as O
from paper_2103_02046_amd import p3m
from paper_2103_02046_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-11
TOL32 = 1e-5


def rms_err(a, b, ref=None):
    ref = np.asarray(b) if ref is None else np.asarray(ref)
    return math.sqrt(((np.asarray(a) - np.asarray(b)) ** 2).sum() / (ref ** 2).sum())


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _sampled_pm(x, prm, pl, Q, idx, phi_full=None):
    """Oracle mesh force of particles idx: potential at their stencil nodes
    (from the full potential if given, else by direct sums), then the gather."""
    g = prm.grid
    phi = np.zeros((g[2], g[1], g[0]))
    if phi_full is not None:
        phi = phi_full
    else:
        nodes = np.unique(np.concatenate([O.stencil_nodes(x[i], prm, pl) for i in idx]))
        vals = O.phi_at(Q, g, pl["hp"], pl["a"], nodes)
        phi.reshape(-1)[nodes] = vals
    sub = O.Params(prm.grid, prm.h, prm.r_cut, prm.split, prm.order, prm.ke_q2, prm.m, prm.dt,
                   qw=None if prm.qw is None else prm.qw[idx])
    return O.gather(x[idx], sub, pl, phi)


@pytest.mark.parametrize("precision", [p3m.FP64, p3m.FP32C])
def test_aniso1m_every_particle(precision):
    wl = W.get("aniso1m")
    x, _ = wl.draw()
    prm = O.Params.from_workload(wl)
    ref, parts = O.forces(x, prm, parts=True)
    c = p3m.Context.from_workload(wl, precision=precision)
    fpp, fpm, pl = c.forces_parts(dev(x))
    fpp, fpm = host(fpp), host(fpm)
    tol = TOL64 if precision == p3m.FP64 else TOL32
    e = rms_err(fpp + fpm, ref)
    print(f"aniso1m precision {precision}: total {e:.3e}; pp {rms_err(fpp, parts['pp'], ref):.3e} "
          f"(own rms {rms_err(fpp, parts['pp']):.3e}), pm {rms_err(fpm, parts['pm'], ref):.3e} "
          f"(own rms {rms_err(fpm, parts['pm']):.3e})", flush=True)
    assert e < tol
    assert rms_err(fpp, parts["pp"], ref) < tol and rms_err(fpm, parts["pm"], ref) < tol
    assert c.status_sync() == p3m.OK


@pytest.mark.parametrize("precision", [p3m.FP64, p3m.FP32C])
def test_sphere8m_sampled(precision):
    wl = W.get("sphere8m")
    x, _ = wl.draw()
    prm = O.Params.from_workload(wl)
    c = p3m.Context.from_workload(wl, precision=precision)
    fpp, fpm, _ = c.forces_parts(dev(x))
    fpp, fpm = host(fpp), host(fpm)
    pl = O.placement(x, prm)
    rng = np.random.default_rng(1)
    idx = np.sort(rng.choice(wl.n, 48, replace=False))
    ref_pp = O.pp_sample(x, prm, pl["rc"], pl["a"], idx)
    Q = O.deposit(x, prm, pl)
    phi = O.conv_fft(Q, prm.grid, pl["hp"], pl["a"])
    ref_pm = _sampled_pm(x, prm, pl, Q, idx, phi)
    tol = TOL64 if precision == p3m.FP64 else TOL32
    tot = ref_pp + ref_pm
    e_pp, e_pm = rms_err(fpp[idx], ref_pp, tot), rms_err(fpm[idx], ref_pm, tot)
    e = rms_err(fpp[idx] + fpm[idx], tot)
    print(f"sphere8m precision {precision}: sampled total {e:.3e} pp {e_pp:.3e} pm {e_pm:.3e} "
          f"(own rms pp {rms_err(fpp[idx], ref_pp):.3e} pm {rms_err(fpm[idx], ref_pm):.3e})", flush=True)
    assert e_pp < tol and e_pm < tol and e < tol
    # whole-mesh invariants of the deposit: total charge
    assert c.status_sync() == p3m.OK


def test_sphere8m_expansion_closed_form():
    """Cold uniform ball: r_rms(t) = sqrt(3/5) R s(t) with
    t w_p sqrt(2/3) = sqrt(s(s-1)) + ln(sqrt(s) + sqrt(s-1)); one plasma
    period (200 steps) gives s = 4.30, checked on the float32-compensated path.
    The float64 path runs the first quarter period, where the two agree.
    (Close encounters of the point charges throw a few particles far out; the
    bounding-box placement then zooms the mesh well past the bulk and the
    late steps carry many pairs per cell, most expensive in float64.)"""
    import time
    wl = W.get("sphere8m")
    x, p = wl.draw()
    wp = 2 * math.pi / (200 * wl.dt)

    def closed_form(t):
        return brentq(lambda s: math.sqrt(s * (s - 1)) + math.log(math.sqrt(s) + math.sqrt(s - 1))
                      - t * wp * math.sqrt(2 / 3), 1 + 1e-12, 50)

    rr0 = math.sqrt(((x - x.mean(0)) ** 2).sum(1).mean())
    out = {}
    for precision, steps in ((p3m.FP32C, wl.steps), (p3m.FP64, 50)):
        c = p3m.Context.from_workload(wl, precision=precision)
        xd, pd = dev(x), dev(p)
        cached = False       # a diagnostics call drops the cached force
        for k in range(0, steps, 25):
            t0 = time.perf_counter()
            c.step(xd, pd, wl.dt, 25, reuse_force=cached)
            torch.cuda.synchronize()
            cached = True
            print(f"sphere8m precision {precision}: step {k + 25} ({time.perf_counter() - t0:.1f} s)",
                  flush=True)
            if k + 25 == 50:
                d = c.diagnostics(xd, pd)
                cached = False
                out[(precision, 50)] = math.sqrt(sum(v * v for v in d["rms"])) / rr0
        d = c.diagnostics(xd, pd)
        out[(precision, steps)] = math.sqrt(sum(v * v for v in d["rms"])) / rr0
        assert c.status_sync() == p3m.OK
        print(f"sphere8m precision {precision}: r_rms ratio {out[(precision, steps)]:.5f} after {steps} "
              f"steps, closed form {closed_form(steps * wl.dt):.5f}, zoom {d['zoom']:.3f}")
    assert out[(p3m.FP32C, wl.steps)] == pytest.approx(closed_form(wl.steps * wl.dt), rel=1e-2)
    assert out[(p3m.FP64, 50)] == pytest.approx(closed_form(50 * wl.dt), rel=1e-2)
    assert out[(p3m.FP32C, 50)] == pytest.approx(out[(p3m.FP64, 50)], rel=1e-5)


@pytest.mark.parametrize("precision", [p3m.FP32C])
def test_halo32m_sampled(precision):
    wl = W.get("halo32m")
    x, _ = wl.draw()
    prm = O.Params.from_workload(wl)
    c = p3m.Context.from_workload(wl, precision=precision)
    xd = dev(x)
    fpp, fpm, _ = c.forces_parts(xd)
    fpp, fpm = host(fpp), host(fpm)
    del xd
    assert c.status_sync() == p3m.OK
    pl = O.placement(x, prm)
    rng = np.random.default_rng(2)
    core, _ = W.halo_split(wl.n)
    idx = np.sort(np.concatenate([rng.choice(core, 24, replace=False),
                                  core + rng.choice(wl.n - core, 8, replace=False)]))
    ref_pp = O.pp_sample(x, prm, pl["rc"], pl["a"], idx)
    print("halo32m: oracle PP sample done", flush=True)
    Q = O.deposit(x, prm, pl)
    two = np.array([idx[0], idx[-1]])           # one core, one halo particle
    ref_pm = _sampled_pm(x, prm, pl, Q, two)
    print("halo32m: oracle potential sample done", flush=True)
    sel = np.searchsorted(idx, two)
    tot = ref_pp[sel] + ref_pm
    e_pm = rms_err(fpm[two], ref_pm, tot)
    e_tot = rms_err(fpp[two] + fpm[two], tot)
    # PP part on all sampled particles, against their PP+mesh total (mesh from the GPU)
    e_pp = rms_err(fpp[idx], ref_pp, ref_pp + fpm[idx])
    print(f"halo32m precision {precision}: sampled pp {e_pp:.3e} (own rms {rms_err(fpp[idx], ref_pp):.3e}) "
          f"pm {e_pm:.3e} total {e_tot:.3e}", flush=True)
    assert e_pp < TOL32 and e_pm < TOL32 and e_tot < TOL32


def _emit(mc):
    def emit(xx, pp):
        out = 0
        for ax in (0, 1):
            dx = xx[:, ax] - xx[:, ax].mean()
            dp = pp[:, ax] - pp[:, ax].mean()
            out = out + torch.sqrt((dx * dx).mean() * (dp * dp).mean() - (dx * dp).mean() ** 2)
        return 0.5 * out / mc
    return emit


def _spread(sig_x, sig_p):
    def spread(xx, pp):
        return (((xx - xx.mean(0)) / sig_x) ** 2).mean() + (((pp - pp.mean(0)) / sig_p) ** 2).mean()
    return spread


def _adjoint_and_fd(wl, c, x, p, nsteps, every, eps_list, ndir, support, emit=None, kinds=(0, 1)):
    """Adjoint gradient of J (default: the transverse emittance) after nsteps,
    and central differences along random directions (supported on particles
    0..support-1) from float64 GPU runs replaying the forward run's placements."""
    emit = _emit(wl.m * W.C_LIGHT) if emit is None else emit
    x0 = dev(x).requires_grad_(True)
    p0 = dev(p).requires_grad_(True)
    xN, pN = p3m.rollout(x0, p0, c, wl.dt, nsteps, every=every)
    emit(xN, pN).backward()
    gx, gp = host(x0.grad), host(p0.grad)
    print("adjoint done", flush=True)
    places = torch.empty((nsteps + 1) * 4, dtype=torch.float64, device="cuda")
    c.step(dev(x), dev(p), wl.dt, nsteps, place_record=places)

    def run(dx, dp):
        xa, pa = dev(x + dx), dev(p + dp)
        c.step(xa, pa, wl.dt, nsteps, place_replay=places)
        assert c.status_sync() == p3m.OK      # every perturbed stencil stayed on the mesh
        return float(emit(xa, pa))

    rng = np.random.default_rng(3)
    sig_x = 1e-3
    sig_p = wl.m * sig_x / (200 * wl.dt)
    out = []
    for k in range(ndir):
        dx = np.zeros_like(x)
        dp = np.zeros_like(p)
        d = rng.standard_normal((support, 3))
        if kinds[k % len(kinds)] == 0:
            dx[:support] = d / np.linalg.norm(d) * sig_x
        else:
            dp[:support] = d / np.linalg.norm(d) * sig_p
        an = float((gx * dx).sum() + (gp * dp).sum())
        fds = [(run(e * dx, e * dp) - run(-e * dx, -e * dp)) / (2 * e) for e in eps_list]
        out.append((an, fds))
        print(f"direction {k}: adjoint {an:.8e} central differences " +
              " ".join(f"{f:.8e}" for f in fds), flush=True)
    return out


def test_adjoint_vs_central_differences_smooth_cutoff():
    """With the Ewald parameter at its configured kappa = a r_c = 3, the PP force
    jumps at the strict cutoff by erfc(3) + (6/sqrt(pi)) e^-9 = 4.4e-4 of the
    Coulomb force there: J is only piecewise smooth and central differences
    pick up the pairs that cross r_c, which the adjoint (the derivative almost
    everywhere) rightly ignores. Raising kappa to 5 brings the jump to 8e-11,
    and every central difference must then match the adjoint to 1e-5. 2^16
    particles, 64^3 mesh, 30 steps, checkpoints every 10. The step is 1e-5 of
    a perturbation of 1 mm norm: float64 atomics make J differ between runs by
    about 1e-16 relative, amplified by the dynamics, which at a step of 1e-6
    already moves the difference quotient by 1e-5."""
    wl0 = W.aniso_tsc(n=1 << 16, grid=64, steps=30)
    wl = dataclasses.replace(wl0, split=5.0 / wl0.r_cut)
    x, p = wl.draw()
    c = p3m.Context.from_workload(wl, precision=p3m.FP64)
    res = _adjoint_and_fd(wl, c, x, p, wl.steps, 10, [1e-5], 6, 4096)
    for an, fds in res:
        assert abs(an - fds[0]) <= 1e-5 * abs(fds[0])


def test_aniso1m_adjoint_vs_central_differences():
    """2^20 particles on the 128^3 mesh with kappa raised to 5 for the reason
    above, 20 steps in two checkpoint segments of 10; the perturbations cover
    2^16 particles' momenta. J is the sum of the coordinate and momentum
    variances: the emittance of this nearly laminar bunch is the small
    difference of large second moments, so its own rounding would swamp the
    difference quotient. The step is 1e-3 of the perturbation: J is O(1) and
    moves by 1e-10 of itself, well clear of its rounding. Perturbed positions
    are left to the 2^16-particle check: the pair force has no softening and
    among 2^20 particles the closest pairs sit ~1e-7 m apart, where a position
    step large enough to beat rounding is already nonlinear. The adjoint must
    agree to 1e-5."""
    wl = dataclasses.replace(W.get("aniso1m"), split=5.0 / W.get("aniso1m").r_cut)
    x, p = wl.draw()
    c = p3m.Context.from_workload(wl, precision=p3m.FP64)
    sig_p = wl.m * 1e-3 / (200 * wl.dt)
    res = _adjoint_and_fd(wl, c, x, p, 20, 10, [1e-3], 6, 1 << 16, emit=_spread(1e-3, sig_p), kinds=(1,))
    for an, fds in res:
        assert abs(an - fds[0]) <= 1e-5 * abs(fds[0])


def test_aniso1m_hvp_symmetric():
    """The force Jacobian is the negative Hessian of the energy, so the
    Hessian-vector product is symmetric: w.Hv = v.Hw at the configuration's
    own size and kappa = 3."""
    wl = W.get("aniso1m")
    x, _ = wl.draw()
    c = p3m.Context.from_workload(wl, precision=p3m.FP64)
    rng = np.random.default_rng(12)
    v, w = rng.standard_normal(x.shape), rng.standard_normal(x.shape)
    xd = dev(x)
    hv, hw = host(c.hvp(xd, dev(v))), host(c.hvp(xd, dev(w)))
    a, b = float((w * hv).sum()), float((v * hw).sum())
    scale = math.sqrt((hv ** 2).sum() * (w ** 2).sum())
    print(f"w.Hv {a:.12e} v.Hw {b:.12e} scale {scale:.3e}", flush=True)
    assert abs(a - b) <= 1e-12 * scale
