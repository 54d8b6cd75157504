"""GPU path at the workloads' full sizes, against the FP64 oracle.

* 2^20-particle anisotropic Gaussian, 128^3 mesh: every particle's force
  compared with the oracle's full force (cell-list PP + numpy FFT PM).
* the same bunch after 100 float-compensated steps: forces at the GPU's
  positions against the oracle's.
* 2^23-particle uniform sphere, 256^3 mesh: charge and potential node by
  node, the mesh force of every particle, PP forces of sampled particles;
  then a run of one plasma period against the closed-form self-similar
  expansion of a cold uniform ball.
* 2^25-particle core/halo bunch, 512^3 mesh: charge node by node, the
  potential at sampled nodes and the mesh force of sampled core and halo
  particles (oracle's direct potential sums), PP forces of 1200 targets
  including the densest cells; float64 and float-compensated.
* adjoint: gradients of the transverse emittance after 30 steps of 2^16
  particles and of the bunch's second moments after 20 steps of 2^20
  (checkpoints every 10) against central differences along random
  directions (momenta only at 2^20), and symmetry of the Hessian-vector product at 2^20.

Tolerances as in test_gpu_parity: float64 1e-11 relative rms, float32
(compensated) 1e-5, both relative to the rms of the total force; the PP and
mesh parts are checked against the same denominator (their share of the
total error), and their errors relative to their own rms are printed.
Per particle (the error an rms hides): max_i |dF_i| / max(|F_i|, rms F)
below 1e-9 (float64) and 1e-4 (float32, ten times the rms target); max_i
|dF_i| / rms F is printed.
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
MAX64 = 1e-9
MAX32 = 1e-4

from parity_util import per_particle, rms_err  # noqa: E402


def check_particles(label, got, ref, precision, rms=None):
    e_rms, e_own, k = per_particle(got, ref, rms)
    print(f"{label}: per particle max |dF|/rms {e_rms:.3e}, max |dF|/max(|F|, rms) {e_own:.3e} "
          f"(particle {k})", flush=True)
    assert e_own < (MAX64 if precision == p3m.FP64 else MAX32)


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


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
    check_particles(f"aniso1m precision {precision}", fpp + fpm, ref, precision)
    assert c.status_sync() == p3m.OK


def test_aniso1m_after_100_steps_fp32c():
    """100 float-compensated leapfrog steps of the 2^20-particle bunch on the
    GPU, then the force at the GPU's positions (expanded and zoomed) against
    the oracle's at the same positions: the parity holds late in the run,
    not only at the initial draw."""
    wl = W.get("aniso1m")
    x, p = wl.draw()
    c = p3m.Context.from_workload(wl, precision=p3m.FP32C)
    xd, pd = dev(x), dev(p)
    c.step(xd, pd, wl.dt, 100)
    xg = host(xd)
    d0 = c.diagnostics(dev(x), dev(p))
    d1 = c.diagnostics(xd, pd)
    fg = host(c.forces(xd))
    prm = O.Params.from_workload(wl)
    ref = O.forces(xg, prm)
    e = rms_err(fg, ref)
    print(f"aniso1m after 100 fp32c steps (zoom {d0['zoom']:.4f} -> {d1['zoom']:.4f}, pairs "
          f"{d0['pairs']:.3e} -> {d1['pairs']:.3e}): force {e:.3e}", flush=True)
    assert e < TOL32
    check_particles("aniso1m after 100 steps", fg, ref, p3m.FP32C)
    assert c.status_sync() == p3m.OK


@pytest.mark.parametrize("precision", [p3m.FP64, p3m.FP32C])
def test_sphere8m_full_mesh(precision):
    """2^23 particles, 256^3 mesh: the charge and the potential node by node,
    the mesh force of every particle (oracle gather of its full potential),
    and the PP force of 2000 sampled particles."""
    wl = W.get("sphere8m")
    x, _ = wl.draw()
    prm = O.Params.from_workload(wl)
    c = p3m.Context.from_workload(wl, precision=precision)
    fpp, fpm, _ = c.forces_parts(dev(x))
    fpp, fpm = host(fpp), host(fpm)
    Qg, phig = host(c.mesh(0)), host(c.mesh(1))
    pl = O.placement(x, prm)
    Q = O.deposit(x, prm, pl)
    phi = O.conv_fft(Q, prm.grid, pl["hp"], pl["a"])
    eq = np.abs(Qg - Q).max() / np.abs(Q).max()
    ephi = rms_err(phig, phi)
    ref_pm = O.gather(x, prm, pl, phi)
    rng = np.random.default_rng(1)
    idx = np.sort(rng.choice(wl.n, 2000, replace=False))
    ref_pp = O.pp_sample(x, prm, pl["rc"], pl["a"], idx)
    tol = TOL64 if precision == p3m.FP64 else TOL32
    tot = ref_pp + ref_pm[idx]
    e_pm = rms_err(fpm, ref_pm)
    e_pp = rms_err(fpp[idx], ref_pp, tot)
    e = rms_err(fpp[idx] + fpm[idx], tot)
    print(f"sphere8m precision {precision}: Q max node {eq:.3e}, phi {ephi:.3e}, pm (every particle) "
          f"{e_pm:.3e}, sampled pp {e_pp:.3e} (own rms {rms_err(fpp[idx], ref_pp):.3e}), sampled total {e:.3e}",
          flush=True)
    assert eq < (1e-12 if precision == p3m.FP64 else 1e-6)
    assert ephi < tol and e_pm < tol and e_pp < tol and e < tol
    rms_tot = math.sqrt((tot ** 2).sum(axis=1).mean())
    check_particles(f"sphere8m pm precision {precision}", fpm, ref_pm, precision, rms=rms_tot)
    check_particles(f"sphere8m sampled total precision {precision}", fpp[idx] + fpm[idx], tot, precision)
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


@pytest.mark.parametrize("precision", [p3m.FP64, p3m.FP32C])
def test_halo32m_sampled(precision):
    """2^25 particles, 512^3 mesh: the charge node by node over the whole
    mesh; the potential at the 216 stencil nodes of 8 sampled particles (core
    and halo, by the oracle's direct sums over the mesh charge) and those
    particles' mesh forces; the PP force of 1200 targets, 400 of them the
    particles nearest the centre (the densest cells, ~3900 neighbours)."""
    wl = W.get("halo32m")
    x, _ = wl.draw()
    prm = O.Params.from_workload(wl)
    c = p3m.Context.from_workload(wl, precision=precision)
    xd = dev(x)
    fpp, fpm, _ = c.forces_parts(xd)
    fpp, fpm = host(fpp), host(fpm)
    del xd
    assert c.status_sync() == p3m.OK
    Qg = host(c.mesh(0))
    phig = host(c.mesh(1))
    print(f"halo32m precision {precision}: GPU done, mesh bits {c.info()['mesh_bits']}", flush=True)
    pl = O.placement(x, prm)
    Q = O.deposit(x, prm, pl)
    eq = np.abs(Qg - Q).max() / np.abs(Q).max()
    print(f"halo32m: Q max node error {eq:.3e}", flush=True)
    assert eq < (1e-12 if precision == p3m.FP64 else 1e-6)
    del Qg
    rng = np.random.default_rng(2)
    core, _ = W.halo_split(wl.n)
    r = np.linalg.norm(x, axis=1)
    dense = np.argsort(r[:core])[:400]
    idx = np.unique(np.concatenate([dense, rng.choice(core, 700, replace=False),
                                    core + rng.choice(wl.n - core, 100, replace=False)]))
    ref_pp = O.pp_sample(x, prm, pl["rc"], pl["a"], idx)
    print(f"halo32m: oracle PP of {len(idx)} targets done (densest target has "
          f"{int(r[dense[0]] * 1e6)} um radius)", flush=True)
    # mesh: 8 particles (5 core incl. the densest, 3 halo), potential at their stencil nodes
    pm_idx = np.unique(np.concatenate([dense[:1], rng.choice(core, 4, replace=False),
                                       core + rng.choice(wl.n - core, 3, replace=False)]))
    nodes = np.unique(np.concatenate([O.stencil_nodes(x[i], prm, pl) for i in pm_idx]))
    vals = O.phi_at(Q, prm.grid, pl["hp"], pl["a"], nodes)
    ephi = rms_err(phig.reshape(-1)[nodes], vals)
    phi = np.zeros_like(Q)
    phi.reshape(-1)[nodes] = vals
    ref_pm = O.gather(x[pm_idx], prm, pl, phi)
    print(f"halo32m: oracle potential at {len(nodes)} nodes done", flush=True)
    tol = TOL64 if precision == p3m.FP64 else TOL32
    sel = np.searchsorted(idx, pm_idx)
    in_pp = idx[np.clip(sel, 0, len(idx) - 1)] == pm_idx
    ref_pp_pm = O.pp_sample(x, prm, pl["rc"], pl["a"], pm_idx)
    tot = ref_pp_pm + ref_pm
    e_pm = rms_err(fpm[pm_idx], ref_pm, tot)
    e_tot = rms_err(fpp[pm_idx] + fpm[pm_idx], tot)
    # PP part on the 1200 targets, against their PP + mesh total (mesh from the GPU)
    e_pp = rms_err(fpp[idx], ref_pp, ref_pp + fpm[idx])
    print(f"halo32m precision {precision}: phi at nodes {ephi:.3e}; sampled pp {e_pp:.3e} "
          f"(own rms {rms_err(fpp[idx], ref_pp):.3e}) pm {e_pm:.3e} total {e_tot:.3e} "
          f"({int(in_pp.sum())} of the mesh sample among the PP targets)", flush=True)
    assert ephi < tol and e_pp < tol and e_pm < tol and e_tot < tol
    check_particles(f"halo32m pp precision {precision}", fpp[idx], ref_pp, precision,
                    rms=math.sqrt(((ref_pp + fpm[idx]) ** 2).sum(axis=1).mean()))
    check_particles(f"halo32m total precision {precision}", fpp[pm_idx] + fpm[pm_idx], tot, precision)


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
