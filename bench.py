"""Throughput of the P3M leapfrog step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload halo32m]
                    [--precision fp32c|fp64] [--fp64-steps 3] [--no-cpu-baseline]

Default workload: the 2^25-particle core/halo bunch on a 512^3 mesh (1024^3
zero-padded FFT), TSC, r_c = 2h, kappa = 3, dt = T_p/200, float-compensated
path; the largest workload that runs on one GPU.

One step = one kick-drift-kick leapfrog step of the whole bunch: push,
placement, linked-cell sort, PP pair forces, deposit, FFT convolution,
gather (every stage of the P3M force evaluation). Inputs are resident in HBM
before the timed region. Warm-up steps run on a copy of the bunch; the K
timed steps then start from the initial state, whose force is evaluated
before the timer starts, so the timed region holds exactly the run's K
steps and K force evaluations.

Prints one JSON line with the metric, a roofline entry for the dominant
kernel (timed live with HIP events on the library's stream during the timed
region, around that stage alone) and the FP64 CPU oracle timed on a bounded
sample on this host. The per-stage breakdown comes from a replica of the same
trajectory run before the timed region with every stage timed.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E, GB/s
PEAK_FP32_VALU = 157.3         # TFLOP/s, vector FP32 (256 CU x 2.4 GHz)
PEAK_FP64_VALU = 78.6          # TFLOP/s, vector FP64
PP_FLOP_PER_PAIR = 40          # per in-cutoff ordered pair: FMA 2, rsqrt/exp/rcp 1 each, the 7-term
                               # polynomial 14, plus the separation, products and Kahan adds


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="halo32m")
    ap.add_argument("--precision", default="fp32c", choices=["fp32c", "fp64"])
    ap.add_argument("--gather", default="variational", choices=["variational", "momentum"],
                    help="mesh force at the particles: variational (default) or momentum-conserving")
    ap.add_argument("--influence", default="sampled", choices=["sampled", "optimal", "principal", "lattice"],
                    help="Fourier table of the mesh kernel (built at create)")
    ap.add_argument("--cathode", action="store_true",
                    help="grounded plane 1 mm below the bunch (image charges on the mesh)")
    ap.add_argument("--pp-cell-div", type=int, default=None, choices=[1, 2],
                    help="PP cells per cutoff along each axis (default: the workload's own)")
    ap.add_argument("--fp64-steps", type=int, default=3,
                    help="leapfrog steps of the float64 path timed for its own particle-steps/s (0: skip)")
    ap.add_argument("--cpu-targets", type=int, default=32768,
                    help="sampled PP targets of the CPU oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of known size (for HBM counter scaling)")
    return ap.parse_args()


def stage_sources():
    return {
        "pp": ["pp.hip", "erfcx_fit.h", "common.h"],
        "fft": ["fft.hip", "common.h"],
        "sort": ["sort.hip", "common.h"],
        "deposit": ["mesh.hip", "common.h"],
        "gather": ["mesh.hip", "bbox.h", "common.h"],
        "reorder": ["sort.hip", "common.h"],
        "push+placement": ["placement.hip", "bbox.h", "common.h"],
    }


def source_hash(stage):
    h = hashlib.sha256()
    for f in stage_sources()[stage]:
        with open(os.path.join(ROOT, "paper_2103_02046_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(stage, workload, precision, launches_per_step):
    """HBM bytes per launch from the committed counter summary, or None if the
    summary is missing or was taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{stage}_{workload}_{precision}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("source_hash") != source_hash(stage):
        return None
    return d.get("bytes_per_launch")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def workload_text(name, wl):
    """The workload spelled out: particles, draw, mesh, assignment, cutoff, split, time step."""
    draws = {
        "gauss": "isotropic Gaussian sigma 1 mm",
        "aniso": "Gaussian sigma (1, 1, 3) mm",
        "sphere": "uniform ball of radius 1 mm at rest",
        "halo": "90% Gaussian core sigma 0.5 mm + 10% r^-2 halo from 0.5 to 5 mm",
    }
    g = wl.grid
    rc_h = wl.r_cut / min(wl.h)
    return (f"{name}: {wl.n} particles, {draws[wl.name]}, seed {wl.seed}; "
            f"{g[0]}x{g[1]}x{g[2]} mesh ({2 * g[0]}x{2 * g[1]}x{2 * g[2]} zero-padded FFT), "
            f"{'TSC' if wl.order == 2 else 'CIC'}, r_c = {rc_h:g} h, kappa = a r_c = {wl.split * wl.r_cut:g}, "
            f"dt = T_p/200 = {wl.dt:.4g} s")


def cpu_baseline(wl, n_targets):
    """The FP64 CPU oracle as it stands (compiled here with -O3 -march=native,
    OpenMP on every core), timed part by part on a bounded sample of one
    leapfrog step of the same workload, scaled to the whole step:
      * PP: the pair forces of sampled targets through the oracle's cell
        list over all particles; timed at K and 2K targets, so the cell build
        (once per evaluation) and the cost per target separate, then scaled
        to N targets;
      * deposit, gather and the kick-drift-kick arrays: all N particles;
      * mesh convolution (numpy FFTs, kernel table included): in full up to
        a 256^3 mesh; above, on the mesh halved per axis and scaled by the
        transform work M log M."""
    import numpy as np
    from oracle import oracle as O
    import tempfile
    so = os.path.join(tempfile.gettempdir(), f"liboracle_native_{os.getpid()}.so")
    O.build_native(so)
    O.use_library(so)
    x, p = wl.draw()
    prm = O.Params.from_workload(wl)
    t_all = time.perf_counter()
    pl = O.placement(x, prm)
    # sampled targets: runs of 256 particles consecutive in an order by PP
    # cell, started at random, so that each run is a spatial neighbourhood
    # (the full evaluation's targets share neighbours in the caches too);
    # the selection is not timed
    rng = np.random.default_rng(123)
    cell = np.floor((x - pl["x0"]) / pl["rc"]).astype(np.int64)
    nc = cell.max(axis=0) + 1
    order = np.argsort((cell[:, 2] * nc[1] + cell[:, 1]) * nc[0] + cell[:, 0], kind="stable")
    del cell
    run = 256
    t_pp = []
    for k in (n_targets, 2 * n_targets):
        starts = rng.choice(max(wl.n - run, 1), max(k // run, 1), replace=False)
        idx = np.sort(np.concatenate([order[s0:s0 + run] for s0 in starts]))
        t0 = time.perf_counter()
        O.pp_sample(x, prm, pl["rc"], pl["a"], idx)
        t_pp.append(time.perf_counter() - t0)
    del order
    per_target = max(t_pp[1] - t_pp[0], 1e-12) / n_targets
    build = max(t_pp[0] - per_target * n_targets, 0.0)
    pp_est = build + per_target * wl.n
    t0 = time.perf_counter()
    Q = O.deposit(x, prm, pl)
    t_dep = time.perf_counter() - t0
    g = np.asarray(prm.grid)
    if g.max() <= 256:
        t0 = time.perf_counter()
        phi = O.mesh_potential(Q, prm, pl)
        t_conv = time.perf_counter() - t0
        conv_note = "in full"
    else:
        gh = tuple(int(v) // 2 for v in g)
        Qh = np.ascontiguousarray(Q[:gh[2], :gh[1], :gh[0]])
        t0 = time.perf_counter()
        O.conv_fft(Qh, gh, pl["hp"], pl["a"])
        t_half = time.perf_counter() - t0
        m_full, m_half = 8.0 * g.prod(), 8.0 * np.prod(gh)
        t_conv = t_half * (m_full * math.log2(m_full)) / (m_half * math.log2(m_half))
        phi = np.zeros_like(Q)   # the gather's cost does not depend on phi's values
        conv_note = f"on the {gh[0]}^3 mesh ({t_half:.1f} s), scaled by M log M"
    t0 = time.perf_counter()
    f = O.gather(x, prm, pl, phi)
    p += 0.5 * prm.dt * f
    x += prm.dt * p / prm.m
    p += 0.5 * prm.dt * f
    t_gat = time.perf_counter() - t0
    step_s = pp_est + t_dep + t_conv + t_gat
    wall = time.perf_counter() - t_all
    try:
        os.remove(so)
    except OSError:
        pass
    return {"value": wl.n / step_s, "unit": "particle-steps/s", "cores": O.threads(),
            "kind": "oracle",
            "sample": (f"one leapfrog step of {wl.name} ({wl.n} particles) estimated from parts: PP of "
                       f"{n_targets} and {2 * n_targets} targets (random runs of 256 in cell order) "
                       f"over the full cell list "
                       f"({t_pp[0]:.2f} s, {t_pp[1]:.2f} s; cell build {build:.2f} s + "
                       f"{per_target * 1e6:.1f} us/target -> {pp_est:.1f} s for all), deposit {t_dep:.2f} s, "
                       f"mesh convolution {t_conv:.1f} s ({conv_note}), gather + kicks + drift "
                       f"{t_gat:.2f} s; {wall:.1f} s of CPU time"),
            "cpu": cpu_model(), "build": "gcc -O3 -march=native -fopenmp -ffp-contract=off; numpy FFT",
            "seconds_per_step": step_s}


def load_balance(waves):
    """Load balance of one pair-kernel launch from the start and end (us) of
    each of its waves: the span, the most waves resident at once, the
    fraction of (resident slots x span) the waves kept busy, the fraction of
    the span with fewer than half that many waves resident (the tail), and
    the spread of the wave durations."""
    import numpy as np
    w = np.asarray(waves)
    if len(w) == 0:
        return None
    t0, t1 = w[:, 0].min(), w[:, 1].max()
    ev = np.concatenate([np.stack([w[:, 0], np.ones(len(w))], 1), np.stack([w[:, 1], -np.ones(len(w))], 1)])
    ev = ev[np.lexsort((ev[:, 1], ev[:, 0]))]
    busy = np.cumsum(ev[:, 1])
    slots = int(busy.max())
    dt = np.diff(ev[:, 0])
    low = float((dt * (busy[:-1] < 0.5 * slots)).sum())
    dur = w[:, 1] - w[:, 0]
    span = t1 - t0
    return {"waves": int(len(w)), "span_us": float(span), "max_resident_waves": slots,
            "busy_fraction": float(dur.sum() / (slots * span)) if span > 0 else None,
            "tail_fraction_below_half_resident": float(low / span) if span > 0 else None,
            "wave_us_mean": float(dur.mean()), "wave_us_p50": float(np.percentile(dur, 50)),
            "wave_us_p99": float(np.percentile(dur, 99)), "wave_us_max": float(dur.max())}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    from paper_2103_02046_amd import p3m
    from paper_2103_02046_amd import workloads as W

    wl = W.get(args.workload)
    prec = p3m.FP32C if args.precision == "fp32c" else p3m.FP64
    x0, p0 = wl.draw()
    dev = torch.device("cuda:0")
    x = torch.tensor(x0, dtype=torch.float64, device=dev)
    p = torch.tensor(p0, dtype=torch.float64, device=dev)
    gmode = p3m.GATHER_MOMENTUM if args.gather == "momentum" else p3m.GATHER_VARIATIONAL
    zc = float(x0[:, 2].min()) - 1e-3 if args.cathode else None
    infl = {"sampled": p3m.INFLUENCE_SAMPLED, "optimal": p3m.INFLUENCE_OPTIMAL,
            "principal": p3m.INFLUENCE_PRINCIPAL, "lattice": p3m.INFLUENCE_LATTICE}[args.influence]
    ckw = dict(gather=gmode, cathode_z=zc, influence=infl)
    if args.pp_cell_div is not None:
        ckw["pp_cell_div"] = args.pp_cell_div
    ctx = p3m.Context.from_workload(wl, precision=prec, **ckw)

    d0 = ctx.diagnostics(x, p)
    info = ctx.info()

    if args.copy_calibration:
        a = torch.empty(64 << 20, dtype=torch.float64, device=dev)   # 512 MiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # warm-up on a copy
    xw, pw = x.clone(), p.clone()
    ctx.step(xw, pw, wl.dt, max(args.warmup, 1))
    del xw, pw
    torch.cuda.synchronize()

    # replica of the trajectory, before the timed region: every stage timed
    # (averages per launch) and the in-cutoff pairs per force evaluation,
    # counted every 10 steps (the diagnostics run outside the timed windows)
    xr = torch.tensor(x0, dtype=torch.float64, device=dev)
    pr = torch.tensor(p0, dtype=torch.float64, device=dev)
    counts = [d0["pairs"]]
    stage_ms = {s: 0.0 for s in p3m.STAGES}
    stage_n = {s: 0 for s in p3m.STAGES}
    done = 0
    waves = None
    while done < args.steps:
        k = min(10, args.steps - done)
        last = done + k >= args.steps
        ctx.profile_begin(8 * (k + 2), pp_waves=last)
        ctx.step(xr, pr, wl.dt, k)
        for s_, (ms_, cnt_) in ctx.profile_end().items():
            stage_ms[s_] += ms_
            stage_n[s_] += cnt_
        if last:
            waves = ctx.pp_waves()   # the pair kernel's waves in the replica's last evaluation
        done += k
        counts.append(ctx.diagnostics(xr, pr)["pairs"])
    pairs = sum(0.5 * (a + b) for a, b in zip(counts, counts[1:])) / max(len(counts) - 1, 1)
    per_launch = {s_: stage_ms[s_] / max(stage_n[s_], 1) for s_ in p3m.STAGES}
    stage = max(per_launch, key=per_launch.get)
    del xr, pr

    # timed region: the K steps from the initial state, whose force is
    # evaluated before the timer starts. Only the dominant stage carries
    # events (each event pair idles the GPU about 2 us between kernels).
    ctx.step(x, p, wl.dt, 0)
    torch.cuda.synchronize()
    ctx.profile_begin(2 * (args.steps + 2), stages=[stage])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(x, p, wl.dt, args.steps, reuse_force=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_end()
    status = ctx.status_sync()
    d1 = ctx.diagnostics(x, p)
    wall = t1 - t0
    value = wl.n * args.steps / wall

    # after the timed region (the float64 kernels draw more power, and the
    # clocks they leave behind would slow what follows): the accuracy of this
    # precision against the float64 path on the same GPU at the initial
    # state, relative rms over all particles and the largest single-particle
    # error against the rms force; then the float64 path's own throughput,
    # a few steps from the initial state with its start force evaluated
    # before the timer
    x = torch.tensor(x0, dtype=torch.float64, device=dev)
    p = torch.tensor(p0, dtype=torch.float64, device=dev)
    f_this = ctx.forces(x)
    ctx64 = p3m.Context.from_workload(wl, precision=p3m.FP64, **ckw)
    f64 = ctx64.forces(x)
    err = float(torch.sqrt(((f_this - f64) ** 2).sum() / (f64 ** 2).sum()))
    err_max = float(torch.linalg.norm(f_this - f64, dim=1).max() / torch.sqrt((f64 ** 2).sum(dim=1).mean()))
    del f_this, f64
    fp64_rate = None
    if args.fp64_steps > 0 and prec != p3m.FP64:
        ctx64.step(x, p, wl.dt, 0)
        torch.cuda.synchronize()
        t64 = time.perf_counter()
        ctx64.step(x, p, wl.dt, args.fp64_steps, reuse_force=True)
        torch.cuda.synchronize()
        fp64_rate = wl.n * args.fp64_steps / (time.perf_counter() - t64)
    del ctx64
    torch.cuda.empty_cache()

    # dominant stage and its roofline, from its launches in the timed region
    ms_tot, launches = prof[stage]
    avg_s = ms_tot / max(launches, 1) * 1e-3
    mesh_nodes = wl.grid[0] * wl.grid[1] * wl.grid[2]
    fbytes = 4 if prec == p3m.FP32C else 8
    mbytes = info["mesh_bits"] // 8
    mdiff = (mbytes == 4 and max(wl.grid) > 128 and args.gather == "variational" and not args.cathode)
    if stage == "pp":
        flops = pairs * PP_FLOP_PER_PAIR
        peak = PEAK_FP32_VALU if prec == p3m.FP32C else PEAK_FP64_VALU
        achieved = flops / avg_s / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak}
    else:
        # compulsory bytes per launch of the stage: the records each kernel must
        # read and write once per particle, PP cell, mesh node and kernel-table entry
        per_stage = {
            # the charge in, the kernel table (mesh precision) and the potential or its
            # three differences out
            "fft": (mbytes * mesh_nodes * (4 if mdiff else 2)
                    + mbytes * (wl.grid[0] + 1) * (wl.grid[1] + 1) * (wl.grid[2] + 1)),
            "sort": 40 * wl.n + 16 * ctx.info()["ncells"],
            "reorder": (4 + 4 + 24 + 2 * 4 * fbytes) * wl.n,
            "deposit": 8 * fbytes * wl.n + mbytes * mesh_nodes,
            # the gather also reads and writes x (the next step's drift, fused)
            "gather": (3 * 4 * fbytes + 4 + 2 * 24 + 24 + 48) * wl.n,
            "push+placement": 48 * ((wl.n + 255) // 256),   # the box partials
        }
        bytes_ = per_stage[stage]
        achieved = bytes_ / avg_s / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS}
    roof["kernel"] = stage
    roof["avg_launch_ms"] = avg_s * 1e3
    if stage == "pp":
        roof["pairs_per_s"] = pairs / avg_s
    roof["traffic"] = traffic_from_profiles(stage, args.workload, args.precision, 1)

    out = {
        "metric": "P3M particle-steps/s at <=1e-5 rms force error vs FP64",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == p3m.FP32C else "f64",
        "data": "synthetic",
        "config": {
            "workload": workload_text(args.workload, wl),
            "precision": ("fp32 pair forces with Kahan sums; fp32 mesh (charge, FFT"
                          + (", three difference meshes" if mdiff else ", potential") + ")"
                          if mbytes == 4 else "fp32 pair forces with Kahan sums; fp64 mesh")
            + "; fp64 kernel table, push, reductions" if prec == p3m.FP32C else "fp64",
            "mesh_bits": info["mesh_bits"],
            "gather": args.gather,
            "boundary": "grounded plane 1 mm below the bunch" if args.cathode else "open",
            "influence": args.influence,
            "pp_cells_per_cutoff": args.pp_cell_div or wl.pp_cell_div,
            "force_rms_err_vs_fp64": err,
            "force_max_particle_err_vs_fp64": err_max,
            "fp64_particle_steps_per_s": fp64_rate,
            "fp64_steps_timed": args.fp64_steps if fp64_rate else 0,
            "zoom_first_last": [d0["zoom"], d1["zoom"]],
            "pairs_per_s_of_step": pairs * args.steps / wall,
            "pairs_per_eval": pairs,
            "pairs_first_last_eval": [d0["pairs"], d1["pairs"]],
            "status": status,
            "stage_ms_per_step": per_launch,
            "stage_ms_from": "replica of the timed trajectory with every stage timed",
            "pp_load_balance": load_balance(waves) if waves is not None else None,
            "pp_load_balance_from": "the pair kernel's waves in the replica's last force evaluation",
        },
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_targets)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
