"""Throughput of the P3M leapfrog step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload aniso1m]
                    [--precision fp32c|fp64] [--cpu-steps 6] [--no-cpu-baseline]

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
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="aniso1m")
    ap.add_argument("--precision", default="fp32c", choices=["fp32c", "fp64"])
    ap.add_argument("--gather", default="variational", choices=["variational", "momentum"],
                    help="mesh force at the particles: variational (default) or momentum-conserving")
    ap.add_argument("--influence", default="sampled", choices=["sampled", "optimal", "principal", "lattice"],
                    help="Fourier table of the mesh kernel (built at create)")
    ap.add_argument("--cathode", action="store_true",
                    help="grounded plane 1 mm below the bunch (image charges on the mesh)")
    ap.add_argument("--cpu-steps", type=int, default=6)
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


def cpu_baseline(wl, steps):
    """The FP64 CPU oracle as it stands, on `steps` leapfrog steps of the same
    workload (the initial force evaluation is not timed)."""
    from oracle import oracle as O
    x, p = wl.draw()
    prm = O.Params.from_workload(wl)
    f = O.forces(x, prm)
    t0 = time.perf_counter()
    O.step(x, p, prm, steps, f)
    t = time.perf_counter() - t0
    return {"value": wl.n * steps / t, "unit": "particle-steps/s", "cores": O.threads(),
            "kind": "oracle",
            "sample": f"{steps} full leapfrog steps of the {wl.n}-particle workload "
                      f"(FP64 C/OpenMP + numpy FFT), {t:.1f} s"}


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
    ctx = p3m.Context.from_workload(wl, precision=prec, gather=gmode, cathode_z=zc, influence=infl)

    # accuracy of this precision against the float64 path on the same GPU
    f_this = ctx.forces(x)
    f64 = p3m.Context.from_workload(wl, precision=p3m.FP64, gather=gmode, cathode_z=zc,
                                    influence=infl).forces(x)
    err = float(torch.sqrt(((f_this - f64) ** 2).sum() / (f64 ** 2).sum()))
    d0 = ctx.diagnostics(x, p)

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
    while done < args.steps:
        k = min(10, args.steps - done)
        ctx.profile_begin(8 * (k + 2))
        ctx.step(xr, pr, wl.dt, k)
        for s_, (ms_, cnt_) in ctx.profile_end().items():
            stage_ms[s_] += ms_
            stage_n[s_] += cnt_
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

    # dominant stage and its roofline, from its launches in the timed region
    ms_tot, launches = prof[stage]
    avg_s = ms_tot / max(launches, 1) * 1e-3
    mesh_nodes = wl.grid[0] * wl.grid[1] * wl.grid[2]
    fbytes = 4 if prec == p3m.FP32C else 8
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
            "fft": 2 * fbytes * mesh_nodes + 8 * (wl.grid[0] + 1) * (wl.grid[1] + 1) * (wl.grid[2] + 1),
            "sort": 40 * wl.n + 16 * ctx.info()["ncells"],
            "reorder": (4 + 4 + 24 + 2 * 4 * fbytes) * wl.n,
            "deposit": 8 * fbytes * wl.n + fbytes * mesh_nodes,
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
            "workload": f"{args.workload}: {wl.n} particles, Gaussian sigma (1,1,3) mm, "
                        f"{wl.grid[0]}^3 mesh ({2 * wl.grid[0]}^3 zero-padded FFT), "
                        f"{'TSC' if wl.order == 2 else 'CIC'}, r_c = 2 h_x, kappa = 3, dt = T_p/200"
            if args.workload == "aniso1m" else args.workload,
            "precision": "fp32 pair forces and FFT with Kahan sums; fp64 table, push, reductions"
            if prec == p3m.FP32C else "fp64",
            "gather": args.gather,
            "boundary": "grounded plane 1 mm below the bunch" if args.cathode else "open",
            "influence": args.influence,
            "force_rms_err_vs_fp64": err,
            "pairs_per_s_of_step": pairs * args.steps / wall,
            "pairs_per_eval": pairs,
            "pairs_first_last_eval": [d0["pairs"], d1["pairs"]],
            "status": status,
            "stage_ms_per_step": per_launch,
            "stage_ms_from": "replica of the timed trajectory with every stage timed",
        },
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
