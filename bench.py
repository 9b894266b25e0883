"""Benchmark: rays/s of the full hot path (camera, DP RK5(4) Kerr geodesics,
sampling, thermal synchrotron coefficients, polarized transfer) on one GPU.

One step = one bl_render of the workload image with the grid already resident
in HBM.  Prints one JSON line.  Kernel durations come from HIP events the
library records around its own launches on its stream.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6   # MI355X dense FP64 vector: 256 CU x 2.4 GHz x 128 FLOP/clk

# Algorithmic FP64 operations per unit of work (per-unit figures stated with
# their derivation in the design notes):
FLOP_PER_TRIAL_STEP = 1800.0      # one Dormand-Prince trial: 6 RHS + stage sums + norm
FLOP_PER_RECORD = 2000.0          # polarized transport of one record (2 connections, 2 RHS of N)
FLOP_PER_SAMPLE_POL = 2500.0      # coefficients, tetrad, projections, exact Stokes step
FLOP_PER_SAMPLE_UNPOL = 600.0     # coefficients (I only) and the segment solution


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_baseline(w, grid, budget_s=15.0, seed=0):
    """The CPU oracle on a random pixel sample of the same workload, timed for
    about budget_s seconds on the host cores; returns rays/s."""
    import numpy as np
    from oracle import oracle as O
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    n = int(w["camera"]["n"])
    rng = np.random.default_rng(seed)
    gh = O.grid(grid)
    done, t_used, batch = 0, 0.0, max(16, cores * 4)
    while t_used < budget_s:
        pix = rng.choice(n * n, size=batch, replace=False)
        t0 = time.perf_counter()
        O.render_pixels(w["camera"], w["spacetime"], w["integrator"], gh, w["plasma"], pix, n_threads=cores)
        dt = time.perf_counter() - t0
        done += batch
        t_used += dt
        if dt < budget_s / 8:
            batch *= 2
    return {"value": done / t_used, "unit": "rays/s", "cores": cores, "kind": "oracle",
            "sample": f"{done} random pixels of the same {n}x{n} image (seed {seed}), {t_used:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3_1024_smr")
    ap.add_argument("--precision", type=int, default=0)
    ap.add_argument("--n", type=int, default=None, help="override the image size")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a 1 GiB device-to-device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(pixels are independent; see the design notes for how the image would shard)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2203_15963_amd import blgpu, synth

    w = synth.workload(args.workload, n=args.n)
    n = int(w["camera"]["n"])
    log("generating grid", w["grid_args"])
    grid = synth.make_grid(w["grid_args"])
    ctx = blgpu.Context(0)
    gg = ctx.grid(grid)
    img = torch.empty(4, n, n, dtype=torch.float64, device="cuda")
    aux = torch.empty(blgpu.NAUX, n, n, dtype=torch.float64, device="cuda")
    log("grid resident:", grid["prims"].nbytes / 1e6, "MB;", len(grid["bounds"]), "blocks")

    def step():
        ctx.render(w["camera"], w["spacetime"], w["integrator"], gg, w["plasma"], precision=args.precision,
                   image=img, aux=aux)

    for k in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup {k + 1}/{args.warmup} done")
    ctx.profile_enable(True)
    ctx.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    log("timed steps done", prof)
    ms = (t1 - t0) * 1e3 / args.steps
    rays = n * n
    value = rays / (ms / 1e3)

    a = aux.cpu().numpy()
    n_trial = float(a[5].sum() + a[6].sum())
    n_samp = float(a[8].sum())
    n_rec = float(a[9].sum())
    pol = bool(w["plasma"]["polarized"])
    f_geo = FLOP_PER_TRIAL_STEP * n_trial
    f_tr = (FLOP_PER_RECORD * n_rec + FLOP_PER_SAMPLE_POL * n_samp) if pol else FLOP_PER_SAMPLE_UNPOL * n_samp
    kern = {}
    for name, (tot, nl) in prof.items():
        kern[name] = {"ms_per_step": tot / args.steps, "launches_per_step": nl / args.steps,
                      "avg_launch_ms": (tot / nl) if nl else 0.0}
    # dominant kernel: largest share of the step
    dom = max(("geodesic", "transfer"), key=lambda k: kern[k]["ms_per_step"])
    flops_step = f_geo if dom == "geodesic" else f_tr
    per_launch = flops_step / max(1.0, kern[dom]["launches_per_step"])
    achieved = per_launch / (kern[dom]["avg_launch_ms"] / 1e3) / 1e12
    roof = {"bound": "alu", "kernel": "k_" + dom, "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None,
            "flop_per_launch": per_launch,
            "units_per_step": {"trial_steps": n_trial, "records": n_rec, "plasma_samples": n_samp}}
    out = {
        "metric": "rays/sec at 1024² (geodesic+polarized transfer) at ≤1e-4 rel. error vs FP64 oracle",
        "value": value, "unit": "rays/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == 0 else "f64+f32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {n}x{n} pixels, spin {w['spacetime']['a']}, "
                               f"inclination {math.degrees(w['camera']['theta']):.0f} deg, "
                               f"{'polarized' if pol else 'unpolarized'}, {len(grid['bounds'])} blocks of "
                               f"{grid['prims'].shape[1]}^3 cells, f_abs=f_rel={w['integrator']['f_abs']}",
                   "precision": args.precision, "pixels": rays},
        "kernels": kern,
        "roofline": roof,
    }
    if args.copy_probe:
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy probe: 1 GiB read + 1 GiB written")
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(w, grid, budget_s=args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
