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

# MI355X vector ALU peak: 256 CU x 2.4 GHz x 4 SIMD x 16 lanes x 2 (FMA) =
# 78.6 TFLOP/s for FP64 and for unpacked FP32 alike.  The published FP32
# figure of 157.3 TFLOP/s counts packed dual FP32 (v_pk_fma_f32), which this
# build disables (-packed-fp32-ops), so 78.6 is the attainable ceiling of both
# arithmetic types here.  Transcendental-unit instructions are counted as one
# operation although they issue at a quarter of the rate, which makes the
# ceiling generous to the hardware.
VALU_PEAK_TFLOPS = 78.6
PUBLISHED_FP32_TFLOPS = 157.3

# Floating-point operations per unit of work, measured on divergence-free
# launches (paper_2203_15963_amd/opcount.py: 64 copies of one ray per wave,
# FMA = 2, add/mul/transcendental = 1, non-negative least squares over 48
# directions): the work the kernels do per unit with every lane useful.  Valid
# only for the kernel sources and flags they were measured on (hash "src").
# Keys: precision -> kernel -> arithmetic type -> unit; units: trial = DP trial
# steps, acc = accepted steps, samp = plasma samples, rec = transport records
# (pieces), ray = rays.
OPS_PER_UNIT = {
    "src": "462cdab4655cc8ef",
    0: {"geodesic": {"F64": {"trial": 1291.6, "acc": 287.4, "ray": 1055.3}, "F32": {"trial": 11.0, "ray": 7.0}},
        "transfer": {"F64": {"samp": 2506.7, "rec": 366.8, "acc": 52.2, "ray": 36330.1}, "F32": {}}},
    1: {"geodesic": {"F64": {"trial": 1216.5, "acc": 424.2, "ray": 5321.1}, "F32": {"trial": 11.0, "ray": 7.0}},
        "transfer": {"F64": {"samp": 16.0, "rec": 30.8}, "F32": {"samp": 1481.5, "rec": 353.4, "ray": 50629.5}}},
}

# Counter passes over this benchmark (rocprofv3), per launch of a kernel, for
# the sources whose hash is "src": issued floating-point operations
# (SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_{F32,F64} x 64 lanes, FMA = 2: masked
# lanes included), VALU lane activity (SQ_THREAD_CYCLES_VALU over 64 x
# SQ_ACTIVE_INST_VALU) and HBM bytes of the transfer and the k_finish launch
# that follows it (FETCH_SIZE and WRITE_SIZE in KiB per dispatch, scaled by
# what the same counters read for a 1 GiB device copy: x2.0 and x1.0).  Keys:
# (precision, kernel class).
_UNITS_1024_SMR = {"trial": 85456054.0, "acc": 72527214.0, "samp": 682634999.0, "rec": 734227814.0,
                   "ray": 1048576.0}
COUNTERS = {
    "src": "462cdab4655cc8ef",
    (1, "transfer"): {"issued_f64": 4.608e+10, "issued_f32": 1.536e+12, "lane_activity": 0.855,
                      "bytes": 2.0 * (14071833.3 + 203358.3) * 1024 + 1.0 * (138002.8 + 65536.0) * 1024,
                      # units of work of that launch (1024^2 SMR image, auxiliary maps)
                      "units": _UNITS_1024_SMR},
    (0, "transfer"): {"issued_f64": 2.427e+12, "issued_f32": 0, "lane_activity": 0.785,
                      "bytes": 2.0 * (16733861.8 + 266234.6) * 1024 + 1.0 * (269202.7 + 65536.0) * 1024,
                      "units": _UNITS_1024_SMR},
}


def source_hash():
    """Hash over the device code of the render kernels (the headers and the
    kernel part of blgpu.hip, which ends where its host side begins;
    comments and blank space removed, so that only code changes count) and
    the library's build flags."""
    import hashlib
    import re
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2203_15963_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".hpp", ".h")):
            with open(os.path.join(d, f)) as fh:
                text = fh.read()
            if f.endswith(".hip"):
                text = text.split("// ============================================================ host side")[0]
            text = re.sub(r"^#include <[^>]*>", " ", text, flags=re.M)   # standard headers
            code = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
            code = re.sub(r"//[^\n]*", " ", code)
            h.update(f.encode() + b"\0" + " ".join(code.split()).encode())
    from paper_2203_15963_amd import build as libbuild
    h.update(" ".join(libbuild.FLAGS[:-2]).encode())
    return h.hexdigest()[:16]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(w, grid, budget_s=20.0, seed=0):
    """The CPU oracle timed on random pixel samples of the same workload: a
    short calibration, then three runs on every host core this process may
    use (their median is the value) and one run on one thread, each sized to
    about a quarter of budget_s.  Returns the baseline record and the oracle's
    pixels (ids, image rows, aux rows) for the accuracy check."""
    import numpy as np
    from oracle import oracle as O
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    n = int(w["camera"]["n"])
    rng = np.random.default_rng(seed)
    gh = O.grid(grid)
    pix_all, io_all, ao_all = [], [], []

    def timed(m, threads):
        pix = rng.choice(n * n, size=min(m, n * n), replace=False)
        t0 = time.perf_counter()
        io, ao = O.render_pixels(w["camera"], w["spacetime"], w["integrator"], gh, w["plasma"], pix,
                                 n_threads=threads)
        dt = time.perf_counter() - t0
        pix_all.append(pix)
        io_all.append(io)
        ao_all.append(ao)
        return len(pix) / dt, dt, len(pix)

    rate, _, _ = timed(4 * cores, cores)
    per_run = budget_s / 4.0
    runs, secs, npx = [], 0.0, 0
    for _ in range(3):
        r, dt, m = timed(max(cores, int(rate * per_run)), cores)
        runs.append(r)
        secs += dt
        npx += m
        rate = r
    r1, dt1, m1 = timed(max(4, int(rate / cores * per_run)), 1)
    value = float(np.median(runs))
    rec = {"value": value, "unit": "rays/s", "cores": cores, "kind": "oracle", "cpu": cpu_model(),
           "runs": runs, "one_thread": {"value": r1, "pixels": m1, "seconds": dt1},
           "sample": f"3 runs of {npx // 3} random pixels of the same {n}x{n} image on {cores} threads "
                     f"(median), {secs:.1f} s; one run of {m1} pixels on 1 thread, {dt1:.1f} s"}
    return rec, np.concatenate(pix_all), np.concatenate(io_all), np.concatenate(ao_all)


def accuracy(img, aux, pix, io, ao, tol):
    """Error of the timed GPU image against the FP64 oracle on the oracle's
    pixels: E_pix = max over Stokes of |X_gpu - X_oracle| / max(I_oracle,
    1e-3 max I) per pixel (max I over the GPU image), its distribution, the
    relative error of the sample's total flux and the pixels whose accepted or
    rejected step counts differ from the oracle's."""
    import numpy as np
    pix, first = np.unique(pix, return_index=True)
    io, ao = io[first], ao[first]
    ig = img.reshape(4, -1)[:, pix].T
    ag = aux.reshape(aux.shape[0], -1)[:, pix].T
    den = np.maximum(np.abs(io[:, 0]), 1e-3 * np.abs(img[0]).max())
    e = (np.abs(ig - io) / den[:, None]).max(axis=1)
    match = (ag[:, 5] == ao[:, 5]) & (ag[:, 6] == ao[:, 6])
    return {"pixels": int(len(pix)), "E_pix_max": float(e.max()), "E_pix_p999": float(np.quantile(e, 0.999)),
            "E_pix_p99": float(np.quantile(e, 0.99)), "E_pix_median": float(np.median(e)),
            "E_pix_rms": float(np.sqrt(np.mean(e * e))),
            "flux_rel_err": float(abs(ig[:, 0].sum() - io[:, 0].sum()) / abs(io[:, 0].sum())),
            "step_count_mismatches": int((~match).sum()),
            "E_pix_max_mismatched": float(e[~match].max()) if (~match).any() else None,
            "tolerance": tol, "within_tolerance": bool(e.max() <= tol)}


def roofline(precision, dom, kern, units):
    """Useful FLOP/s of the dominant kernel against the VALU ceiling, with the
    counters' issued operations and HBM bytes beside it."""
    lm = kern[dom]["avg_launch_ms"] / 1e3
    nl = max(1.0, kern[dom]["launches_per_step"])
    src = source_hash()
    out = {"bound": "alu", "kernel": "k_" + dom, "achieved": None, "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
           "frac": None, "traffic": None, "traffic_unit": "bytes/launch",
           "peak_note": f"{VALU_PEAK_TFLOPS} TFLOP/s = 256 CU x 2.4 GHz x 128 FLOP/clk: FP64 and unpacked FP32 "
                        f"(packed FP32, the published {PUBLISHED_FP32_TFLOPS}, is disabled in this build)",
           "units_per_step": units, "source_hash": src}
    if OPS_PER_UNIT["src"] == src:
        model = OPS_PER_UNIT[precision][dom]
        ops = {t: sum(c * units[u] for u, c in model[t].items()) / nl for t in ("F64", "F32")}
        useful = ops["F64"] + ops["F32"]
        out["achieved"] = useful / lm / 1e12
        out["frac"] = out["achieved"] / VALU_PEAK_TFLOPS
        out["ops_per_launch"] = {"f64": ops["F64"], "f32": ops["F32"]}
    else:
        out["stale"] = "per-unit operation counts were measured on other kernel sources"
    cn = COUNTERS.get((precision, dom)) if COUNTERS["src"] == src else None
    if cn is not None:
        issued = cn["issued_f64"] + cn["issued_f32"]
        out["issued"] = {"tflops": issued / lm / 1e12, "frac": issued / lm / 1e12 / VALU_PEAK_TFLOPS,
                         "f64_per_launch": cn["issued_f64"], "f32_per_launch": cn["issued_f32"],
                         "lane_activity": cn["lane_activity"]}
        out["traffic"] = cn["bytes"]
        if out["achieved"] is not None:
            out["useful_over_issued"] = out["achieved"] / out["issued"]["tflops"]
    return out


def kernel_table(prof, steps):
    return {name: {"ms_per_step": tot / steps, "launches_per_step": nl / steps,
                   "avg_launch_ms": (tot / nl) if nl else 0.0} for name, (tot, nl) in prof.items()}


def run_batch(args):
    """64 images of uneven size, frequency, inclination and spin on one grid:
    one batched render per step (autotuned schedule) against one bl_render
    per image with the same schedule."""
    import numpy as np
    import torch
    from paper_2203_15963_amd import blgpu, synth

    bw = synth.batch_workload()
    grid_f32 = args.precision == 1 and not args.grid_f64
    grid = synth.make_grid(bw["grid_args"], dtype=np.float32 if grid_f32 else np.float64)
    ctx = blgpu.Context(0)
    gg = ctx.grid(grid)
    imgs = bw["images"]
    rays = sum(int(c["n"]) ** 2 for c, _ in imgs)
    outs = [(torch.empty(4, c["n"], c["n"], dtype=torch.float64, device="cuda"),
             torch.empty(blgpu.NAUX, c["n"], c["n"], dtype=torch.float64, device="cuda")) for c, _ in imgs]
    log(f"{len(imgs)} images, {rays} rays")
    tuning = ctx.get_tuning()
    tune_ms = None
    if not args.no_autotune:
        tuning, tune_ms = ctx.autotune(imgs, bw["integrator"], gg, bw["plasma"], precision=args.precision,
                                       max_trials=args.tune_trials, outputs=outs)
        log("autotuned", tuning, f"{tune_ms:.1f} ms")

    def batched():
        ctx.render_batch(imgs, bw["integrator"], gg, bw["plasma"], precision=args.precision, outputs=outs)

    def per_image():
        for (cam, st), (im, ax) in zip(imgs, outs):
            ctx.render(cam, st, bw["integrator"], gg, bw["plasma"], precision=args.precision, image=im, aux=ax)

    res = {}
    for name, fn in (("per_image", per_image), ("batched", batched)):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        ctx.profile_enable(True)
        ctx.profile_read()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        prof = ctx.profile_read()
        ctx.profile_enable(False)
        res[name] = ((t1 - t0) * 1e3 / args.steps, kernel_table(prof, args.steps))
        log(name, f"{res[name][0]:.2f} ms per batch")
    ms, kern = res["batched"]
    units = {"trial": 0.0, "acc": 0.0, "samp": 0.0, "rec": 0.0, "ray": float(rays)}
    for _, ax in outs:
        x = ax.cpu().numpy()
        units["trial"] += float(x[5].sum() + x[6].sum())
        units["acc"] += float(x[5].sum())
        units["samp"] += float(x[8].sum())
        units["rec"] += float(x[9].sum())
    dom = max(("geodesic", "transfer"), key=lambda k: kern[k]["ms_per_step"])
    out = {
        "metric": "rays/sec of a 64-image batch (geodesic+polarized transfer), one batched launch sequence",
        "value": rays / (ms / 1e3), "unit": "rays/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == 0 else "f64+f32", "data": "synthetic",
        "config": {"workload": f"c4_batch64: {len(imgs)} images of 64^2 to 512^2 pixels ({rays} rays), "
                               "86-690 GHz, inclinations 17-90 deg, spins 0-0.98, shared 128^3 grid, polarized",
                   "precision": args.precision, "grid_dtype": "f32" if grid_f32 else "f64", "pixels": rays},
        "per_image_launches": {"ms_per_step": res["per_image"][0], "value": rays / (res["per_image"][0] / 1e3)},
        "batch_speedup": res["per_image"][0] / ms,
        "tuning": tuning, "autotune_ms": tune_ms,
        "kernels": kern,
        "roofline": roofline(args.precision, dom, kern, units),
    }
    print(json.dumps(out), flush=True)


def run_learned(args):
    """Learned step proposals on the single-image workload: log the plain
    integrator over 128 random cameras (spin U[0, 0.98], cos inclination
    U[0, 1], 32^2 pixels each), train the network on the GPU (untimed), then
    time renders with learned proposals and with the plain controller."""
    import numpy as np
    import torch
    from paper_2203_15963_amd import blgpu, learned, synth

    w = synth.workload(args.workload, n=args.n)
    n = int(w["camera"]["n"])
    grid_f32 = args.precision == 1 and not args.grid_f64
    grid64 = synth.make_grid(w["grid_args"], dtype=np.float64)
    grid = dict(grid64, prims=grid64["prims"].astype(np.float32)) if grid_f32 else grid64
    ctx = blgpu.Context(0)
    gg = ctx.grid(grid)
    t0 = time.perf_counter()
    model, losses, n_steps, rec = learned.train_step_model(ctx, n_images=128, n=32, seed=3, epochs=args.epochs,
                                                           batch=16384)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    losses = losses.cpu().numpy()
    log(f"logged {n_steps} steps, trained in {t_train:.1f} s, losses {losses.tolist()}")
    del rec
    ctx.set_step_model(model)
    res = {}
    K = args.step_model   # the network proposes after every K-th accepted step
    for sm in (0, K):
        img = torch.empty(4, n, n, dtype=torch.float64, device="cuda")
        aux = torch.empty(blgpu.NAUX, n, n, dtype=torch.float64, device="cuda")

        def step():
            ctx.render(w["camera"], w["spacetime"], w["integrator"], gg, w["plasma"], precision=args.precision,
                       image=img, aux=aux, step_model=sm)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        ctx.profile_enable(True)
        ctx.profile_read()
        ta = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        tb = time.perf_counter()
        prof = ctx.profile_read()
        ctx.profile_enable(False)
        a = aux.cpu().numpy()
        res[sm] = {"ms": (tb - ta) * 1e3 / args.steps, "kern": kernel_table(prof, args.steps),
                   "img": img.cpu().numpy(), "acc": float(a[5].mean()), "rej": float(a[6].mean()),
                   "units": {"trial": float(a[5].sum() + a[6].sum()), "acc": float(a[5].sum()),
                             "samp": float(a[8].sum()), "rec": float(a[9].sum()), "ray": float(n * n)}}
        log("step_model", sm, f"{res[sm]['ms']:.2f} ms")
    il, ip = res[K]["img"], res[0]["img"]
    den = np.maximum(np.abs(ip[0]), 1e-3 * np.abs(ip[0]).max())
    diff = {"E_pix": float((np.abs(il - ip) / den).max()),
            "L1_I": float(np.abs(il[0] - ip[0]).sum() / np.abs(ip[0]).sum())}

    vs_oracle = None
    if not args.no_cpu_baseline:
        # equal image accuracy: both images against a converged FP64 oracle
        # (sampling limit ds_max/4) on sampled pixels
        from oracle import oracle as O
        rng = np.random.default_rng(5)
        pix = rng.choice(n * n, size=min(n * n, 192), replace=False)
        fine = dict(w["integrator"], ds_max=w["integrator"]["ds_max"] / 4)
        log("converged oracle on", len(pix), "pixels ...")
        iref, _ = O.render_pixels(w["camera"], w["spacetime"], fine, O.grid(grid64), w["plasma"], pix)
        floor = 1e-3 * np.abs(ip[0]).max()
        den = np.maximum(np.abs(iref[:, 0]), floor)
        vs_oracle = {"reference": f"FP64 oracle with ds_max/4 on {len(pix)} random pixels (FP64 cells)"}
        for name, im in (("learned", il), ("plain", ip)):
            x = im.reshape(4, -1)[:, pix].T
            vs_oracle[name] = {"E_pix": float((np.abs(x - iref) / den[:, None]).max()),
                               "L1_I": float(np.abs(x[:, 0] - iref[:, 0]).sum() / np.abs(iref[:, 0]).sum())}

    def summary(r):
        return {"rays_per_s": n * n / (r["ms"] / 1e3), "ms_per_step": r["ms"],
                "rejected_fraction": r["rej"] / (r["acc"] + r["rej"]), "accepted_per_ray": r["acc"],
                "trials_per_ray": r["acc"] + r["rej"],
                "geodesic_ms_per_step": r["kern"]["geodesic"]["ms_per_step"],
                "transfer_ms_per_step": r["kern"]["transfer"]["ms_per_step"]}

    out = {
        "metric": "rays/sec at 1024² (geodesic+polarized transfer) with learned step proposals",
        "value": n * n / (res[K]["ms"] / 1e3), "unit": "rays/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res[K]["ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64+f32+bf16" if args.precision == 1 else "f64+bf16", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {n}x{n} pixels with learned step proposals (MLP 11-64-64-64-1, "
                               f"BF16 on the matrix cores, proposing after every {K}-th accepted step)", "precision": args.precision,
                   "grid_dtype": "f32" if grid_f32 else "f64", "pixels": n * n},
        "learned": summary(res[K]), "plain": summary(res[0]),
        "speedup_vs_plain": res[0]["ms"] / res[K]["ms"],
        "image_difference_learned_vs_plain": diff,
        "image_error_vs_converged_oracle": vs_oracle,
        "training": {"logged_steps": n_steps, "epochs": args.epochs, "seconds": t_train,
                     "loss_train_heldout": losses.tolist()},
        "kernels": res[K]["kern"],
        "roofline": roofline(args.precision, "transfer", res[K]["kern"], res[K]["units"]),
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3_1024_smr")
    ap.add_argument("--precision", type=int, default=1,
                    help="1 = mixed (FP64 geodesics, FP32 grid, coefficients and transfer; the default), "
                         "0 = plain FP64")
    ap.add_argument("--grid-f64", action="store_true", help="keep the grid in FP64 in the mixed form")
    ap.add_argument("--n", type=int, default=None, help="override the image size")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-autotune", action="store_true", help="batched workload: keep the default schedule")
    ap.add_argument("--autotune", action="store_true", help="single image: autotune the schedule first (untimed)")
    ap.add_argument("--tuning", default=None, help="schedule as JSON, e.g. '{\"tile_w\": 8, \"tile_h\": 8}'")
    ap.add_argument("--tune-trials", type=int, default=14)
    ap.add_argument("--step-model", type=int, default=0,
                    help="K >= 1: learned step proposals (trains the network first), the network proposing for "
                         "the first step and after every K-th accepted one")
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--freqs", type=int, default=0,
                    help="single image: also time a K-frequency render from one geodesic pass (K frequencies "
                         "evenly spaced in wavelength over 152-324 GHz, as for true-colour images)")
    ap.add_argument("--models", type=int, default=0,
                    help="single image: also time K electron-temperature models (R_high from 1 to 160, evenly "
                         "spaced in log) rendered from one geodesic pass (bl_render_models)")
    ap.add_argument("--nonthermal", action="store_true",
                    help="single image: also time a render with thermal, power-law and kappa electrons in equal "
                         "thirds (p = 3, gamma 4..1000; kappa = 4, w = 1/2)")
    ap.add_argument("--averages", action="store_true",
                    help="single image: also time a render with the 21 averaged-quantity maps (bl_render_averages)")
    ap.add_argument("--adaptive", action="store_true",
                    help="single image: also time an adaptive render of the same camera (root N/4 in 8x8 blocks, "
                         "two refinement levels up to N, absolute-gradient criterion)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a 1 GiB device-to-device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(pixels are independent; see the design notes for how the image would shard)",
              file=sys.stderr)
        sys.exit(2)
    if args.workload.startswith("c4"):
        run_batch(args)
        return
    if args.step_model >= 1:
        run_learned(args)
        return

    import numpy as np
    import torch
    from paper_2203_15963_amd import blgpu, synth

    w = synth.workload(args.workload, n=args.n)
    n = int(w["camera"]["n"])
    log("generating grid", w["grid_args"])
    grid_f32 = args.precision == 1 and not args.grid_f64
    # the FP64 cells are the oracle's input; the mixed form stores them rounded to FP32
    grid64 = synth.make_grid(w["grid_args"], dtype=np.float64)
    grid = dict(grid64, prims=grid64["prims"].astype(np.float32)) if grid_f32 else grid64
    ctx = blgpu.Context(0)
    torch.cuda.synchronize()
    te0 = time.perf_counter()
    gg = ctx.grid(grid)
    torch.cuda.synchronize()
    grid_ms = (time.perf_counter() - te0) * 1e3
    img = torch.empty(4, n, n, dtype=torch.float64, device="cuda")
    aux = torch.empty(blgpu.NAUX, n, n, dtype=torch.float64, device="cuda")
    log("grid resident:", grid["prims"].nbytes / 1e6, "MB;", len(grid["bounds"]), "blocks")

    if args.tuning:
        ctx.set_tuning(json.loads(args.tuning))
    tune_ms = None
    if args.autotune:
        _, tune_ms = ctx.autotune([(w["camera"], w["spacetime"])], w["integrator"], gg, w["plasma"],
                                  precision=args.precision, max_trials=args.tune_trials, outputs=[(img, aux)])
        log("autotuned", ctx.get_tuning(), f"{tune_ms:.1f} ms")

    def step():
        ctx.render(w["camera"], w["spacetime"], w["integrator"], gg, w["plasma"], precision=args.precision,
                   image=img, aux=aux)

    for k in range(args.warmup):
        te0 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        if k == 0:
            first_ms = (time.perf_counter() - te0) * 1e3
        log(f"warmup {k + 1}/{args.warmup} done")
    ctx.profile_enable(True)
    ctx.profile_read()
    # per-step HIP events on the stream the library enqueues on (torch's current stream)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        evs[k][0].record()
        step()
        evs[k][1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    log("timed steps done", prof)
    ms = (t1 - t0) * 1e3 / args.steps
    step_ms = sorted(a.elapsed_time(b) for a, b in evs)
    rays = n * n
    value = rays / (ms / 1e3)

    a = aux.cpu().numpy()
    units = {"trial": float(a[5].sum() + a[6].sum()), "acc": float(a[5].sum()), "samp": float(a[8].sum()),
             "rec": float(a[9].sum()), "ray": float(rays)}
    pol = bool(w["plasma"]["polarized"])
    kern = kernel_table(prof, args.steps)
    # dominant kernel: largest share of the step
    dom = max(("geodesic", "transfer"), key=lambda k: kern[k]["ms_per_step"])
    roof = roofline(args.precision, dom, kern, units)
    out = {
        "metric": "rays/sec at 1024² (geodesic+polarized transfer) at ≤1e-4 rel. error vs FP64 oracle",
        "value": value, "unit": "rays/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == 0 else "f64+f32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {n}x{n} pixels, spin {w['spacetime']['a']}, "
                               f"inclination {math.degrees(w['camera']['theta']):.0f} deg, "
                               f"{'polarized' if pol else 'unpolarized'}, {len(grid['bounds'])} blocks of "
                               f"{grid['prims'].shape[1]}^3 cells, f_abs=f_rel={w['integrator']['f_abs']}",
                   "precision": args.precision, "grid_dtype": "f32" if grid_f32 else "f64", "pixels": rays},
        "step_ms": {"median": step_ms[len(step_ms) // 2], "min": step_ms[0], "max": step_ms[-1],
                    "timer": "HIP events around each render on the library's stream"},
        "end_to_end_ms": {"grid_create": grid_ms, "first_render": first_ms if args.warmup > 0 else None,
                          "note": "host-to-device copy of the cells and bl_grid_create; the first render "
                                  "includes the workspace allocation"},
        "tuning": ctx.get_tuning(),
        "kernels": kern,
        "roofline": roof,
    }
    if args.freqs > 1:
        K = args.freqs
        lam = [1.0 / 324e9 + (1.0 / 152e9 - 1.0 / 324e9) * k / (K - 1) for k in range(K)]
        nus = [1.0 / v for v in lam]
        outs = [(torch.empty(4, n, n, dtype=torch.float64, device="cuda"),
                 torch.empty(blgpu.NAUX, n, n, dtype=torch.float64, device="cuda")) for _ in range(K)]

        def mstep():
            ctx.render_multifreq(w["camera"], w["spacetime"], w["integrator"], gg, w["plasma"], nus,
                                 precision=args.precision, outputs=outs)

        mstep()
        torch.cuda.synchronize()
        log(f"multi-frequency warmup done ({K} frequencies)")
        ctx.profile_enable(True)
        ctx.profile_read()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            mstep()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        mprof = ctx.profile_read()
        ctx.profile_enable(False)
        mms = (t1 - t0) * 1e3 / args.steps
        out["multifreq"] = {"n_freq": K, "nu_hz": nus, "ms_per_render": mms, "ms_per_image": mms / K,
                            "images_per_s": K / (mms / 1e3), "rays_per_s": K * rays / (mms / 1e3),
                            "single_frequency_ms": ms, "speedup_vs_separate_renders": K * ms / mms,
                            "kernels": kernel_table(mprof, args.steps)}
        log("multi-frequency", out["multifreq"]["ms_per_render"], "ms per render of", K, "frequencies")
    if args.models > 1:
        K = args.models
        rhs = [math.exp(math.log(160.0) * k / (K - 1)) for k in range(K)]
        pls = [dict(w["plasma"], r_high=rh) for rh in rhs]
        outs = [(torch.empty(4, n, n, dtype=torch.float64, device="cuda"),
                 torch.empty(blgpu.NAUX, n, n, dtype=torch.float64, device="cuda")) for _ in range(K)]

        def mdstep():
            ctx.render_models(w["camera"], w["spacetime"], w["integrator"], gg, pls, precision=args.precision,
                              outputs=outs)

        mdstep()
        torch.cuda.synchronize()
        ctx.profile_enable(True)
        ctx.profile_read()
        t0 = time.perf_counter()
        for k in range(args.steps):
            mdstep()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        mdprof = ctx.profile_read()
        ctx.profile_enable(False)
        mdms = (t1 - t0) * 1e3 / args.steps
        out["models"] = {"n_models": K, "r_high": rhs, "ms_per_render": mdms, "ms_per_image": mdms / K,
                         "rays_per_s": K * rays / (mdms / 1e3), "single_model_ms": ms,
                         "speedup_vs_separate_renders": K * ms / mdms, "kernels": kernel_table(mdprof, args.steps)}
        log("models", mdms, "ms per render of", K, "electron models")
    if args.nonthermal:
        pl_nt = dict(w["plasma"], fractions=(1 / 3, 1 / 3, 1 / 3))

        def ntstep():
            return ctx.render(w["camera"], w["spacetime"], w["integrator"], gg, pl_nt, precision=args.precision)

        ntstep()
        torch.cuda.synchronize()
        ctx.profile_enable(True)
        ctx.profile_read()
        t0 = time.perf_counter()
        for k in range(args.steps):
            ntstep()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ntprof = ctx.profile_read()
        ctx.profile_enable(False)
        ntms = (t1 - t0) * 1e3 / args.steps
        out["nonthermal"] = {"fractions": [1 / 3, 1 / 3, 1 / 3], "ms_per_render": ntms,
                             "rays_per_s": rays / (ntms / 1e3), "thermal_render_ms": ms,
                             "kernels": kernel_table(ntprof, args.steps)}
        log("nonthermal", ntms, "ms per render (equal thirds)")
    if args.averages:
        def astep():
            return ctx.render_averages(w["camera"], w["spacetime"], w["integrator"], gg, w["plasma"],
                                       precision=args.precision)

        astep()
        torch.cuda.synchronize()
        ctx.profile_enable(True)
        ctx.profile_read()
        t0 = time.perf_counter()
        for k in range(args.steps):
            astep()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        aprof = ctx.profile_read()
        ctx.profile_enable(False)
        ams = (t1 - t0) * 1e3 / args.steps
        out["averages"] = {"ms_per_render": ams, "single_render_ms": ms, "extra_ms": ams - ms,
                           "kernels": kernel_table(aprof, args.steps)}
        log("averages", ams, "ms per render with the 21 maps")
    if args.adaptive:
        n = int(w["camera"]["n"])
        cam0 = dict(w["camera"], n=n // 4)
        i0, _ = ctx.render(cam0, w["spacetime"], w["integrator"], gg, w["plasma"], precision=args.precision)
        thr = 0.02 * float(i0[0].max())
        ad = dict(block=8, max_level=2, frac=5 / 64, thr=[None, thr, None, None, None])

        def adstep():
            return ctx.render_adaptive(cam0, w["spacetime"], w["integrator"], gg, w["plasma"], ad,
                                       precision=args.precision)

        counts = [len(l[0]) for l in adstep()]
        torch.cuda.synchronize()
        ctx.profile_enable(True)
        ctx.profile_read()
        t0 = time.perf_counter()
        for k in range(args.steps):
            adstep()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        dprof = ctx.profile_read()
        ctx.profile_enable(False)
        dms = (t1 - t0) * 1e3 / args.steps
        arays = 64 * sum(counts)
        out["adaptive"] = {"root_n": n // 4, "block": 8, "max_level": 2, "finest_n": n,
                           "criterion": "|grad I|_abs > 0.02 max(I_root) in at least 5 of a block's 64 pixels",
                           "threshold": thr, "blocks_per_level": counts, "rays": arays,
                           "ms_per_render": dms, "rays_per_s": arays / (dms / 1e3),
                           "uniform_finest_ms": ms, "uniform_finest_rays": n * n,
                           "speedup_vs_uniform_finest": ms / dms, "kernels": kernel_table(dprof, args.steps)}
        log("adaptive", dms, "ms per render,", arays, "rays, blocks per level", counts)
    if args.copy_probe:
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy probe: 1 GiB read + 1 GiB written")
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        img_np = img.cpu().numpy()
        out["cpu_baseline"], pix, io, ao = cpu_baseline(w, grid64, budget_s=args.cpu_budget)
        out["accuracy"] = accuracy(img_np, a, pix, io, ao, 1e-4 if args.precision == 1 else 1e-10)
        out["accuracy"]["reference"] = "FP64 oracle on the FP64 cells, pixels of the CPU-baseline runs"
        log("accuracy", out["accuracy"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
