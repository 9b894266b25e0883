"""Floating-point operations per unit of work of the HIP kernels, measured.

Method: divergence-free launches.  An 8x8 image whose camera width is 1e-9 M
sends 64 copies of one ray through the pipeline, so the geodesic kernel runs
them as one wave of identical lanes and the persistent transfer kernel hands
all 64 to one wave as well.  Every VALU instruction of those dispatches then
executes with all lanes doing the same work, and the per-wave instruction
counters (SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_{F32,F64}) equal the operations of
one ray.  Launches aimed in many directions give one equation each,

    geodesic:  ops(ray) = c_trial * trial_steps + c_acc * accepted_steps + c_ray
    transfer:  ops(ray) = c_samp * plasma_samples + c_rec * records
                          + c_acc * accepted_steps + c_ray

and non-negative least squares gives the per-unit figures.  An FMA counts as two
operations; add, multiply and each transcendental-unit instruction (rcp,
sqrt, exp, log, sin, ...) as one.

The same counters over a benchmark run give the operations the kernels
issued there (masked lanes included); `issued` summarises them per kernel
together with the VALU lane activity and the HBM byte counters when those
passes are given.

Usage, on the GPU machine (the counter pass needs rocprofv3):

    rocprofv3 --pmc SQ_INSTS_VALU_ADD_F32 SQ_INSTS_VALU_MUL_F32 SQ_INSTS_VALU_FMA_F32 \
        SQ_INSTS_VALU_TRANS_F32 SQ_INSTS_VALU_ADD_F64 SQ_INSTS_VALU_MUL_F64 \
        SQ_INSTS_VALU_FMA_F64 SQ_INSTS_VALU_TRANS_F64 -d <dir> -o ops -- \
        python3 -m paper_2203_15963_amd.opcount run --precision 1 --out <cases.json>
    python3 -m paper_2203_15963_amd.opcount fit <dir>/.../ops_results.db <cases.json>
"""
import argparse
import json
import math
import sqlite3
import sys

import numpy as np
from scipy.optimize import nnls

COUNTERS = ["SQ_INSTS_VALU_ADD_F32", "SQ_INSTS_VALU_MUL_F32", "SQ_INSTS_VALU_FMA_F32", "SQ_INSTS_VALU_TRANS_F32",
            "SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_TRANS_F64"]


def directions(n_dirs, seed=5, max_tilt=0.16):
    """Camera k_i (spherical KS, covariant) tilted off the radial direction
    by up to max_tilt radians, uniform over the disc of tilts."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_dirs):
        rho = max_tilt * math.sqrt(rng.random())
        ang = 2 * math.pi * rng.random()
        out.append((rho * math.cos(ang), rho * math.sin(ang)))
    return out


def run(workload="c3_1024_smr", precision=1, n_dirs=48, out=None, seed=5):
    import torch
    from paper_2203_15963_amd import blgpu, synth

    w = synth.workload(workload, n=8)
    grid = synth.make_grid(w["grid_args"], dtype=np.float32 if precision == 1 else np.float64)
    ctx = blgpu.Context(0)
    gg = ctx.grid(grid)
    cases = []
    r = w["camera"]["r"]
    st = math.sin(w["camera"]["theta"])
    for t1, t2 in directions(n_dirs, seed):
        cam = dict(w["camera"], width=1e-9, k_cov=(1.0, r * t1, r * st * t2))
        img, aux = ctx.render(cam, w["spacetime"], w["integrator"], gg, w["plasma"], precision=precision)
        torch.cuda.synchronize()
        a = aux.cpu().numpy().reshape(blgpu.NAUX, -1)
        acc, rej, samp, rec = a[5], a[6], a[8], a[9]
        uniform = bool((acc == acc[0]).all() and (rej == rej[0]).all() and (samp == samp[0]).all()
                       and (rec == rec[0]).all())
        cases.append({"tilt": [t1, t2], "uniform": uniform, "acc": float(acc[0]), "trial": float(acc[0] + rej[0]),
                      "samp": float(samp[0]), "rec": float(rec[0]), "status": float(a[7][0])})
        print(f"[opcount] tilt ({t1:+.3f},{t2:+.3f}) uniform={uniform} acc={acc[0]:.0f} rej={rej[0]:.0f} "
              f"samp={samp[0]:.0f} rec={rec[0]:.0f}", flush=True)
    ctx.close()
    doc = {"workload": workload, "precision": precision, "n_dirs": n_dirs, "seed": seed,
           "polarized": int(w["plasma"]["polarized"]), "cases": cases}
    if out:
        with open(out, "w") as f:
            json.dump(doc, f)
    return doc


def _dispatch_counters(db):
    con = sqlite3.connect(db)
    rows = con.execute("select dispatch_id, kernel_name, counter_name, sum(value) from counters_collection "
                       "group by dispatch_id, counter_name order by dispatch_id").fetchall()
    disp = {}
    for d, k, c, v in rows:
        e = disp.setdefault(d, {"kernel": k, "c": {}})
        e["c"][c] = float(v)
    return [disp[d] for d in sorted(disp)]


def _flops(c, suffix):
    return (c.get("SQ_INSTS_VALU_ADD_" + suffix, 0.0) + c.get("SQ_INSTS_VALU_MUL_" + suffix, 0.0)
            + 2.0 * c.get("SQ_INSTS_VALU_FMA_" + suffix, 0.0) + c.get("SQ_INSTS_VALU_TRANS_" + suffix, 0.0))


def fit(db, cases_json):
    doc = json.load(open(cases_json))
    cases = doc["cases"]
    ds = _dispatch_counters(db)
    geo = [d for d in ds if "k_geodesic" in d["kernel"]]
    tr = [d for d in ds if "k_transfer" in d["kernel"]]
    if len(geo) != len(cases) or len(tr) != len(cases):
        raise SystemExit(f"dispatch count mismatch: {len(geo)} geodesic, {len(tr)} transfer, {len(cases)} cases")
    keep = [i for i, c in enumerate(cases) if c["uniform"]]
    res = {"workload": doc["workload"], "precision": doc["precision"], "cases_used": len(keep),
           "cases": len(cases)}
    for name, disp, cols in (("geodesic", geo, ["trial", "acc"]), ("transfer", tr, ["samp", "rec", "acc"])):
        A = np.array([[cases[i][k] for k in cols] + [1.0] for i in keep])
        for suffix in ("F64", "F32"):
            y = np.array([_flops(disp[i]["c"], suffix) for i in keep])
            coef, _ = nnls(A, y)   # a unit cannot cost negative work
            pred = A @ coef
            rel = float(np.max(np.abs(pred - y) / np.maximum(y, 1.0))) if len(y) else 0.0
            res[f"{name}_{suffix}"] = {**{f"per_{k}": float(v) for k, v in zip(cols + ["ray"], coef)},
                                       "max_rel_residual": rel, "mean_ops_per_ray": float(y.mean())}
    return res


def issued(dbs):
    """Per kernel name: dispatches, issued FP64 / FP32 operations per dispatch
    (instruction counters x 64 lanes, FMA = 2), VALU lane activity
    (SQ_THREAD_CYCLES_VALU / (64 SQ_ACTIVE_INST_VALU)) and FETCH_SIZE /
    WRITE_SIZE (KiB) per dispatch, from any number of counter databases."""
    acc = {}
    for db in dbs:
        for d in _dispatch_counters(db):
            e = acc.setdefault(d["kernel"], {})
            for c, v in d["c"].items():
                e.setdefault(c, []).append(v)
    out = {}
    for k, e in acc.items():
        mean = {c: float(np.mean(v)) for c, v in e.items()}
        r = {"dispatches": max(len(v) for v in e.values())}
        if "SQ_INSTS_VALU_FMA_F64" in mean:
            r["issued_f64"] = 64.0 * _flops(mean, "F64")
            r["issued_f32"] = 64.0 * _flops(mean, "F32")
        if "SQ_ACTIVE_INST_VALU" in mean and mean["SQ_ACTIVE_INST_VALU"] > 0:
            r["lane_activity"] = mean["SQ_THREAD_CYCLES_VALU"] / (64.0 * mean["SQ_ACTIVE_INST_VALU"])
            r["valu_insts"] = mean.get("SQ_INSTS_VALU")
        for c in ("FETCH_SIZE", "WRITE_SIZE"):
            if c in mean:
                r[c] = mean[c]
        out[k] = r
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    r = sub.add_parser("run")
    r.add_argument("--workload", default="c3_1024_smr")
    r.add_argument("--precision", type=int, default=1)
    r.add_argument("--n-dirs", type=int, default=48)
    r.add_argument("--out", required=True)
    f = sub.add_parser("fit")
    f.add_argument("db")
    f.add_argument("cases")
    s = sub.add_parser("issued")
    s.add_argument("dbs", nargs="+")
    a = ap.parse_args(argv)
    if a.cmd == "run":
        run(a.workload, a.precision, a.n_dirs, a.out)
    elif a.cmd == "fit":
        print(json.dumps(fit(a.db, a.cases), indent=1))
    else:
        print(json.dumps(issued(a.dbs), indent=1))


if __name__ == "__main__":
    main()
