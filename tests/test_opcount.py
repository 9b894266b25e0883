"""Host logic of the per-unit operation fit (no GPU): a synthetic counter
database built from known per-unit costs must give those costs back."""
import json
import sqlite3

import numpy as np

from paper_2203_15963_amd import opcount


def _make(tmp_path, truth, cases):
    db = tmp_path / "ops.db"
    con = sqlite3.connect(db)
    con.execute("create table counters_collection (dispatch_id int, kernel_name text, counter_name text, value real)")
    did = 0
    for c in cases:
        for kern, units in (("k_geodesic<true>", ("trial", "acc")), ("k_transfer<true, float>", ("samp", "rec", "acc"))):
            did += 1
            name = "geodesic" if "geodesic" in kern else "transfer"
            for suffix in ("F64", "F32"):
                t = truth[name][suffix]
                ops = sum(t[u] * c[u] for u in units) + t["ray"]
                # split the operations over the four instruction classes: FMA counts twice
                fma = 0.25 * ops / 2.0
                rest = ops - 2.0 * fma
                for cls, v in (("FMA", fma), ("ADD", rest / 3), ("MUL", rest / 3), ("TRANS", rest / 3)):
                    # counters are reported per shader engine: split over 4 rows
                    for _ in range(4):
                        con.execute("insert into counters_collection values (?,?,?,?)",
                                    (did, kern, f"SQ_INSTS_VALU_{cls}_{suffix}", v / 4))
        con.execute("insert into counters_collection values (?,?,?,?)", (did + 1000, "k_fill_int", "SQ_INSTS_VALU_ADD_F32", 0))
    con.commit()
    cj = tmp_path / "cases.json"
    cj.write_text(json.dumps({"workload": "t", "precision": 1, "cases": cases}))
    return str(db), str(cj)


def test_fit_recovers_known_costs(tmp_path):
    rng = np.random.default_rng(0)
    truth = {"geodesic": {"F64": {"trial": 1900.0, "acc": 140.0, "ray": 700.0},
                          "F32": {"trial": 0.0, "acc": 3.0, "ray": 10.0}},
             "transfer": {"F64": {"samp": 400.0, "rec": 120.0, "acc": 900.0, "ray": 3000.0},
                          "F32": {"samp": 2600.0, "rec": 800.0, "acc": 0.0, "ray": 500.0}}}
    cases = []
    for _ in range(20):
        acc = float(rng.integers(40, 200))
        cases.append({"uniform": True, "acc": acc, "trial": acc + float(rng.integers(0, 30)),
                      "samp": float(rng.integers(0, 900)), "rec": float(rng.integers(50, 1000))})
    cases.append({"uniform": False, "acc": 1.0, "trial": 1.0, "samp": 1.0, "rec": 1.0})
    db, cj = _make(tmp_path, truth, cases)
    res = opcount.fit(db, cj)
    assert res["cases_used"] == 20
    for name in ("geodesic", "transfer"):
        for suffix in ("F64", "F32"):
            got = res[f"{name}_{suffix}"]
            for u, v in truth[name][suffix].items():
                assert abs(got[f"per_{u}"] - v) <= 1e-6 * (1 + abs(v)), (name, suffix, u, got)


def test_directions_within_tilt():
    d = opcount.directions(200, seed=1, max_tilt=0.1)
    r = np.hypot(*np.array(d).T)
    assert r.max() <= 0.1 and r.min() >= 0.0 and len(set(d)) == 200
