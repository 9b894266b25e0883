"""The benchmark's command line on a machine without a GPU: a request for
more than one GPU ends at once with a message and a non-zero status, before
any device is touched (the build targets one GPU)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    msg = (r.stdout + r.stderr).lower()
    assert "one gpu" in msg or "1 gpu" in msg or "single gpu" in msg, msg[-500:]
    assert '"metric"' not in r.stdout


def _bench():
    sys.path.insert(0, ROOT)
    import bench
    return bench


def test_useful_operations_do_not_exceed_issued_ones():
    """The per-unit counts (divergence-free launches) applied to the units of
    the launch the counters were taken on give at most the operations that
    launch issued (masked lanes add issued work, never remove it), and the
    ratio is about the measured lane activity (within 0.06: the activity
    counter averages over every VALU instruction, integer, move and compare
    ones included, weighted by their cycles, the ratio over floating-point
    operations only; the FP64 kernel's divergent branches carry more of the
    former)."""
    b = _bench()
    if b.OPS_PER_UNIT["src"] != b.COUNTERS["src"]:
        return
    for key, cn in b.COUNTERS.items():
        if key == "src":
            continue
        prec, dom = key
        model = b.OPS_PER_UNIT[prec][dom]
        useful = sum(c * cn["units"][u] for t in ("F64", "F32") for u, c in model[t].items())
        issued = cn["issued_f64"] + cn["issued_f32"]
        assert useful <= issued, (key, useful, issued)
        assert abs(useful / issued - cn["lane_activity"]) <= 0.06, (key, useful / issued, cn["lane_activity"])


def test_roofline_fraction_is_bounded_by_the_ceiling():
    """At the launch time that the issued operations fill the VALU ceiling
    exactly, the reported (useful) fraction is at most 1."""
    b = _bench()
    src = b.source_hash()
    if b.COUNTERS["src"] != src or b.OPS_PER_UNIT["src"] != src:
        return
    for key, cn in b.COUNTERS.items():
        if key == "src":
            continue
        prec, dom = key
        t_min = (cn["issued_f64"] + cn["issued_f32"]) / (b.VALU_PEAK_TFLOPS * 1e12)
        r = b.roofline(prec, dom, {dom: {"avg_launch_ms": t_min * 1e3, "launches_per_step": 1.0}}, cn["units"])
        assert r["frac"] <= 1.0 and abs(r["issued"]["frac"] - 1.0) < 1e-9


def test_accuracy_metric_definition():
    """E_pix per pixel = max over Stokes of |X_gpu - X_oracle| over
    max(I_oracle, 1e-3 max I of the image); repeated pixels count once; step
    count mismatches are counted and their E_pix reported apart."""
    import numpy as np
    import bench
    n = 8
    img = np.zeros((4, n * n))
    img[0] = np.linspace(1.0, 2.0, n * n)            # max I = 2
    aux = np.zeros((10, n * n))
    aux[5], aux[6] = 50.0, 5.0
    pix = np.array([3, 10, 10, 40])
    io = img[:, pix].T.copy()
    ao = aux[:, pix].T.copy()
    io[0, 2] += 1e-3                                  # U off by 1e-3 on pixel 3
    io[1, 0] = 1e-6                                   # a dark pixel: the floor 2e-3 applies
    img[0, 10] = 1e-6 + 4e-9                          # ... with an error of 4e-9 in I
    io[3, 0] *= 1.0 + 1e-5                            # pixel 40: I off by 1e-5 relative
    ao[3, 6] = 6.0                                    # and a rejected-step mismatch
    r = bench.accuracy(img.reshape(4, n, n), aux.reshape(10, n, n), pix, io, ao, 1e-4)
    assert r["pixels"] == 3
    e3 = 1e-3 / io[0, 0]
    e10 = 4e-9 / 2e-3
    e40 = abs(img[0, 40] - io[3, 0]) / io[3, 0]
    assert abs(r["E_pix_max"] - e3) < 1e-12
    assert abs(r["E_pix_median"] - e40) < 1e-12
    assert r["step_count_mismatches"] == 1
    assert abs(r["E_pix_max_mismatched"] - e40) < 1e-12
    assert r["within_tolerance"] is False and e10 < 1e-5
