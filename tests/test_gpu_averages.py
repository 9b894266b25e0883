"""Averaged quantities through the C ABI (bl_render_averages; paper section
4, Auxiliary Images) against the FP64 oracle's: each of the 21 maps agrees
to 1e-10 of its largest value in FP64 and 1e-4 in the mixed form, on pixels
whose step counts match; the image and aux maps equal bl_render's."""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-averages]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_2203_15963_amd import blgpu
    blgpu.load()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = blgpu.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _compare(ctx, oracle, name, n, precision, tol, cuts=None):
    from paper_2203_15963_amd import synth
    w = synth.workload(name, n=n)
    g = synth.make_grid(w["grid_args"])
    gg = ctx.grid(g)
    pl = dict(w["plasma"], cuts=cuts) if cuts else w["plasma"]
    if cuts:
        ctx.set_cuts(cuts)
    try:
        im, ax, av = ctx.render_averages(w["camera"], w["spacetime"], w["integrator"], gg, w["plasma"],
                                         precision=precision)
        i1, a1 = ctx.render(w["camera"], w["spacetime"], w["integrator"], gg, w["plasma"], precision=precision)
    finally:
        ctx.set_cuts(None)
    torch.cuda.synchronize()
    assert torch.equal(im, i1) and torch.equal(ax, a1)
    io, ao, avo = oracle.render(w["camera"], w["spacetime"], w["integrator"], g, pl, averages=True)
    a, v = ax.cpu().numpy(), av.cpu().numpy()
    match = (a[5] == ao[5]) & (a[6] == ao[6])
    assert match.sum() >= 0.98 * match.size
    worst = 0.0
    for m in range(21):
        scale = np.abs(avo[m]).max()
        if scale == 0.0:
            assert np.all(v[m][match] == 0.0), m
            continue
        e = np.abs(v[m] - avo[m])[match].max() / scale
        worst = max(worst, e)
        assert e <= tol, (m, e)
    _say(name, n, "precision", precision, "cuts" if cuts else "", "worst map error", worst)


@pytest.mark.parametrize("name,n,precision", [("c2_256_pol", 12, 0), ("c2_256_pol", 12, 1), ("c1_64_unpol", 10, 0),
                                              ("c3_1024_smr", 10, 1)])
def test_averages_match_oracle(ctx, oracle, name, n, precision):
    _compare(ctx, oracle, name, n, precision, 1e-10 if precision == 0 else 1e-4)


def test_averages_with_cuts_match_oracle(ctx, oracle):
    _compare(ctx, oracle, "c2_256_pol", 10, 0, 1e-10, cuts={"theta_e": (3.0, math.inf), "r": (4.0, 40.0)})


@pytest.mark.parametrize("precision", [0, 1])
def test_averages_full_size_sampled(ctx, oracle, precision):
    """The 21 averaged maps of the 1024^2 SMR image (the benchmark's
    --averages configuration; FP32 grid in the mixed form) on 120 random
    pixels against the oracle on the same cell values; the image and the
    geodesic maps of the same call equal a plain render's bit for bit.  A
    map's error is taken relative to its largest sampled value."""
    from paper_2203_15963_amd import synth
    w = synth.workload("c3_1024_smr", n=1024)
    g = synth.make_grid(w["grid_args"])
    if precision == 1:
        g = dict(g, prims=g["prims"].astype(np.float32))
    gg = ctx.grid(g)
    args = (w["camera"], w["spacetime"], w["integrator"], gg, w["plasma"])
    im, ax, av = ctx.render_averages(*args, precision=precision)
    i1, a1 = ctx.render(*args, precision=precision)
    torch.cuda.synchronize()
    assert torch.equal(im, i1) and torch.equal(ax, a1)
    gg.close()
    n = 1024
    rng = np.random.default_rng(71 + precision)
    pix = rng.choice(n * n, size=120, replace=False)
    go = dict(g, prims=g["prims"].astype(np.float64))
    io, ao, avo = oracle.render_pixels(w["camera"], w["spacetime"], w["integrator"], go, w["plasma"], pix,
                                       averages=True)
    a = ax.cpu().numpy().reshape(-1, n * n)[:, pix].T
    v = av.cpu().numpy().reshape(21, n * n)[:, pix].T
    assert np.array_equal(a[:, 5:8], ao[:, 5:8])
    tol = 1e-10 if precision == 0 else 1e-4
    worst = 0.0
    for m in range(21):
        scale = np.abs(avo[:, m]).max()
        if scale == 0.0:
            assert np.all(v[:, m] == 0.0), m
            continue
        e = np.abs(v[:, m] - avo[:, m]).max() / scale
        worst = max(worst, e)
        assert e <= tol, (m, e)
    _say("c3_1024_smr 1024^2 sampled, precision", precision, "worst map error", worst)
