"""Nonthermal electrons on the GPU (paper sections 2.6 and 4.5): power-law and
kappa populations and their admixtures with the thermal one, against the FP64
oracle -- per-sample coefficients, whole images in the FP64 form (E_pix <=
1e-10) and the mixed form (1e-4), unpolarized and polarized (whose Stokes
step then has no Kirchhoff relation between source and absorption) -- and
the boundary's answers for what it does not take: invalid populations,
nonthermal electrons with data cuts or in a batch, another camera kind, and a
learned step without a network (a missing state)."""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-10
TOL_MIXED = 1e-4
MIXES = {"power law": (0.0, 1.0, 0.0), "kappa": (0.0, 0.0, 1.0), "thirds": (1 / 3, 1 / 3, 1 / 3),
         "mostly thermal": (0.8, 0.15, 0.05)}


def _say(*a):
    print("[gpu-nonthermal]", *a, flush=True)
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


_GRIDS = {}


def _grid(w):
    from paper_2203_15963_amd import synth
    key = repr(sorted(w["grid_args"].items()))
    if key not in _GRIDS:
        _GRIDS[key] = synth.make_grid(w["grid_args"])
    return _GRIDS[key]


def _wl(name, n, fractions, **pl):
    from paper_2203_15963_amd import synth
    w = synth.workload(name, n=n)
    w["plasma"].update(fractions=fractions, **pl)
    return w


def test_coefficients_match_oracle(ctx, oracle):
    """Per sample: the admixture's eight coefficients (invariant form) and the
    plasma state equal the oracle's at random points of the polarized grid."""
    w = _wl("c2_256_pol", 8, MIXES["thirds"])
    g = _grid(w)
    gg = ctx.grid(g)
    rng = np.random.default_rng(17)
    a = w["spacetime"]["a"]
    states, norms = [], []
    while len(states) < 300:
        x = rng.uniform(-45, 45, 3)
        if np.linalg.norm(x) < 3:
            continue
        k = np.concatenate([[-1.0], rng.normal(size=3)])
        gm, gi = oracle.metric(a, np.concatenate([[0.0], x]))
        A, B, Cq = gi[0, 0], gi[0, 1:] @ k[1:], k[1:] @ gi[1:, 1:] @ k[1:]
        k[0] = (-B + math.sqrt(B * B - A * Cq)) / A
        states.append(np.concatenate([[0.0], x, k]))
        norms.append(2.3e11 / -k[0])
    states, norms = np.array(states), np.array(norms)
    for name, fr in MIXES.items():
        pl = dict(w["plasma"], fractions=fr)
        out = ctx.eval_samples(w["spacetime"], gg, pl, states, norms)
        torch.cuda.synchronize()
        out = out.cpu().numpy()
        n_plasma = 0
        worst = 0.0
        for s in range(len(states)):
            ref = oracle.sample_point(w["spacetime"], g, pl, states[s], norms[s])
            assert out[s, 52] == ref[28]
            if ref[28] == 0:
                continue
            n_plasma += 1
            for m in range(8):
                d = abs(out[s, 24 + m] - ref[m])
                scale = max(abs(ref[m]), 1e-300)
                worst = max(worst, d / scale if ref[m] != 0 else d)
                assert d <= 1e-11 * scale, (name, s, m, out[s, 24 + m], ref[m])
        _say("coefficients", name, "plasma samples", n_plasma, "worst relative difference", worst)
        assert n_plasma > 80


def _compare(ctx, oracle, w, precision, tol):
    g = _grid(w)
    gg = ctx.grid(g)
    img, aux = ctx.render(w["camera"], w["spacetime"], w["integrator"], gg, w["plasma"], precision=precision)
    torch.cuda.synchronize()
    img, aux = img.cpu().numpy(), aux.cpu().numpy()
    io, ao = oracle.render(w["camera"], w["spacetime"], w["integrator"], g, w["plasma"])
    match = (ao[5] == aux[5]) & (ao[6] == aux[6]) & (ao[7] == aux[7])
    I = io[0]
    den = np.maximum(np.abs(I), 1e-3 * np.abs(I).max())
    e = (np.abs(img - io) / den).max(axis=0)
    _say("render", w["plasma"]["fractions"], "polarized", w["plasma"]["polarized"], "precision", precision,
         "E_pix", float(e.max()), "mismatched", int((~match).sum()), "max I", float(np.abs(I).max()))
    assert match.all()
    assert e.max() <= tol
    assert np.abs(I).max() > 0
    for q in (3, 4):   # optical depth and integrated emissivity of the mixture
        assert np.abs(aux[q] - ao[q]).max() <= tol * np.abs(ao[q]).max()
    return img, io


@pytest.mark.parametrize("mix", list(MIXES))
@pytest.mark.parametrize("precision", [0, 1])
def test_polarized_render_matches_oracle(ctx, oracle, mix, precision):
    w = _wl("c2_256_pol", 12, MIXES[mix])
    _compare(ctx, oracle, w, precision, TOL_FP64 if precision == 0 else TOL_MIXED)


@pytest.mark.parametrize("mix", ["power law", "thirds"])
@pytest.mark.parametrize("precision", [0, 1])
def test_unpolarized_render_matches_oracle(ctx, oracle, mix, precision):
    w = _wl("c1_64_unpol", 16, MIXES[mix])
    _compare(ctx, oracle, w, precision, TOL_FP64 if precision == 0 else TOL_MIXED)


def test_other_population_parameters(ctx, oracle):
    """Another power law (p = 2.5, gamma 10..1e4) and kappa distribution
    (kappa = 3.5, w = 1) on the SMR grid."""
    w = _wl("c3_1024_smr", 11, (0.4, 0.3, 0.3), pl_p=2.5, pl_gamma_min=10.0, pl_gamma_max=1e4, kappa=3.5,
            kappa_w=1.0)
    _compare(ctx, oracle, w, 0, TOL_FP64)


def test_full_size_sampled(ctx, oracle):
    """The 256^2 polarized workload with the paper's equal thirds, FP64, on
    200 sampled pixels."""
    w = _wl("c2_256_pol", 256, MIXES["thirds"])
    g = _grid(w)
    gg = ctx.grid(g)
    img, aux = ctx.render(w["camera"], w["spacetime"], w["integrator"], gg, w["plasma"], precision=0)
    torch.cuda.synchronize()
    img, aux = img.cpu().numpy(), aux.cpu().numpy()
    rng = np.random.default_rng(23)
    pix = rng.choice(256 * 256, size=200, replace=False)
    io, ao = oracle.render_pixels(w["camera"], w["spacetime"], w["integrator"], g, w["plasma"], pix)
    ig, ag = img.reshape(4, -1)[:, pix].T, aux.reshape(10, -1)[:, pix].T
    den = np.maximum(np.abs(io[:, 0]), 1e-3 * np.abs(img[0]).max())
    e = (np.abs(ig - io) / den[:, None]).max(axis=1)
    _say("256^2 thirds sampled E_pix", float(e.max()))
    assert np.array_equal(ag[:, 5:8], ao[:, 5:8])
    assert e.max() <= TOL_FP64


def test_multifrequency_render_equals_single_renders(ctx):
    w = _wl("c2_256_pol", 10, MIXES["thirds"])
    gg = ctx.grid(_grid(w))
    nus = [150e9, 345e9]
    outs = ctx.render_multifreq(w["camera"], w["spacetime"], w["integrator"], gg, w["plasma"], nus, precision=0)
    for nu, (im, ax) in zip(nus, outs):
        i1, a1 = ctx.render(dict(w["camera"], nu_hz=nu), w["spacetime"], w["integrator"], gg, w["plasma"],
                            precision=0)
        torch.cuda.synchronize()
        assert torch.equal(im, i1) and torch.equal(ax, a1)


def test_boundary_refusals(ctx):
    from paper_2203_15963_amd import blgpu, synth
    w = _wl("c2_256_pol", 4, MIXES["thirds"])
    gg = ctx.grid(_grid(w))
    args = (w["camera"], w["spacetime"], w["integrator"], gg)

    def status(fn):
        with pytest.raises(blgpu.BlError) as ei:
            fn()
        torch.cuda.synchronize()
        return ei.value.status

    # invalid populations
    assert status(lambda: ctx.render(*args, dict(w["plasma"], fractions=(0.5, 0.6, 0.0)))) == blgpu.STATUS[
        "E_INVALID_ARG"]
    assert status(lambda: ctx.render(*args, dict(w["plasma"], kappa=2.2))) == blgpu.STATUS["E_INVALID_ARG"]
    assert status(lambda: ctx.render(*args, dict(w["plasma"], pl_p=1.0))) == blgpu.STATUS["E_INVALID_ARG"]
    # nonthermal electrons with data cuts, or in a batch
    ctx.set_cuts({"r": (4.0, 40.0)})
    try:
        assert status(lambda: ctx.render(*args, w["plasma"])) == blgpu.STATUS["E_UNSUPPORTED"]
    finally:
        ctx.set_cuts(None)
    assert status(lambda: ctx.render_batch([(w["camera"], w["spacetime"])], w["integrator"], gg,
                                           w["plasma"])) == blgpu.STATUS["E_UNSUPPORTED"]
    # a camera kind other than the plane-parallel one
    assert status(lambda: ctx.render(dict(w["camera"], kind=1), w["spacetime"], w["integrator"], gg,
                                     w["plasma"])) == blgpu.STATUS["E_UNSUPPORTED"]
    # learned steps without a network on a fresh context; a grid of another context
    c2 = blgpu.Context(0)
    try:
        g2 = c2.grid(_grid(w))
        assert status(lambda: c2.render(*args[:3], g2, w["plasma"], step_model=1)) == blgpu.STATUS["E_STATE"]
        assert status(lambda: ctx.render(*args[:3], g2, w["plasma"])) == blgpu.STATUS["E_STATE"]
        g2.close()
    finally:
        c2.close()
    # and the context still renders
    img, aux = ctx.render(*args, w["plasma"])
    torch.cuda.synchronize()
    assert torch.isfinite(img).all()


def test_mixed_full_size_sampled(ctx, oracle):
    """The 1024^2 SMR image with the paper's equal thirds in the mixed form
    (FP32 grid and the FP32 general Stokes step), 100 sampled pixels against
    the oracle on the same cell values, to the mixed tolerance."""
    from paper_2203_15963_amd import synth
    w = _wl("c3_1024_smr", 1024, MIXES["thirds"])
    g = _grid(w)
    g32 = dict(g, prims=g["prims"].astype(np.float32))
    gg = ctx.grid(g32)
    img, aux = ctx.render(w["camera"], w["spacetime"], w["integrator"], gg, w["plasma"], precision=1)
    torch.cuda.synchronize()
    gg.close()
    img, aux = img.cpu().numpy(), aux.cpu().numpy()
    n = 1024
    rng = np.random.default_rng(29)
    pix = rng.choice(n * n, size=100, replace=False)
    go = dict(g, prims=g32["prims"].astype(np.float64))
    io, ao = oracle.render_pixels(w["camera"], w["spacetime"], w["integrator"], go, w["plasma"], pix)
    ig, ag = img.reshape(4, -1)[:, pix].T, aux.reshape(10, -1)[:, pix].T
    den = np.maximum(np.abs(io[:, 0]), 1e-3 * np.abs(img[0]).max())
    e = (np.abs(ig - io) / den[:, None]).max(axis=1)
    _say("1024^2 thirds mixed sampled E_pix", float(e.max()), "median", float(np.median(e)))
    assert np.array_equal(ag[:, 5:8], ao[:, 5:8])
    assert e.max() <= TOL_MIXED
