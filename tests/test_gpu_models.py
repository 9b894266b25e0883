"""Several plasma models on one geodesic pass through the C ABI (paper
section 5: an imaging study varies the frequency and the electron model of a
snapshot; section 4.8: several frequencies for fixed camera and data).  Every
output -- with its own R_high, R_low, sigma_max, polarization, electron
populations and frequency -- equals a single render with that plasma and
frequency bit for bit, and the FP64 oracle at the parity tolerance."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-10
TOL_MIXED = 1e-4

# (overrides of the workload's plasma, frequency in Hz)
MODELS = [
    ({}, 230e9),
    ({"r_high": 160.0, "r_low": 3.0}, 230e9),
    ({"r_high": 1.0, "sigma_max": 0.3}, 345e9),
    ({"polarized": 0, "r_high": 40.0}, 86e9),
    ({"fractions": (1 / 3, 1 / 3, 1 / 3)}, 230e9),
    ({"fractions": (0.0, 0.0, 1.0), "kappa": 3.5, "polarized": 0}, 230e9),
]


def _say(*a):
    print("[gpu-models]", *a, flush=True)
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


def _workload(name, n):
    from paper_2203_15963_amd import synth
    w = synth.workload(name, n=n)
    key = repr(sorted(w["grid_args"].items()))
    if key not in _GRIDS:
        _GRIDS[key] = synth.make_grid(w["grid_args"])
    return w, _GRIDS[key]


def _plasmas(w, models):
    return [dict(w["plasma"], **over) for over, _ in models], [nu for _, nu in models]


@pytest.mark.parametrize("precision", [0, 1])
def test_models_equal_single_renders(ctx, precision):
    w, g = _workload("c2_256_pol", 14)
    if precision == 1:
        g = dict(g, prims=g["prims"].astype(np.float32))
    gg = ctx.grid(g)
    pls, nus = _plasmas(w, MODELS)
    _say("c2_256_pol 14^2 precision", precision, "models", len(pls))
    outs = ctx.render_models(w["camera"], w["spacetime"], w["integrator"], gg, pls, nus, precision=precision)
    for k, ((im, ax), pl, nu) in enumerate(zip(outs, pls, nus)):
        im1, ax1 = ctx.render(dict(w["camera"], nu_hz=nu), w["spacetime"], w["integrator"], gg, pl,
                              precision=precision)
        torch.cuda.synchronize()
        assert torch.equal(im, im1), k
        assert torch.equal(ax, ax1), k
    # the models differ: no two images are copies of one another
    for a in range(len(outs)):
        for b in range(a):
            assert not torch.equal(outs[a][0], outs[b][0]), (a, b)


def test_models_at_the_camera_frequency(ctx):
    """Without frequencies every output is at the camera's."""
    w, g = _workload("c1_64_unpol", 10)
    gg = ctx.grid(g)
    pls = [dict(w["plasma"], r_high=rh) for rh in (5.0, 20.0, 80.0)]
    outs = ctx.render_models(w["camera"], w["spacetime"], w["integrator"], gg, pls)
    for (im, ax), pl in zip(outs, pls):
        im1, ax1 = ctx.render(w["camera"], w["spacetime"], w["integrator"], gg, pl)
        torch.cuda.synchronize()
        assert torch.equal(im, im1) and torch.equal(ax, ax1)


def test_models_match_oracle(ctx, oracle):
    w, g = _workload("c2_256_pol", 10)
    gg = ctx.grid(g)
    pls, nus = _plasmas(w, MODELS)
    outs = ctx.render_models(w["camera"], w["spacetime"], w["integrator"], gg, pls, nus, precision=0)
    torch.cuda.synchronize()
    for k, ((im, ax), pl, nu) in enumerate(zip(outs, pls, nus)):
        io, ao = oracle.render(dict(w["camera"], nu_hz=nu), w["spacetime"], w["integrator"], g, pl)
        im, ax = im.cpu().numpy(), ax.cpu().numpy()
        I = io[0]
        den = np.maximum(np.abs(I), 1e-3 * np.abs(I).max())
        e = (np.abs(im - io) / den).max()
        _say("model", k, MODELS[k][0], "nu", nu, "E_pix", float(e))
        assert np.array_equal(ax[5:8], ao[5:8])
        assert np.abs(I).max() > 0
        assert e <= TOL_FP64


def test_models_refusals(ctx):
    from paper_2203_15963_amd import blgpu
    w, g = _workload("c2_256_pol", 4)
    gg = ctx.grid(g)
    args = (w["camera"], w["spacetime"], w["integrator"], gg)

    def status(fn):
        with pytest.raises(blgpu.BlError) as ei:
            fn()
        torch.cuda.synchronize()
        return ei.value.status

    assert status(lambda: ctx.render_models(*args, [])) == blgpu.STATUS["E_INVALID_ARG"]
    bad = [w["plasma"], dict(w["plasma"], mu=-1.0)]
    assert status(lambda: ctx.render_models(*args, bad)) == blgpu.STATUS["E_INVALID_ARG"]
    assert status(lambda: ctx.render_models(*args, [w["plasma"]] * 2, [230e9, 0.0])) == blgpu.STATUS[
        "E_INVALID_ARG"]
    # a nonthermal output with data cuts
    ctx.set_cuts({"r": (4.0, 40.0)})
    try:
        mixed_models = [w["plasma"], dict(w["plasma"], fractions=(0.5, 0.5, 0.0))]
        assert status(lambda: ctx.render_models(*args, mixed_models)) == blgpu.STATUS["E_UNSUPPORTED"]
        # thermal outputs with cuts are rendered
        outs = ctx.render_models(*args, [w["plasma"], dict(w["plasma"], r_high=80.0)])
        im1, _ = ctx.render(*args, dict(w["plasma"], r_high=80.0))
        torch.cuda.synchronize()
        assert torch.equal(outs[1][0], im1)
    finally:
        ctx.set_cuts(None)
