"""Multi-frequency render through the C ABI (one geodesic pass, one transfer
per frequency on the same step records): every frequency's image and aux
maps equal a single-frequency render of that frequency bit for bit, and the
FP64 oracle at the parity tolerance."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

NUS = [86e9, 230e9, 690e9]


def _say(*a):
    print("[gpu-multifreq]", *a, flush=True)
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


def _workload(name, n, freq_mode=None):
    from paper_2203_15963_amd import synth
    w = synth.workload(name, n=n)
    if freq_mode is not None:
        w["camera"]["freq_mode"] = freq_mode
    return w, synth.make_grid(w["grid_args"])


@pytest.mark.parametrize("name,n,precision,freq_mode", [("c2_256_pol", 12, 0, None), ("c2_256_pol", 12, 1, None),
                                                        ("c2_256_pol", 10, 0, 1), ("c1_64_unpol", 9, 1, None)])
def test_multifreq_equals_single_frequency_renders(ctx, name, n, precision, freq_mode):
    w, g = _workload(name, n, freq_mode)
    gg = ctx.grid(g)
    _say(name, n, "precision", precision, "freq_mode", w["camera"]["freq_mode"], "frequencies", NUS)
    outs = ctx.render_multifreq(w["camera"], w["spacetime"], w["integrator"], gg, w["plasma"], NUS,
                                precision=precision)
    for nu, (im, ax) in zip(NUS, outs):
        im1, ax1 = ctx.render(dict(w["camera"], nu_hz=nu), w["spacetime"], w["integrator"], gg, w["plasma"],
                              precision=precision)
        torch.cuda.synchronize()
        assert torch.equal(im, im1), nu
        assert torch.equal(ax, ax1), nu
    # the frequencies differ: the images are not copies of one another
    assert not torch.equal(outs[0][0], outs[1][0])


def test_multifreq_matches_oracle(ctx, oracle):
    w, g = _workload("c2_256_pol", 10)
    gg = ctx.grid(g)
    outs = ctx.render_multifreq(w["camera"], w["spacetime"], w["integrator"], gg, w["plasma"], NUS)
    torch.cuda.synchronize()
    for nu, (im, ax) in zip(NUS, outs):
        io, ao = oracle.render(dict(w["camera"], nu_hz=nu), w["spacetime"], w["integrator"], g, w["plasma"])
        ig, ag = im.cpu().numpy(), ax.cpu().numpy()
        match = (ag[5] == ao[5]) & (ag[6] == ao[6])
        den = np.maximum(np.abs(io[0]), 1e-3 * np.abs(io[0]).max())
        e = (np.abs(ig - io) / den[None]).max(axis=0)
        _say("nu", nu, "E_pix(matched)", e[match].max(), "matched", int(match.sum()), "of", match.size)
        assert match.sum() >= 0.98 * match.size
        assert e[match].max() <= 1e-10


def test_multifreq_rejects_bad_arguments(ctx):
    from paper_2203_15963_amd import blgpu
    w, g = _workload("c1_64_unpol", 4)
    gg = ctx.grid(g)
    with pytest.raises(blgpu.BlError):
        ctx.render_multifreq(w["camera"], w["spacetime"], w["integrator"], gg, w["plasma"], [230e9, -1.0])
    with pytest.raises(blgpu.BlError):
        ctx.render_multifreq(w["camera"], w["spacetime"], w["integrator"], gg, w["plasma"], [])
