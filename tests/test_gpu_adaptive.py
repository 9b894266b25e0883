"""Adaptive ray tracing through the C ABI (bl_render_adaptive; paper section
4, Adaptive Ray Tracing):
  - every block of every level equals the same pixels of a bl_render at
    that level's resolution N 2^l: step counts and statuses exactly, the
    image to the tolerance that separates a batched render (which the levels
    use) from a single one (1e-12 in FP64, 1e-4 mixed);
  - the refinement decisions: the oracle's criteria applied to the GPU's own
    level images give exactly the GPU's next-level block lists (integers:
    bit-exact), for each criterion alone and for regions;
  - against the FP64 oracle's adaptive render: identical block lists and
    images within the FP64 tolerance on pixels whose step counts match;
  - edge cases: single-pixel blocks, one block, level 0 only, a level that
    refines nothing, the capacity error and bad arguments."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-10


def _say(*a):
    print("[gpu-adaptive]", *a, flush=True)
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


_CACHE = {}


def _setup(ctx, name, n):
    from paper_2203_15963_amd import synth
    key = (name, n)
    if key not in _CACHE:
        w = synth.workload(name, n=n)
        g = synth.make_grid(w["grid_args"])
        _CACHE[key] = (w, g, ctx.grid(g))
    return _CACHE[key]


def _mid_threshold(values, q=0.6):
    """A threshold between two well-separated values near the q-quantile,
    so that rounding differences cannot move a value across it."""
    v = np.unique(np.asarray(values, dtype=np.float64).ravel())
    if len(v) < 2:
        return float(v[0]) if len(v) else 0.0
    gaps = [(v[i + 1] - v[i]) / max(abs(v[i + 1]), 1e-300) for i in range(len(v) - 1)]
    k0 = int(q * (len(v) - 1))
    best = max(range(max(0, k0 - 5), min(len(gaps), k0 + 6)), key=lambda i: gaps[i])
    return 0.5 * (v[best] + v[best + 1])


def _root_threshold(ctx, w, gg, kind, b, precision):
    from oracle import adaptive as A
    img, _ = ctx.render(w["camera"], w["spacetime"], w["integrator"], gg, w["plasma"], precision=precision)
    I = img[0].cpu().numpy()
    n = I.shape[0]
    vals = [A.criterion_map(I[by * b:(by + 1) * b, bx * b:(bx + 1) * b], kind)
            for by in range(n // b) for bx in range(n // b)]
    return _mid_threshold(np.concatenate([v.ravel() for v in vals]))


def _close(ib, ab, i1, a1, precision):
    """Block vs the same pixels of a single render: step counts and status
    equal (FP64) or nearly all equal (mixed), images within tolerance."""
    ib, ab, i1, a1 = (x.cpu().numpy() for x in (ib, ab, i1, a1))
    match = (ab[5] == a1[5]) & (ab[6] == a1[6])
    if precision == 0:
        assert match.all() and np.array_equal(ab[7], a1[7])
    else:
        assert match.mean() >= 0.9
    den = np.maximum(np.abs(i1[0]), 1e-3 * max(np.abs(i1[0]).max(), 1e-300))
    e = (np.abs(ib - i1) / den).max(axis=0)[match]
    assert e.size == 0 or e.max() <= (1e-12 if precision == 0 else 1e-4)
    return e.max() if e.size else 0.0


def _check_against_uniform(ctx, w, gg, levels, b, precision):
    n = int(w["camera"]["n"])
    for level, (blk, img, aux) in enumerate(levels):
        bl = blk.cpu().numpy()
        assert (bl[:, 0] == level).all()
        full_i, full_a = ctx.render(dict(w["camera"], n=n << level), w["spacetime"], w["integrator"], gg,
                                    w["plasma"], precision=precision)
        worst = 0.0
        for k, (_, bx, by) in enumerate(bl):
            sl = (slice(None), slice(by * b, by * b + b), slice(bx * b, bx * b + b))
            worst = max(worst, _close(img[k], aux[k], full_i[sl], full_a[sl], precision))
        _say("level", level, "blocks", len(bl), "E vs uniform render", worst)


def _check_decisions(w, levels, ad):
    from oracle import adaptive as A
    n, b = int(w["camera"]["n"]), int(ad["block"])
    for level in range(len(levels) - 1 if len(levels) > 1 else 0):
        blk, img, _ = levels[level]
        bl = [tuple(int(x) for x in r) for r in blk.cpu().numpy()]
        I = img[:, 0].cpu().numpy()
        flags = [A.refines(I[k], level, A.block_center(n, b, w["camera"]["width"], level, bx, by), ad)
                 for k, (_, bx, by) in enumerate(bl)]
        nxt = [tuple(int(x) for x in r) for r in levels[level + 1][0].cpu().numpy()]
        assert nxt == A.children(bl, flags), level
    if len(levels) < ad["max_level"] + 1 and levels:
        # the render stopped early: nothing refined on its last level
        blk, img, _ = levels[-1]
        I = img[:, 0].cpu().numpy()
        level = len(levels) - 1
        for k, (_, bx, by) in enumerate(blk.cpu().numpy()):
            assert not A.refines(I[k], level, A.block_center(n, b, w["camera"]["width"], level, bx, by), ad)


@pytest.mark.parametrize("precision", [0, 1])
def test_blocks_equal_uniform_renders(ctx, precision):
    from oracle import adaptive as A
    w, g, gg = _setup(ctx, "c2_256_pol", 16)
    thr = _root_threshold(ctx, w, gg, A.GRAD_ABS, 4, precision)
    ad = dict(block=4, max_level=2, frac=2 / 16, thr=[None, thr, None, None, None])
    levels = ctx.render_adaptive(w["camera"], w["spacetime"], w["integrator"], gg, w["plasma"], ad,
                                 precision=precision)
    torch.cuda.synchronize()
    _say("precision", precision, "blocks per level", [len(l[0]) for l in levels])
    assert len(levels) == 3 and len(levels[1][0]) > 0
    _check_against_uniform(ctx, w, gg, levels, 4, precision)
    _check_decisions(w, levels, ad)


@pytest.mark.parametrize("kind", [0, 1, 2, 3, 4])
def test_each_criterion_decides_like_the_oracle(ctx, kind):
    from oracle import adaptive as A
    w, g, gg = _setup(ctx, "c2_256_pol", 16)
    thr = _root_threshold(ctx, w, gg, kind, 4, 1)
    t = [None] * 5
    t[kind] = thr
    ad = dict(block=4, max_level=2, frac=3 / 16, thr=t)
    levels = ctx.render_adaptive(w["camera"], w["spacetime"], w["integrator"], gg, w["plasma"], ad, precision=1)
    torch.cuda.synchronize()
    _say("criterion", kind, "thr", thr, "blocks per level", [len(l[0]) for l in levels])
    _check_decisions(w, levels, ad)


def test_regions_decide_like_the_oracle(ctx):
    w, g, gg = _setup(ctx, "c2_256_pol", 16)
    wd = w["camera"]["width"]
    ad = dict(block=4, max_level=3, frac=1.0, thr=[None] * 5,
              regions=[(-0.3 * wd, 0.1 * wd, -0.2 * wd, 0.25 * wd, 2), (0.2 * wd, 0.5 * wd, 0.2 * wd, 0.5 * wd, 3)])
    levels = ctx.render_adaptive(w["camera"], w["spacetime"], w["integrator"], gg, w["plasma"], ad, precision=1)
    torch.cuda.synchronize()
    _say("regions: blocks per level", [len(l[0]) for l in levels])
    assert len(levels) == 4
    _check_decisions(w, levels, ad)


def test_adaptive_matches_oracle(ctx, oracle):
    from oracle import adaptive as A
    w, g, gg = _setup(ctx, "c1_64_unpol", 12)
    thr = _root_threshold(ctx, w, gg, A.GRAD_REL, 3, 0)
    ad = dict(block=3, max_level=2, frac=2 / 9, thr=[None, None, thr, None, None])
    levels = ctx.render_adaptive(w["camera"], w["spacetime"], w["integrator"], gg, w["plasma"], ad, precision=0)
    torch.cuda.synchronize()
    ol = A.render_adaptive(w["camera"], w["spacetime"], w["integrator"], g, w["plasma"], ad)
    _say("gpu blocks", [len(l[0]) for l in levels], "oracle blocks", [len(l[0]) for l in ol])
    assert len(levels) == len(ol) >= 2
    for (blk, img, aux), (oblk, oimg, oaux) in zip(levels, ol):
        assert np.array_equal(blk.cpu().numpy(), oblk)
        ig, ag = img.cpu().numpy(), aux.cpu().numpy()
        match = (ag[:, 5] == oaux[:, 5]) & (ag[:, 6] == oaux[:, 6])
        assert match.mean() >= 0.98
        I = oimg[:, 0]
        den = np.maximum(np.abs(I), 1e-3 * np.abs(I).max())
        e = (np.abs(ig - oimg) / den[:, None]).max(axis=1)
        _say("level", int(blk[0, 0]), "E_pix(matched)", e[match].max())
        assert e[match].max() <= TOL_FP64


def test_edge_cases(ctx):
    from paper_2203_15963_amd import blgpu
    w, g, gg = _setup(ctx, "c1_64_unpol", 8)
    args = (w["camera"], w["spacetime"], w["integrator"], gg, w["plasma"])
    # single-pixel blocks refined by value (gradients of one pixel are 0)
    img0, _ = ctx.render(*args, precision=1)
    thr = _mid_threshold(img0[0].cpu().numpy())
    ad = dict(block=1, max_level=2, frac=1.0, thr=[thr, None, None, None, None])
    levels = ctx.render_adaptive(*args, ad, precision=1)
    torch.cuda.synchronize()
    _say("single-pixel blocks per level", [len(l[0]) for l in levels])
    assert len(levels[0][0]) == 64 and len(levels) >= 2
    _check_against_uniform(ctx, w, gg, levels, 1, 1)
    _check_decisions(w, levels, ad)
    ad1 = dict(ad, thr=[None, 0.0, None, None, None])
    l1 = ctx.render_adaptive(*args, ad1, precision=1)
    assert len(l1) == 1   # no gradient inside one-pixel blocks: nothing refines
    # one block covering the image, level 0 only
    l0 = ctx.render_adaptive(*args, dict(block=8, max_level=0, frac=1.0), precision=1)
    assert len(l0) == 1
    _close(l0[0][1][0], l0[0][2][0], img0, ctx.render(*args, precision=1)[1], 1)
    # everything refines: level 1 is the whole 16 x 16 image in 16 blocks
    la = ctx.render_adaptive(*args, dict(block=4, max_level=1, frac=1.0, regions=[(-1e9, 1e9, -1e9, 1e9, 5)]),
                             precision=1)
    assert [len(l[0]) for l in la] == [4, 16]
    _check_against_uniform(ctx, w, gg, la, 4, 1)
    # capacity: 4 root blocks fit, their 16 children do not
    with pytest.raises(blgpu.BlError) as e:
        ctx.render_adaptive(*args, dict(block=4, max_level=1, frac=1.0, regions=[(-1e9, 1e9, -1e9, 1e9, 5)]),
                            max_blocks=10, precision=1)
    assert e.value.status == -4
    for bad in (dict(block=3, max_level=1, frac=1.0), dict(block=4, max_level=1, frac=0.0),
                dict(block=4, max_level=1, frac=0.5, thr=[float("nan"), None, None, None, None]),
                dict(block=4, max_level=18, frac=1.0)):
        with pytest.raises(blgpu.BlError) as e:
            ctx.render_adaptive(*args, bad, max_blocks=64, precision=1)
        assert e.value.status == -1


def test_bench_configuration_sampled(ctx, oracle):
    """The adaptive configuration the benchmark times (1024² SMR workload,
    root 256² in 8² blocks, two levels, absolute-gradient criterion at 2 % of
    the root's peak in 5 of 64 pixels, mixed form, FP32 grid) against the
    FP64 oracle on sampled pixels of every level, read through the block
    geometry (a level-l pixel is pixel (bx 8 + i, by 8 + j) of the 256 2^l
    image)."""
    from paper_2203_15963_amd import synth
    w = synth.workload("c3_1024_smr", n=1024)
    g = synth.make_grid(w["grid_args"])
    g32 = dict(g, prims=g["prims"].astype(np.float32))
    g64r = dict(g, prims=g32["prims"].astype(np.float64))
    gg = ctx.grid(g32)
    cam0 = dict(w["camera"], n=256)
    i0, _ = ctx.render(cam0, w["spacetime"], w["integrator"], gg, w["plasma"], precision=1)
    ad = dict(block=8, max_level=2, frac=5 / 64, thr=[None, 0.02 * float(i0[0].max()), None, None, None])
    levels = ctx.render_adaptive(cam0, w["spacetime"], w["integrator"], gg, w["plasma"], ad, precision=1)
    torch.cuda.synchronize()
    _say("bench configuration: blocks per level", [len(l[0]) for l in levels])
    assert len(levels) == 3
    rng = np.random.default_rng(21)
    for level, (blk, img, aux) in enumerate(levels):
        nl = 256 << level
        bl, ig, ag = blk.cpu().numpy(), img.cpu().numpy(), aux.cpu().numpy()
        ks = rng.choice(len(bl), size=min(12, len(bl)), replace=False)
        ij = rng.integers(0, 8, size=(len(ks), 2))
        pix = [(bl[k, 1] * 8 + i) + nl * (bl[k, 2] * 8 + j) for k, (i, j) in zip(ks, ij)]
        io, ao = oracle.render_pixels(dict(cam0, n=nl), w["spacetime"], w["integrator"], g64r, w["plasma"], pix)
        gi = np.array([ig[k, :, j, i] for k, (i, j) in zip(ks, ij)])
        ga = np.array([ag[k, :, j, i] for k, (i, j) in zip(ks, ij)])
        match = (ga[:, 5] == ao[:, 5]) & (ga[:, 6] == ao[:, 6])
        den = np.maximum(np.abs(io[:, 0]), 1e-3 * float(np.abs(ig[:, 0]).max()))
        e = (np.abs(gi - io) / den[:, None]).max(axis=1)
        _say("level", level, "sampled E_pix(matched)", e[match].max() if match.any() else 0.0,
             "mismatched", int((~match).sum()), "of", len(pix))
        assert (~match).sum() <= 1
        assert e[match].max() <= 1e-4


def test_adaptive_with_data_cuts(ctx):
    """Data cuts set on the context act on every level: each block equals the
    same pixels of a cut bl_render at that level's resolution."""
    w, g, gg = _setup(ctx, "c2_256_pol", 8)
    ctx.set_cuts({"sigma": (float("-inf"), 0.05), "r": (4.0, float("inf"))})
    try:
        ad = dict(block=4, max_level=2, frac=1.0, regions=[(-1e9, 0.0, -1e9, 1e9, 5)])
        levels = ctx.render_adaptive(w["camera"], w["spacetime"], w["integrator"], gg, w["plasma"], ad, precision=1)
        torch.cuda.synchronize()
        _say("cuts: blocks per level", [len(l[0]) for l in levels])
        assert [len(l[0]) for l in levels] == [4, 8, 32]
        _check_against_uniform(ctx, w, gg, levels, 4, 1)
    finally:
        ctx.set_cuts(None)


def test_adaptive_polarized_fp64_matches_oracle(ctx, oracle):
    from oracle import adaptive as A
    w, g, gg = _setup(ctx, "c2_256_pol", 8)
    # (with B = 2 the Laplacian criteria are 0 by the edge rule: use the gradient)
    ad = dict(block=2, max_level=1, frac=0.5, thr=[None, _root_threshold(ctx, w, gg, A.GRAD_ABS, 2, 0), None, None,
                                                    None])
    levels = ctx.render_adaptive(w["camera"], w["spacetime"], w["integrator"], gg, w["plasma"], ad, precision=0)
    torch.cuda.synchronize()
    ol = A.render_adaptive(w["camera"], w["spacetime"], w["integrator"], g, w["plasma"], ad)
    _say("polarized: gpu blocks", [len(l[0]) for l in levels], "oracle blocks", [len(l[0]) for l in ol])
    assert len(levels) == len(ol) == 2
    for (blk, img, aux), (oblk, oimg, oaux) in zip(levels, ol):
        assert np.array_equal(blk.cpu().numpy(), oblk)
        ig, ag = img.cpu().numpy(), aux.cpu().numpy()
        match = (ag[:, 5] == oaux[:, 5]) & (ag[:, 6] == oaux[:, 6])
        assert match.mean() >= 0.98
        den = np.maximum(np.abs(oimg[:, 0]), 1e-3 * np.abs(oimg[:, 0]).max())
        e = (np.abs(ig - oimg) / den[:, None]).max(axis=1)
        _say("polarized level", int(blk[0, 0]), "E_pix(matched)", e[match].max())
        assert e[match].max() <= TOL_FP64
