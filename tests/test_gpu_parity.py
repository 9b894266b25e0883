"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

FP64 form: on every pixel whose accepted/rejected step counts equal the
oracle's, E_pix = max_Stokes |X_gpu - X_oracle| / max(I_oracle(pixel),
1e-3 max I_oracle) <= 1e-10.  Pixels whose counts differ (an accept/reject or
termination decision flipped by rounding: the GPU contracts to FMA, the oracle
does not) are counted and must stay rare.
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-10


def _say(*a):
    print("[gpu-parity]", *a, flush=True)
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


def _wl(name, n, **over):
    from paper_2203_15963_amd import synth
    w = synth.workload(name, n=n)
    for k, v in over.items():
        w[k].update(v)
    return w


_GRIDS = {}


def _grid(w):
    from paper_2203_15963_amd import synth
    key = repr(sorted(w["grid_args"].items()))
    if key not in _GRIDS:
        _GRIDS[key] = synth.make_grid(w["grid_args"])
    return _GRIDS[key]


def epix(img_g, img_o, counts_match):
    I = img_o[0]
    floor = 1e-3 * np.abs(I).max()
    den = np.maximum(np.abs(I), floor)
    if floor == 0:
        den = np.ones_like(I)
    e = (np.abs(img_g - img_o) / den).max(axis=0)
    return e[counts_match].max() if counts_match.any() else 0.0, e


def _mismatches(ag, ao, where):
    """Pixels whose accepted or rejected step counts (or status) differ from
    the oracle's, each with what differs."""
    bad = []
    for idx in np.flatnonzero((ag[:, 5] != ao[:, 5]) | (ag[:, 6] != ao[:, 6]) | (ag[:, 7] != ao[:, 7])):
        bad.append((int(where[idx]), {"n_acc": (ag[idx, 5], ao[idx, 5]), "n_rej": (ag[idx, 6], ao[idx, 6]),
                                      "status": (ag[idx, 7], ao[idx, 7])}))
    return bad


def _compare_render(ctx, oracle, w, pixels=None, precision=0, tol=TOL_FP64, max_mismatch=0, grid_f32=False):
    g = _grid(w)
    n = int(w["camera"]["n"])
    _say("render", w["camera"]["n"], w["plasma"]["polarized"], w["grid_args"].get("kind"), "precision", precision,
         "f32 grid" if grid_f32 else "")
    if grid_f32:
        # the device holds the float-rounded cells; the oracle reads the same values
        g32 = dict(g, prims=g["prims"].astype(np.float32))
        gg = ctx.grid(g32)
        g = dict(g, prims=g32["prims"].astype(np.float64))
    else:
        gg = ctx.grid(g)
    img, aux = ctx.render(w["camera"], w["spacetime"], w["integrator"], gg, w["plasma"], precision=precision)
    torch.cuda.synchronize()
    img, aux = img.cpu().numpy(), aux.cpu().numpy()
    if pixels is None:
        io, ao = oracle.render(w["camera"], w["spacetime"], w["integrator"], g, w["plasma"])
        match = (ao[5] == aux[5]) & (ao[6] == aux[6])
        ep, e = epix(img, io, match)
        bad = _mismatches(aux.reshape(10, -1).T, ao.reshape(10, -1).T, np.arange(n * n))
        _say("E_pix(matched)", ep, "mismatched", len(bad), "of", n * n, "max E_pix(all)", e.max(),
             "mismatched pixels:", [(p, float(e.reshape(-1)[p]), c) for p, c in bad[:10]])
        assert ep <= tol
        # pixels whose step counts differ (a decision flipped by rounding) are
        # listed above; their number is bounded by max_mismatch (0 unless a
        # test states otherwise)
        assert len(bad) <= max_mismatch * n * n
        # geodesic auxiliary maps on matched pixels
        for q in (0, 1, 2):
            assert np.abs(aux[q] - ao[q])[match].max() <= 1e-9 * (1 + np.abs(ao[q]).max())
        assert np.array_equal(aux[7][match], ao[7][match])
        assert np.array_equal(aux[9][match], ao[9][match])
        if precision == 0:
            assert np.array_equal(aux[8][match], ao[8][match])
        else:
            # the sigma cut is taken in FP32: a sample right at sigma_max may flip
            assert np.abs(aux[8] - ao[8])[match].sum() <= 1e-3 * ao[8].sum() + 2
        for q in (3, 4):
            d = np.abs(aux[q] - ao[q])[match]
            assert d.max() <= tol * (1e-30 + np.abs(ao[q]).max())
        return img, aux, io, ao
    pix = np.asarray(pixels)
    io, ao = oracle.render_pixels(w["camera"], w["spacetime"], w["integrator"], g, w["plasma"], pix)
    ig = img.reshape(4, -1)[:, pix].T
    ag = aux.reshape(10, -1)[:, pix].T
    match = (ag[:, 5] == ao[:, 5]) & (ag[:, 6] == ao[:, 6])
    full_max = np.abs(img[0]).max()
    den = np.maximum(np.abs(io[:, 0]), 1e-3 * full_max)
    e = (np.abs(ig - io) / den[:, None]).max(axis=1)
    bad = _mismatches(ag, ao, pix)
    _say("sampled E_pix(matched)", e[match].max() if match.any() else 0, "mismatched", len(bad),
         "of", len(pix), "mismatched pixels:", [(p, c) for p, c in bad[:10]])
    assert e[match].max() <= tol
    assert len(bad) <= max_mismatch * len(pix)
    return img, aux, io, ao


def test_camera_rays_match_oracle(ctx, oracle):
    for name, n in [("c1_64_unpol", 16), ("c3_1024_smr", 13)]:
        w = _wl(name, n)
        _say("camera", name, n)
        state, norm = ctx.camera_rays(w["camera"], w["spacetime"])
        torch.cuda.synchronize()
        state, norm = state.cpu().numpy(), norm.cpu().numpy()
        for p in range(n * n):
            y, nn = oracle.camera_ray(w["camera"], w["spacetime"], p % n, p // n)
            assert np.abs(state[p] - y).max() <= 1e-13 * np.abs(y).max()
            assert abs(norm[p] - nn) <= 1e-13 * nn


def test_geodesics_match_oracle(ctx, oracle):
    w = _wl("c1_64_unpol", 24)
    _say("geodesics 24^2")
    state, aux = ctx.trace_geodesics(w["camera"], w["spacetime"], w["integrator"])
    torch.cuda.synchronize()
    state, aux = state.cpu().numpy(), aux.cpu().numpy()
    n = 24
    mism = 0
    for p in range(n * n):
        t = oracle.trace_pixel(w["camera"], w["spacetime"], w["integrator"], p % n, p // n)
        i, j = p % n, p // n
        if aux[5, j, i] != t["n_acc"] or aux[6, j, i] != t["n_rej"]:
            mism += 1
            continue
        assert aux[7, j, i] == t["status"]
        assert np.abs(state[p] - t["y_end"]).max() <= 1e-9 * (1 + np.abs(t["y_end"]).max())
        assert abs(aux[2, j, i] - t["lambda"]) <= 1e-10 * t["lambda"]
        assert abs(aux[1, j, i] - t["s"]) <= 1e-10 * t["s"]
        assert abs(aux[0, j, i] - t["dt"]) <= 1e-10 * t["dt"]
    _say("geodesic count mismatches", mism)
    assert mism == 0


def test_samples_match_oracle(ctx, oracle):
    """Geodesic right-hand side, connection, coefficients and tetrad at
    random points in the polarized workload's grid."""
    w = _wl("c2_256_pol", 8)
    g = _grid(w)
    gg = ctx.grid(g)
    rng = np.random.default_rng(7)
    a = w["spacetime"]["a"]
    states, norms = [], []
    while len(states) < 400:
        x = rng.uniform(-45, 45, 3)
        if np.linalg.norm(x) < 3:
            continue
        k = np.concatenate([[-1.0], rng.normal(size=3)])
        gmat, gi = oracle.metric(a, np.concatenate([[0.0], x]))
        A, B, Cq = gi[0, 0], gi[0, 1:] @ k[1:], k[1:] @ gi[1:, 1:] @ k[1:]
        k[0] = (-B + math.sqrt(B * B - A * Cq)) / A
        states.append(np.concatenate([[0.0], x, k]))
        norms.append(2.3e11 / -k[0])
    states, norms = np.array(states), np.array(norms)
    _say("eval_samples 400")
    out = ctx.eval_samples(w["spacetime"], gg, w["plasma"], states, norms)
    torch.cuda.synchronize()
    out = out.cpu().numpy()
    nplasma = 0
    for s in range(len(states)):
        y = states[s]
        rhs = oracle.geodesic_rhs(a, y)
        assert np.abs(out[s, 0:8] - rhs).max() <= 1e-12 * (1 + np.abs(rhs).max())
        gam = oracle.christoffel(a, y[:4])
        ku = oracle.metric(a, y[:4])[1] @ y[4:]
        G = np.einsum("acd,c->ad", gam, ku)
        assert np.abs(out[s, 8:24].reshape(4, 4) - G).max() <= 1e-12 * (1 + np.abs(G).max())
        ref = oracle.sample_point(w["spacetime"], g, w["plasma"], y, norms[s])
        assert out[s, 52] == ref[28]
        if ref[28] == 0:
            continue
        nplasma += 1
        for m in range(8):
            assert abs(out[s, 24 + m] - ref[m]) <= 1e-11 * max(abs(ref[m]), 1e-300), (s, m, out[s, 24 + m], ref[m])
        assert np.allclose(out[s, 32:36], ref[8:12], rtol=1e-12, atol=0)
        assert np.abs(out[s, 36:52] - ref[12:28]).max() <= 1e-10 * (1 + np.abs(ref[12:28]).max())
    _say("plasma samples", nplasma)
    assert nplasma > 100


def test_render_rays_missing_the_grid(ctx, oracle):
    """A 120 M wide field around the grid (80 M and 100 M boxes): corner rays
    never meet the grid's box (no step is sampled, the walk has nothing to do
    and every step counts as one vacuum record) and others only graze it;
    polarized and unpolarized, FP64 and mixed.  (Impact parameters stay below
    the camera radius of 100 M, so every ray passes inside the camera sphere
    and escapes through it.)"""
    for name, pol in (("c1_64_unpol", 0), ("c2_256_pol", 1)):
        w = _wl(name, 12, camera={"width": 120.0})
        img, aux, io, ao = _compare_render(ctx, oracle, w)
        assert (ao[9] == ao[5]).sum() > 0, "no ray without a sampled step"
        assert (io[0] == 0).any()
        _compare_render(ctx, oracle, w, precision=1, tol=TOL_MIXED)


def test_render_unpolarized_uniform(ctx, oracle):
    _compare_render(ctx, oracle, _wl("c1_64_unpol", 20))


def test_render_polarized_uniform(ctx, oracle):
    _compare_render(ctx, oracle, _wl("c2_256_pol", 14))


@pytest.mark.parametrize("precision", [0, 1])
def test_render_polarized_sigma_cut(ctx, oracle, precision):
    """A low sigma cut (0.01) leaves vacuum holes inside the emitting region,
    so on most rays samples with and without a Stokes step alternate: the
    transfer then takes the full-N transport into a Stokes step (a state not
    packed by the previous sample) and unpacks a packed state before a sample
    without one, besides the packed path (about 160 such transitions on this
    12x12 image, counted with the oracle)."""
    w = _wl("c2_256_pol", 12, plasma=dict(sigma_max=0.01))
    _compare_render(ctx, oracle, w, precision=precision, tol=TOL_FP64 if precision == 0 else TOL_MIXED)


def _cut_set(w):
    """theta_e >= 3, 4 <= r <= 40 and the half of the grid on the camera's side
    of the plane through the origin orthogonal to the line of sight."""
    cam = w["camera"]
    nrm = (math.sin(cam["theta"]) * math.cos(cam["phi"]), math.sin(cam["theta"]) * math.sin(cam["phi"]),
           math.cos(cam["theta"]))
    return {"theta_e": (3.0, math.inf), "r": (4.0, 40.0),
            "plane": {"side": 1, "origin": (0.0, 0.0, 0.0), "normal": nrm}}


@pytest.mark.parametrize("precision", [0, 1])
def test_render_with_data_cuts(ctx, oracle, precision):
    """Data cuts (paper section 4.1) installed with bl_set_cuts against the
    oracle with the same cuts."""
    w = _wl("c2_256_pol", 12)
    cuts = _cut_set(w)
    w["plasma"]["cuts"] = cuts
    ctx.set_cuts(cuts)
    try:
        _compare_render(ctx, oracle, w, precision=precision, tol=TOL_FP64 if precision == 0 else TOL_MIXED)
    finally:
        ctx.set_cuts(None)


@pytest.mark.parametrize("precision", [0, 1])
def test_cuts_without_effect_reproduce_the_uncut_render(ctx, precision):
    """Installed cuts with infinite limits run the cut instantiation of the
    transfer kernels, whose results must equal the plain kernels' bit for bit
    (the FP64 one sits at the edge of the register file)."""
    w = _wl("c2_256_pol", 12)
    gg = ctx.grid(_grid(w))
    args = (w["camera"], w["spacetime"], w["integrator"], gg, w["plasma"])
    i0, a0 = ctx.render(*args, precision=precision)
    ctx.set_cuts({k: (-math.inf, math.inf) for k in ("rho", "ne", "p", "theta_e", "b", "sigma", "beta_inv", "r")})
    try:
        i1, a1 = ctx.render(*args, precision=precision)
    finally:
        ctx.set_cuts(None)
    torch.cuda.synchronize()
    assert torch.equal(i0, i1) and torch.equal(a0, a1)


def test_complementary_cuts_partition_the_samples(ctx):
    """The two sides of a plane cut hold every plasma sample exactly once."""
    w = _wl("c2_256_pol", 12)
    gg = ctx.grid(_grid(w))
    plane = _cut_set(w)["plane"]
    args = (w["camera"], w["spacetime"], w["integrator"], gg, w["plasma"])
    _, a0 = ctx.render(*args)
    halves = []
    for side in (1, -1):
        ctx.set_cuts({"plane": dict(plane, side=side)})
        halves.append(ctx.render(*args)[1])
    ctx.set_cuts(None)
    _, a1 = ctx.render(*args)
    torch.cuda.synchronize()
    n0, nh = a0[8].cpu().numpy(), [h[8].cpu().numpy() for h in halves]
    assert np.array_equal(nh[0] + nh[1], n0) and nh[0].sum() > 0 and nh[1].sum() > 0
    assert torch.equal(a0, a1)   # removing the cuts restores the uncut render


def test_set_cuts_rejects_bad_arguments(ctx):
    from paper_2203_15963_amd import blgpu
    with pytest.raises(blgpu.BlError):
        ctx.set_cuts({"rho": (math.nan, 1.0)})
    with pytest.raises(blgpu.BlError):
        ctx.set_cuts({"plane": {"side": 2, "origin": (0, 0, 0), "normal": (1, 0, 0)}})
    ctx.set_cuts(None)


def test_render_polarized_smr(ctx, oracle):
    _compare_render(ctx, oracle, _wl("c3_1024_smr", 11))


def test_overflow_path_matches(ctx, oracle):
    """With a tiny per-ray record slot every long ray is traced again into an
    extension slot; the image must not change."""
    w = _wl("c2_256_pol", 10, integrator=dict(record_cap=24))
    _compare_render(ctx, oracle, w)


def test_overflow_beyond_extension_slots(ctx, oracle):
    """More long rays than a chunk has extension slots (1024): the rest go to
    the single-wave fallback.  Both paths in one render, against the oracle."""
    w = _wl("c2_256_pol", 40, integrator=dict(record_cap=24))
    img, aux, io, ao = _compare_render(ctx, oracle, w)
    n_long = int((aux[5] + 2 > 24).sum())
    _say("rays beyond the record slot", n_long)
    assert n_long > 1024


def test_edge_cases(ctx, oracle):
    from paper_2203_15963_amd import blgpu
    # one pixel, ragged sizes
    _compare_render(ctx, oracle, _wl("c1_64_unpol", 1))
    _compare_render(ctx, oracle, _wl("c1_64_unpol", 7))
    # step cap: every ray stops with MAXSTEPS at the same place
    w = _wl("c1_64_unpol", 6, integrator=dict(max_steps=12))
    img, aux, io, ao = _compare_render(ctx, oracle, w)
    assert np.all(aux[7] == 3)
    # zero tolerances: steps shrink until they underflow
    w = _wl("c1_64_unpol", 3, integrator=dict(f_abs=0.0, f_rel=0.0))
    img, aux, io, ao = _compare_render(ctx, oracle, w)
    assert np.all(aux[7] == 4)
    # flat spacetime (even N: with odd N the central ray runs exactly through
    # the coordinate origin, where the Kerr-Schild radius is singular on the
    # ring disk and the result depends on the last bits of the arithmetic; the
    # oracle's FMA and non-FMA builds already differ there)
    w = _wl("c2_256_pol", 8, spacetime=dict(flat=1, r_in=0.0))
    _compare_render(ctx, oracle, w)
    # invalid arguments come back as status codes
    with pytest.raises(blgpu.BlError):
        ctx.render(dict(_wl("c1_64_unpol", 4)["camera"], n=0), _wl("c1_64_unpol", 4)["spacetime"],
                   {}, ctx.grid(_grid(_wl("c1_64_unpol", 4))), {})
    with pytest.raises(blgpu.BlError):
        ctx.trace_geodesics(_wl("c1_64_unpol", 4)["camera"], dict(a=1.5, r_in=1.0), {})


def test_full_size_sampled(ctx, oracle):
    """The benchmark workload at its full size (1024^2, SMR, polarized, FP64)
    against the oracle on sampled pixels."""
    w = _wl("c3_1024_smr", 1024)
    rng = np.random.default_rng(11)
    pix = rng.choice(1024 * 1024, size=48, replace=False)
    pix = np.concatenate([pix, [0, 1023, 1024 * 512 + 512, 1024 * 1024 - 1]])
    _compare_render(ctx, oracle, w, pixels=pix)


def test_deterministic(ctx):
    w = _wl("c2_256_pol", 12)
    gg = ctx.grid(_grid(w))
    a1, x1 = ctx.render(w["camera"], w["spacetime"], w["integrator"], gg, w["plasma"])
    a2, x2 = ctx.render(w["camera"], w["spacetime"], w["integrator"], gg, w["plasma"])
    torch.cuda.synchronize()
    assert torch.equal(a1, a2) and torch.equal(x1, x2)


# ------------------------------------------------------------ mixed precision
TOL_MIXED = 1e-4


def test_render_mixed_unpolarized(ctx, oracle):
    _compare_render(ctx, oracle, _wl("c1_64_unpol", 16), precision=1, tol=TOL_MIXED)


def test_render_mixed_polarized_smr(ctx, oracle):
    _compare_render(ctx, oracle, _wl("c3_1024_smr", 12), precision=1, tol=TOL_MIXED)


def test_render_mixed_fp32_grid(ctx, oracle):
    """Grid stored in FP32 (half the bytes): compare with the oracle run on the
    same float-rounded cell values."""
    w = _wl("c2_256_pol", 12)
    g = _grid(w)
    g32 = dict(g, prims=g["prims"].astype(np.float32))
    g64r = dict(g, prims=g32["prims"].astype(np.float64))
    n = 12
    gg = ctx.grid(g32)
    img, aux = ctx.render(w["camera"], w["spacetime"], w["integrator"], gg, w["plasma"], precision=1)
    torch.cuda.synchronize()
    img, aux = img.cpu().numpy(), aux.cpu().numpy()
    io, ao = oracle.render(w["camera"], w["spacetime"], w["integrator"], g64r, w["plasma"])
    match = (ao[5] == aux[5]) & (ao[6] == aux[6])
    ep, e = epix(img, io, match)
    _say("mixed fp32 grid E_pix", ep, "matched", int(match.sum()))
    assert ep <= TOL_MIXED and match.sum() == n * n


def test_full_size_sampled_mixed(ctx, oracle):
    """The benchmark configuration (1024^2 SMR polarized, mixed precision, FP32
    grid) against the FP64 oracle on sampled pixels."""
    w = _wl("c3_1024_smr", 1024)
    rng = np.random.default_rng(12)
    pix = rng.choice(1024 * 1024, size=48, replace=False)
    pix = np.concatenate([pix, [0, 1023, 1024 * 512 + 512, 1024 * 1024 - 1]])
    _compare_render(ctx, oracle, w, pixels=pix, precision=1, tol=TOL_MIXED, grid_f32=True)


def test_full_size_sampled_mixed_f64_grid(ctx, oracle):
    w = _wl("c3_1024_smr", 1024)
    rng = np.random.default_rng(13)
    pix = rng.choice(1024 * 1024, size=32, replace=False)
    _compare_render(ctx, oracle, w, pixels=pix, precision=1, tol=TOL_MIXED)


# ------------------------------------------------------------ batched renders
def _batch_small(seed=7, n_images=6, n_min=5, n_max=14, polarized=1):
    from paper_2203_15963_amd import synth
    return synth.batch_workload(n_images=n_images, n_min=n_min, n_max=n_max, seed=seed, polarized=polarized)


def _batch_grid(bw):
    return _grid({"grid_args": bw["grid_args"]})


def test_batch_matches_single_and_oracle(ctx, oracle):
    """Each image of a batch (uneven sizes, spins, inclinations, frequencies)
    equals its own bl_render and matches the oracle at the FP64 tolerance."""
    bw = _batch_small()
    g = _grid({"grid_args": bw["grid_args"]})
    gg = ctx.grid(g)
    outs = ctx.render_batch(bw["images"], bw["integrator"], gg, bw["plasma"], precision=0,
                            tuning_=dict(tile_w=8, tile_h=8, order=1, refill_min=4))
    torch.cuda.synchronize()
    for k, (cam, st) in enumerate(bw["images"]):
        ib, ab = outs[k][0].cpu().numpy(), outs[k][1].cpu().numpy()
        i1, a1 = ctx.render(cam, st, bw["integrator"], gg, bw["plasma"], precision=0)
        torch.cuda.synchronize()
        i1, a1 = i1.cpu().numpy(), a1.cpu().numpy()
        assert np.array_equal(ab[5:8], a1[5:8]) and np.array_equal(ab[8:10], a1[8:10])
        e_self = epix(ib, i1, np.ones(ib.shape[1:], bool))[0]
        io, ao = oracle.render(cam, st, bw["integrator"], g, bw["plasma"])
        match = (ao[5] == ab[5]) & (ao[6] == ab[6])
        e_or = epix(ib, io, match)[0]
        _say("batch image", k, "n", cam["n"], "a", st["a"], "nu", cam["nu_hz"], "E vs single", e_self,
             "E vs oracle", e_or, "mismatched", int((~match).sum()))
        assert e_self <= 1e-13
        assert e_or <= TOL_FP64 and (~match).sum() == 0


def test_batch_mixed_matches_oracle(ctx, oracle):
    bw = _batch_small(seed=8, n_images=4)
    g = _grid({"grid_args": bw["grid_args"]})
    g32 = dict(g, prims=g["prims"].astype(np.float32))
    g64r = dict(g, prims=g32["prims"].astype(np.float64))
    gg = ctx.grid(g32)
    outs = ctx.render_batch(bw["images"], bw["integrator"], gg, bw["plasma"], precision=1,
                            tuning_=dict(tile_w=16, tile_h=4))
    torch.cuda.synchronize()
    for k, (cam, st) in enumerate(bw["images"]):
        ib, ab = outs[k][0].cpu().numpy(), outs[k][1].cpu().numpy()
        io, ao = oracle.render(cam, st, bw["integrator"], g64r, bw["plasma"])
        match = (ao[5] == ab[5]) & (ao[6] == ab[6])
        e = epix(ib, io, match)[0]
        _say("mixed batch image", k, "n", cam["n"], "E", e)
        assert e <= TOL_MIXED and (~match).sum() == 0


def test_schedule_does_not_change_results(ctx):
    """Pixel tiles (ragged at the image edge), tiny chunks, wave caps and
    refill thresholds change only the schedule: the single-image render is
    bit-identical under every schedule."""
    w = _wl("c2_256_pol", 20)
    gg = ctx.grid(_grid(w))
    ref_i, ref_a = ctx.render(w["camera"], w["spacetime"], w["integrator"], gg, w["plasma"], precision=0)
    torch.cuda.synchronize()
    ref_i, ref_a = ref_i.cpu(), ref_a.cpu()
    default = ctx.get_tuning()
    schedules = [dict(tile_w=8, tile_h=8), dict(tile_w=64, tile_h=1, chunk_rays=64),
                 dict(tile_w=16, tile_h=4, transfer_waves_per_cu=1, refill_min=16, chunk_rays=128),
                 dict(refill_min=64, chunk_rays=192)]
    try:
        for t in schedules:
            ctx.set_tuning(t)
            i, a = ctx.render(w["camera"], w["spacetime"], w["integrator"], gg, w["plasma"], precision=0)
            torch.cuda.synchronize()
            _say("schedule", t)
            assert torch.equal(i.cpu(), ref_i) and torch.equal(a.cpu(), ref_a)
            # the batch kernels take per-lane image parameters: same steps, rounding-level differences
            (ib, ab), = ctx.render_batch([(w["camera"], w["spacetime"])], w["integrator"], gg, w["plasma"],
                                         precision=0)
            torch.cuda.synchronize()
            assert torch.equal(ab.cpu()[5:], ref_a[5:])
            assert epix(ib.cpu().numpy(), ref_i.numpy(), np.ones((20, 20), bool))[0] <= 1e-13
    finally:
        ctx.set_tuning(default)


def test_batch_overflow_path(ctx, oracle):
    """Rays longer than a small record slot go through the overflow kernel,
    which maps queued ray ids back to their images."""
    bw = _batch_small(seed=9, n_images=3, n_min=6, n_max=9)
    integ = dict(bw["integrator"], record_cap=24)
    g = _grid({"grid_args": bw["grid_args"]})
    gg = ctx.grid(g)
    outs = ctx.render_batch(bw["images"], integ, gg, bw["plasma"], precision=0, tuning_=dict(tile_w=8, tile_h=8))
    torch.cuda.synchronize()
    for k, (cam, st) in enumerate(bw["images"]):
        ib, ab = outs[k][0].cpu().numpy(), outs[k][1].cpu().numpy()
        io, ao = oracle.render(cam, st, bw["integrator"], g, bw["plasma"])
        match = (ao[5] == ab[5]) & (ao[6] == ab[6])
        e = epix(ib, io, match)[0]
        _say("overflow batch image", k, "E", e, "long rays", int((ab[5] + 2 > 24).sum()))
        assert e <= TOL_FP64


def test_autotune_returns_valid_schedule(ctx):
    bw = _batch_small(seed=10, n_images=5, n_min=8, n_max=24)
    gg = ctx.grid(_grid({"grid_args": bw["grid_args"]}))
    default = ctx.get_tuning()
    try:
        ref = ctx.render_batch(bw["images"], bw["integrator"], gg, bw["plasma"], precision=0)
        torch.cuda.synchronize()
        ref = [(i.cpu(), a.cpu()) for i, a in ref]
        best, ms = ctx.autotune(bw["images"], bw["integrator"], gg, bw["plasma"], precision=0, max_trials=6)
        _say("autotune", best, ms)
        assert ms > 0 and ctx.get_tuning() == best
        assert best["tile_w"] * best["tile_h"] in (0, 64)
        outs = ctx.render_batch(bw["images"], bw["integrator"], gg, bw["plasma"], precision=0)
        torch.cuda.synchronize()
        for (i, a), (ri, ra) in zip(outs, ref):
            assert torch.equal(i.cpu(), ri) and torch.equal(a.cpu(), ra)
    finally:
        ctx.set_tuning(default)
