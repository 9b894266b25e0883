"""Pins of the oracle's data cuts (paper section 4.1, Data Cuts): limits on
rho, n_e, p, Theta_e, B, sigma, beta^-1 and r, and a half-space plane.

- each limit acts on its own quantity: at a plasma sample, an upper limit just
  below the sample's value makes it vacuum and one just above does not (a
  limit wired to another quantity, orders of magnitude apart, fails this);
- complementary cuts partition the samples of an image: the sample counts of
  the two halves add up exactly to the uncut count, and the additive
  auxiliary sums (I_j and tau) to rounding;
- infinite limits change nothing, and a limit that excludes every sample
  leaves a vacuum image with unchanged geodesic maps."""
import math

import numpy as np
import pytest

from paper_2203_15963_amd import synth

INF = math.inf
KEYS = ("rho", "ne", "p", "theta_e", "b", "sigma", "beta_inv", "r")


@pytest.fixture(scope="module")
def wl():
    w = synth.workload("c2_256_pol", n=6)
    return w, synth.make_grid(w["grid_args"])


def _render(oracle, w, g, cuts=None):
    pl = dict(w["plasma"], cuts=cuts) if cuts is not None else w["plasma"]
    return oracle.render(w["camera"], w["spacetime"], w["integrator"], g, pl)


def _plasma_sample(oracle, w, g):
    """A state inside the emitting region with the sample's quantities."""
    y, n = oracle.camera_ray(w["camera"], w["spacetime"], 3, 3)
    for s in np.linspace(0.2, 0.8, 61):
        # points along the line from the camera towards the origin
        x = np.asarray(y[1:4]) * (1.0 - s)
        yy = np.array([0.0, *x, *y[4:]])
        out = oracle.sample_point(w["spacetime"], g, w["plasma"], yy, n)
        if out[28] == 1.0:
            _, prim = oracle.grid_sample(g, x, 1)
            rho, p, sigma = prim[0], prim[1], out[29]
            vals = dict(rho=rho, ne=out[8], p=p, theta_e=out[9], b=out[10], sigma=sigma,
                        beta_inv=sigma * rho / (2.0 * p),
                        r=oracle.ks_radius(w["spacetime"]["a"], *x))
            return yy, n, vals
    raise AssertionError("no plasma sample found")


@pytest.mark.parametrize("key", KEYS)
def test_each_limit_acts_on_its_quantity(oracle, wl, key):
    w, g = wl
    y, n, vals = _plasma_sample(oracle, w, g)
    q = vals[key]
    assert q > 0
    for hi, plasma in ((q * (1 - 1e-9), 0.0), (q * (1 + 1e-9), 1.0)):
        out = oracle.sample_point(w["spacetime"], g, dict(w["plasma"], cuts={key: (-INF, hi)}), y, n)
        assert out[28] == plasma, (key, q, hi)
    for lo, plasma in ((q * (1 + 1e-9), 0.0), (q * (1 - 1e-9), 1.0)):
        out = oracle.sample_point(w["spacetime"], g, dict(w["plasma"], cuts={key: (lo, INF)}), y, n)
        assert out[28] == plasma, (key, q, lo)


def test_plane_side(oracle, wl):
    w, g = wl
    y, n, _ = _plasma_sample(oracle, w, g)
    x = y[1:4]
    nrm = (1.0, 0.0, 0.0)
    for side in (1, -1):
        for x0 in (x[0] - 1e-6, x[0] + 1e-6):
            cuts = {"plane": {"side": side, "origin": (x0, 0.0, 0.0), "normal": nrm}}
            out = oracle.sample_point(w["spacetime"], g, dict(w["plasma"], cuts=cuts), y, n)
            d = x[0] - x0
            assert out[28] == (0.0 if (side > 0 and d < 0) or (side < 0 and d > 0) else 1.0)


def test_infinite_limits_change_nothing(oracle, wl):
    w, g = wl
    i0, a0 = _render(oracle, w, g)
    i1, a1 = _render(oracle, w, g, {k: (-INF, INF) for k in KEYS})
    assert np.array_equal(i0, i1) and np.array_equal(a0, a1)


def _check_partition(full, parts):
    (i0, a0), halves = full, parts
    ns = sum(a[8] for _, a in halves)
    assert np.array_equal(ns, a0[8])
    assert all(a[8].sum() > 0 for _, a in halves)   # both halves hold samples
    for q in (3, 4):   # tau and I_j
        s = sum(a[q] for _, a in halves)
        assert np.allclose(s, a0[q], rtol=1e-11, atol=1e-300)


def test_complementary_plane_cuts_partition_the_samples(oracle, wl):
    """The plane through the origin orthogonal to the line of sight splits
    the emitting region into a near and a far half."""
    w, g = wl
    cam = w["camera"]
    nrm = (math.sin(cam["theta"]) * math.cos(cam["phi"]), math.sin(cam["theta"]) * math.sin(cam["phi"]),
           math.cos(cam["theta"]))
    full = _render(oracle, w, g)
    halves = [_render(oracle, w, g, {"plane": {"side": s, "origin": (0.0, 0.0, 0.0), "normal": nrm}})
              for s in (1, -1)]
    _check_partition(full, halves)


@pytest.mark.parametrize("key,t", [("beta_inv", 0.05), ("r", 8.0), ("theta_e", 3.0)])
def test_complementary_limits_partition_the_samples(oracle, wl, key, t):
    w, g = wl
    full = _render(oracle, w, g)
    halves = [_render(oracle, w, g, {key: (-INF, t)}), _render(oracle, w, g, {key: (t, INF)})]
    _check_partition(full, halves)


def test_cut_excluding_everything_gives_vacuum(oracle, wl):
    w, g = wl
    i0, a0 = _render(oracle, w, g)
    i1, a1 = _render(oracle, w, g, {"rho": (-INF, 0.0)})
    assert np.all(i1 == 0.0) and np.all(a1[[3, 4, 8]] == 0.0)
    assert np.array_equal(a1[[0, 1, 2, 5, 6, 7]], a0[[0, 1, 2, 5, 6, 7]])
