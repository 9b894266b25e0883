"""Pins of the FP64 step-network oracle (oracle/mlp.py) to what the
definitions fix: BF16 rounding bit patterns, closed forms of the forward
pass, an explicit-loop evaluation, and finite differences of the loss."""
import math

import numpy as np
import pytest

from oracle import mlp as M


def _rand_model(rng, scale=0.5):
    m = rng.normal(0.0, scale, M.NMODEL)
    m[M.MU:M.SIG] = rng.normal(0.0, 1.0, M.NIN)
    m[M.SIG:M.NMODEL] = rng.uniform(0.5, 2.0, M.NIN)
    return m


def test_bf16_round_to_nearest_even():
    e = 2.0 ** -8   # half the BF16 spacing at 1
    vals = np.array([1.0, 1 + e, 1 + 3 * e, 1 + e + 2.0 ** -20, -(1 + 3 * e), 0.0, 2.0 ** -130, 65504.0])
    want = np.array([1.0, 1.0, 1 + 4 * e, 1 + 2 * e, -(1 + 4 * e), 0.0, 2.0 ** -130, 65536.0])
    assert np.array_equal(M.bf16_round(vals), want)
    assert np.isnan(M.bf16_round(np.array([np.nan])))[0]


def test_forward_constant_hidden_layers():
    """W1 = W2 = W3 = 0 and b1 = b2 = b3 = c: every hidden unit is silu(c), so
    y = silu(c) sum(w4) + b4 for any input."""
    rng = np.random.default_rng(1)
    m = _rand_model(rng)
    c = 0.37
    m[M.W1:M.B1] = 0.0
    m[M.W2:M.B2] = 0.0
    m[M.W3:M.B3] = 0.0
    m[M.B1:M.W2] = c
    m[M.B2:M.W3] = c
    m[M.B3:M.W4] = c
    X = rng.normal(size=(5, M.NIN))
    y, _ = M.forward(m, X)
    s = c / (1 + math.exp(-c))
    assert np.allclose(y, s * m[M.W4:M.B4].sum() + m[M.B4], rtol=1e-14, atol=1e-14)


def test_forward_single_path():
    """One path through the network: feature 3 -> unit 5 -> unit 7 -> unit 2
    with unit weights and zero biases gives y = w4[2] silu(silu(silu(x_n3)))."""
    m = np.zeros(M.NMODEL)
    m[M.SIG:M.NMODEL] = 1.0
    m[M.W1 + 5 * M.NIN + 3] = 1.0
    m[M.W2 + 7 * M.NH + 5] = 1.0
    m[M.W3 + 2 * M.NH + 7] = 1.0
    m[M.W4 + 2] = 1.5
    X = np.zeros((3, M.NIN))
    X[:, 3] = [-2.0, 0.5, 3.0]
    y, _ = M.forward(m, X)
    f = lambda z: z / (1 + np.exp(-z))
    # every other hidden unit is silu(0) = 0 at each layer
    assert np.allclose(y, 1.5 * f(f(f(X[:, 3]))), rtol=1e-14, atol=0)


def test_forward_matches_explicit_loops():
    rng = np.random.default_rng(2)
    m = _rand_model(rng)
    X = rng.normal(size=(3, M.NIN))
    y, _ = M.forward(m, X)
    p = M.unpack(m)
    sil = lambda z: z / (1 + math.exp(-z))
    for r in range(3):
        xn = [(X[r, i] - p["mu"][i]) / p["sig"][i] for i in range(M.NIN)]
        h = [sil(sum(p["W1"][o, i] * xn[i] for i in range(M.NIN)) + p["b1"][o]) for o in range(M.NH)]
        for W, b in ((p["W2"], p["b2"]), (p["W3"], p["b3"])):
            h = [sil(sum(W[o, i] * h[i] for i in range(M.NH)) + b[o]) for o in range(M.NH)]
        yr = sum(p["w4"][i] * h[i] for i in range(M.NH)) + p["b4"]
        assert abs(yr - y[r]) <= 1e-12 * (1 + abs(yr))


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    m = _rand_model(rng, 0.3)
    X = rng.normal(size=(20, M.NIN))
    t = rng.normal(size=20)
    _, _, g = M.loss_and_grad(m, X, t)
    # parameters from every block
    blocks = [(M.W1, M.B1), (M.B1, M.W2), (M.W2, M.B2), (M.B2, M.W3), (M.W3, M.B3), (M.B3, M.W4), (M.W4, M.B4),
              (M.B4, M.NPARAM)]
    idx = np.concatenate([rng.choice(np.arange(a, b), size=min(8, b - a), replace=False) for a, b in blocks])
    for k in idx:
        hstep = 1e-5 * max(1.0, abs(m[k]))
        mp, mm = m.copy(), m.copy()
        mp[k] += hstep
        mm[k] -= hstep
        fd = (M.loss_and_grad(mp, X, t)[1] - M.loss_and_grad(mm, X, t)[1]) / (2 * hstep)
        assert abs(fd - g[k]) <= 1e-6 * (abs(g[k]) + 1e-3 * np.abs(g).max()), (k, fd, g[k])


def test_bf16_emulation_stays_near_fp64():
    rng = np.random.default_rng(4)
    m = _rand_model(rng, 0.3)
    X = rng.normal(size=(64, M.NIN))
    t = rng.normal(size=64)
    y0, l0, g0 = M.loss_and_grad(m, X, t)
    y1, l1, g1 = M.loss_and_grad(m, X, t, bf16=True)
    assert np.abs(y1 - y0).max() <= 0.05 * (1 + np.abs(y0).max())
    assert np.linalg.norm(g1 - g0) <= 0.05 * np.linalg.norm(g0)
    assert not np.array_equal(g0, g1)


def test_features_of_a_state():
    f = M.features([1.0, 2.0, 3.0, 4.0, 5.0, 6.0, 7.0], -1.0, 0.5, -0.25, 0.0)
    assert np.allclose(f, [1, 2, 3, 4, -1, 5, 6, 7, 0.5, math.log(0.25), math.log(1e-10)])
