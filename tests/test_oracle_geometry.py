"""Pins of the oracle's metric, geodesic right-hand side, connection and
Dormand-Prince tableau against facts fixed by the paper and by mathematics
(not by re-typing the oracle's own formulas)."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

SPINS = [0.0, 0.5, 0.9, 0.98]
RNG = np.random.default_rng(12345)


def _points(n=12):
    pts = []
    while len(pts) < n:
        x = RNG.uniform(-30, 30, 3)
        if np.linalg.norm(x) > 3.0:
            pts.append(np.concatenate([[0.0], x]))
    return pts


@pytest.mark.parametrize("a", SPINS)
def test_metric_inverse_and_determinant(oracle, a):
    # g g^-1 = 1; det g = -1 (sqrt(-g) = 1 holds for Kerr-Schild Cartesian form)
    for x in _points():
        g, gi = oracle.metric(a, x)
        assert np.abs(g @ gi - np.eye(4)).max() < 1e-14
        assert abs(np.linalg.det(g) + 1.0) < 1e-12


def _sks_matrix(a, r, th):
    # the spherical Kerr-Schild metric printed in the paper (section 2)
    f = 2.0 * r ** 3 / (r ** 4 + a * a * (r * math.cos(th)) ** 2)
    s = math.sin(th)
    return np.array([
        [-(1 - f), f, 0, -a * f * s * s],
        [f, 1 + f, 0, -a * (1 + f) * s * s],
        [0, 0, 2 * r / f, 0],
        [-a * f * s * s, -a * (1 + f) * s * s, 0, (r * r + a * a + a * a * f * s * s) * s * s]])


@pytest.mark.parametrize("a", SPINS)
def test_cks_metric_matches_printed_spherical_metric(oracle, a):
    """J^T g_CKS J equals the paper's spherical-KS matrix, with J the Jacobian
    of the paper's printed map x = sin(th)(r cos(ph) - a sin(ph)), ..."""
    for r, th, ph in [(3.0, 0.7, 0.3), (10.0, 1.2, 2.0), (2.5, 2.5, -1.0), (40.0, 0.1, 4.0)]:
        st, ct, sp, cp = math.sin(th), math.cos(th), math.sin(ph), math.cos(ph)
        x = np.array([0.0, st * (r * cp - a * sp), st * (r * sp + a * cp), r * ct])
        assert abs(oracle.ks_radius(a, *x[1:]) - r) < 1e-12 * r
        J = np.zeros((4, 4))
        J[0, 0] = 1.0
        J[1, 1:] = [st * cp, ct * (r * cp - a * sp), st * (-r * sp - a * cp)]
        J[2, 1:] = [st * sp, ct * (r * sp + a * cp), st * (r * cp - a * sp)]
        J[3, 1:] = [ct, -r * st, 0.0]
        g, _ = oracle.metric(a, x)
        assert np.allclose(J.T @ g @ J, _sks_matrix(a, r, th), rtol=1e-12, atol=1e-12)


def test_schwarzschild_and_flat_limits(oracle):
    x = np.array([0.0, 3.0, -4.0, 12.0])  # R = 13
    g, gi = oracle.metric(0.0, x)
    assert abs(g[0, 0] + (1 - 2 / 13.0)) < 1e-15          # g_tt = -(1 - 2M/r)
    assert abs(oracle.ks_radius(0.0, 3.0, -4.0, 12.0) - 13.0) < 1e-14
    g, gi = oracle.metric(0.9, x, flat=1)
    assert np.array_equal(g, np.diag([-1.0, 1, 1, 1])) and np.array_equal(gi, np.diag([-1.0, 1, 1, 1]))


@pytest.mark.parametrize("a", SPINS)
def test_metric_derivatives_vs_finite_differences(oracle, a):
    for x in _points(6):
        dg, dgi = oracle.metric_deriv(a, x)
        for c in range(3):
            e = 1e-5
            xp, xm = x.copy(), x.copy()
            xp[1 + c] += e
            xm[1 + c] -= e
            gp, gip = oracle.metric(a, xp)
            gm, gim = oracle.metric(a, xm)
            assert np.abs(dg[c] - (gp - gm) / (2 * e)).max() < 1e-8
            assert np.abs(dgi[c] - (gip - gim) / (2 * e)).max() < 1e-8


def _hamiltonian(oracle, a, y):
    _, gi = oracle.metric(a, y[:4])
    k = y[4:]
    return 0.5 * k @ gi @ k


@pytest.mark.parametrize("a", SPINS)
def test_rhs_is_hamiltons_equations(oracle, a):
    """eq. (geodesic) is Hamilton's equations of H = 1/2 g^ab k_a k_b:
    dx/dl = dH/dk, dk/dl = -dH/dx, checked by finite differences of H."""
    for x in _points(6):
        k = np.concatenate([[-1.0], RNG.normal(size=3)])
        y = np.concatenate([x, k])
        dy = oracle.geodesic_rhs(a, y)
        e = 1e-6
        for m in range(8):
            yp, ym = y.copy(), y.copy()
            yp[m] += e
            ym[m] -= e
            dH = (_hamiltonian(oracle, a, yp) - _hamiltonian(oracle, a, ym)) / (2 * e)
            if m < 4:   # dk_m/dl = -dH/dx^m  (zero for t)
                assert abs(dy[4 + m] + dH) < 1e-7 * (1 + abs(dH))
            else:       # dx^m/dl = dH/dk_m
                assert abs(dy[m - 4] - dH) < 1e-7 * (1 + abs(dH))


@pytest.mark.parametrize("a", [0.5, 0.98])
def test_christoffel_geodesic_consistency(oracle, a):
    """Along the Hamiltonian flow, d k^a/dl = -Gamma^a_bc k^b k^c: the
    connection (plain definition from d g) agrees with the independently
    written right-hand side."""
    for x in _points(5):
        k = np.concatenate([[-1.0], RNG.normal(size=3)])
        y = np.concatenate([x, k])
        dy = oracle.geodesic_rhs(a, y)
        e = 1e-6
        ku = lambda yy: oracle.metric(a, yy[:4])[1] @ yy[4:]
        dku = (ku(y + e * dy) - ku(y - e * dy)) / (2 * e)
        gam = oracle.christoffel(a, x)
        kup = ku(y)
        pred = -np.einsum("abc,b,c->a", gam, kup, kup)
        assert np.abs(dku - pred).max() < 1e-7 * (1 + np.abs(pred).max())


def test_christoffel_vs_finite_difference_definition(oracle):
    a = 0.7
    x = np.array([0.0, 4.0, -2.0, 3.0])
    e = 1e-5
    dgs = [np.zeros((4, 4))]
    for c in range(3):
        xp, xm = x.copy(), x.copy()
        xp[1 + c] += e
        xm[1 + c] -= e
        dgs.append((oracle.metric(a, xp)[0] - oracle.metric(a, xm)[0]) / (2 * e))
    d = np.array(dgs)  # d[mu, a, b]
    _, gi = oracle.metric(a, x)
    gam = 0.5 * (np.einsum("ad,bdc->abc", gi, d) + np.einsum("ad,cdb->abc", gi, d)
                 - np.einsum("ad,dbc->abc", gi, d))
    assert np.abs(gam - oracle.christoffel(a, x)).max() < 1e-8


# ------------------------------------------------------------------ tableau
def _golden_tableau():
    path = os.path.join(os.path.dirname(__file__), "golden", "dp_tableau.txt")
    rows = {"c": [], "A": [], "b5": None, "b4": None, "bm": None}
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        tag, rest = line.split(" ", 1)
        if tag == "c":
            parts = rest.split("|")
            rows["c"].append(Fraction(parts[0].strip()))
            rows["A"].append([Fraction(v) for v in parts[1].split()] if len(parts) > 1 else [])
        else:
            rows[tag] = [Fraction(v) for v in rest.split()]
    return rows


def test_tableau_matches_paper_and_order_conditions(oracle):
    T = _golden_tableau()
    c, A, b5, b4, bm = oracle.dp_tableau()
    for i in range(7):
        assert c[i] == float(T["c"][i])
        for j, v in enumerate(T["A"][i]):
            assert A[i, j] == float(v)
    assert list(b5) == [float(v) for v in T["b5"]]
    assert list(b4) == [float(v) for v in T["b4"]]
    assert list(bm) == [float(v) for v in T["bm"]]
    cs, As = T["c"], T["A"]
    # row sums equal the nodes
    for i in range(1, 7):
        assert sum(As[i]) == cs[i]
    # fifth-order quadrature conditions of b5 and fourth-order ones of b4
    for k in range(5):
        assert sum(b * ci ** k for b, ci in zip(T["b5"], cs)) == Fraction(1, k + 1)
    for k in range(4):
        assert sum(b * ci ** k for b, ci in zip(T["b4"], cs)) == Fraction(1, k + 1)
    # an order-4 tree condition: sum b_i a_ij c_j = 1/6
    s = sum(T["b5"][i] * sum(As[i][j] * cs[j] for j in range(i)) for i in range(7))
    assert s == Fraction(1, 6)


def test_midpoint_row_is_half_step(oracle):
    """The printed midpoint row sums to 1; with y_mid = y0 + (h/2) sum bm k it
    meets sum bm c^k = (1/2)^k/(k+1) for k <= 3 (fourth order at theta = 1/2)."""
    T = _golden_tableau()
    for k in range(4):
        s = sum(b * ci ** k for b, ci in zip(T["bm"], T["c"]))
        assert Fraction(1, 2) * s == Fraction(1, 2) ** (k + 1) / (k + 1)


def test_dense_quartic_reproduces_quartics(oracle):
    h = -0.7
    coef = RNG.normal(size=(5, 8))
    p = lambda th: sum(coef[q] * th ** q for q in range(5))
    dp = lambda th: sum(q * coef[q] * th ** (q - 1) for q in range(1, 5)) / h
    for th in [0.0, 0.1, 0.37, 0.5, 0.9, 1.0]:
        out = oracle.dense_quartic(p(0), p(1), dp(0), dp(1), p(0.5), h, th)
        assert np.abs(out - p(th)).max() < 1e-13
