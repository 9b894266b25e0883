"""Pins of the oracle's radiative-transfer pieces: the unpolarized segment
solution (eq. unpolarized), the constant-coefficient polarized solution
against scipy's matrix exponential and closed forms (Faraday rotation,
conversion, dichroism, Kirchhoff), and the coordinate transport of the
coherency tensor against the geodesic flow."""
import math

import numpy as np
import pytest
from scipy.linalg import expm


def test_unpolarized_slab(oracle):
    # uniform slab: I = S (1 - e^-tau), any segmentation
    j, alpha = 3.0e-3, 0.2
    for nseg, total in [(1, 5.0), (7, 5.0), (64, 40.0)]:
        I = 0.0
        for _ in range(nseg):
            I = oracle.unpol_segment(I, j, alpha, total / nseg)
        exact = j / alpha * -math.expm1(-alpha * total)
        assert abs(I - exact) < 1e-14 * j / alpha
    # pure emission
    assert oracle.unpol_segment(2.0, 0.5, 0.0, 3.0) == 2.0 + 1.5
    # optically thick cap: Delta tau >= 100 gives j/alpha exactly
    assert oracle.unpol_segment(7.0, 2.0, 4.0, 25.0) == 0.5
    # incoming intensity is attenuated
    I = oracle.unpol_segment(1.0, 0.0, 0.5, 2.0)
    assert abs(I - math.exp(-1.0)) < 1e-15


def _Mmat(aI, aQ, aU, aV, rQ, rU, rV):
    return np.array([[aI, aQ, aU, aV],
                     [aQ, aI, rV, -rU],
                     [aU, -rV, aI, rQ],
                     [aV, rU, -rQ, aI]], dtype=float)


@pytest.mark.parametrize("seed", range(6))
def test_stokes_exact_vs_scipy_expm(oracle, seed):
    rng = np.random.default_rng(seed)
    c = rng.normal(size=7) * [1, 0.3, 0.3, 0.3, 2, 2, 2]
    c[0] = abs(c[0]) + 0.6
    M = _Mmat(*c)
    J = rng.normal(size=4)
    S0 = rng.normal(size=4)
    for s in [1e-3, 0.5, 3.0]:
        A = np.zeros((5, 5))
        A[:4, :4] = -M * s
        A[:4, 4] = J * s
        E = expm(A)
        ref = E[:4, :4] @ S0 + E[:4, 4]
        got = oracle.stokes_exact(S0, J, M, s)
        assert np.abs(got - ref).max() < 1e-12 * (1 + np.abs(ref).max())


def test_faraday_rotation(oracle):
    """rho_V alone rotates the polarization angle by rho_V s / 2."""
    rV, s = 0.37, 2.1
    S0 = np.array([1.0, 0.6, 0.0, 0.1])
    S = oracle.stokes_exact(S0, np.zeros(4), _Mmat(0, 0, 0, 0, 0, 0, rV), s)
    chi0 = 0.5 * math.atan2(S0[2], S0[1])
    chi = 0.5 * math.atan2(S[2], S[1])
    assert abs(chi - chi0 - 0.5 * rV * s) < 1e-14
    assert abs(math.hypot(S[1], S[2]) - 0.6) < 1e-14
    assert S[0] == pytest.approx(1.0, abs=1e-15) and S[3] == pytest.approx(0.1, abs=1e-15)


def test_faraday_conversion(oracle):
    """rho_Q alone rotates (U, V) at rate rho_Q: dU = -rho_Q V, dV = rho_Q U."""
    rQ, s = 0.8, 1.3
    S0 = np.array([1.0, 0.2, 0.5, 0.0])
    S = oracle.stokes_exact(S0, np.zeros(4), _Mmat(0, 0, 0, 0, rQ, 0, 0), s)
    assert S[1] == pytest.approx(0.2, abs=1e-15)
    assert S[2] == pytest.approx(0.5 * math.cos(rQ * s), abs=1e-14)
    assert S[3] == pytest.approx(0.5 * math.sin(rQ * s), abs=1e-14)


def test_dichroism(oracle):
    """alpha_Q alone: I +- Q decay at alpha_I +- alpha_Q."""
    aI, aQ, s = 0.9, 0.4, 1.7
    S0 = np.array([1.0, 0.3, 0.0, 0.0])
    S = oracle.stokes_exact(S0, np.zeros(4), _Mmat(aI, aQ, 0, 0, 0, 0, 0), s)
    assert S[0] + S[1] == pytest.approx((1.3) * math.exp(-(aI + aQ) * s), rel=1e-14)
    assert S[0] - S[1] == pytest.approx((0.7) * math.exp(-(aI - aQ) * s), rel=1e-14)


def test_kirchhoff_thick_limit(oracle):
    """With J = B M e_I (thermal emission), S tends to B e_I whatever the
    rotativities, and S = B e_I is a fixed point."""
    B = 2.5
    M = _Mmat(1.0, 0.3, 0.0, 0.2, 3.0, 0.0, 7.0)
    J = B * M[:, 0]
    S = oracle.stokes_exact(np.zeros(4), J, M, 60.0)
    assert np.abs(S - [B, 0, 0, 0]).max() < 1e-12
    S = oracle.stokes_exact(np.array([B, 0, 0, 0]), J, M, 0.7)
    assert np.abs(S - [B, 0, 0, 0]).max() < 1e-13


def test_transport_of_photon_momentum(oracle):
    """k^a k^b is parallel transported along the geodesic, so the transport
    right-hand side applied to N = k k must equal d(k k)/dl computed from the
    independently written geodesic right-hand side.  This fixes the relative
    sign of the two connection terms (the same sign on both)."""
    rng = np.random.default_rng(3)
    for a in [0.3, 0.9]:
        for _ in range(4):
            x = np.concatenate([[0.0], rng.uniform(-8, 8, 3)])
            if np.linalg.norm(x[1:]) < 3:
                continue
            k = np.concatenate([[-1.0], rng.normal(size=3)])
            y = np.concatenate([x, k])
            _, gi = oracle.metric(a, x)
            ku = gi @ k
            dR, dI = oracle.transport_rhs(a, y, np.outer(ku, ku), np.zeros((4, 4)))
            dy = oracle.geodesic_rhs(a, y)
            e = 1e-6
            kup = lambda yy: oracle.metric(a, yy[:4])[1] @ yy[4:]
            dku = (kup(y + e * dy) - kup(y - e * dy)) / (2 * e)
            ref = np.outer(dku, ku) + np.outer(ku, dku)
            assert np.abs(dR - ref).max() < 1e-7 * (1 + np.abs(ref).max())
            assert np.abs(dI).max() == 0.0


def test_transport_preserves_contractions(oracle):
    """For N = A B^T + B A^T (real) and antisymmetric imaginary parts, the
    transport is linear and keeps N Hermitian; with the metric it keeps the
    scalar g_ac g_bd N^ab N^cd stationary (metric compatibility)."""
    rng = np.random.default_rng(9)
    a = 0.8
    x = np.array([0.0, 5.0, -3.0, 2.0])
    k = np.array([-1.0, 0.3, -0.5, 0.8])
    y = np.concatenate([x, k])
    Ar, Br = rng.normal(size=4), rng.normal(size=4)
    Nr = np.outer(Ar, Br) + np.outer(Br, Ar)
    Ni = np.outer(Ar, Br) - np.outer(Br, Ar)
    dR, dI = oracle.transport_rhs(a, y, Nr, Ni)
    assert np.abs(dR - dR.T).max() < 1e-13 and np.abs(dI + dI.T).max() < 1e-13
    g, _ = oracle.metric(a, x)
    dy = oracle.geodesic_rhs(a, y)
    e = 1e-6
    gp = oracle.metric(a, x + e * dy[:4])[0]
    gm = oracle.metric(a, x - e * dy[:4])[0]
    dg = (gp - gm) / (2 * e)
    for N, dN in [(Nr, dR), (Ni, dI)]:
        s = np.einsum("ac,bd,ab,cd->", g, g, N, N)
        ds = (2 * np.einsum("ac,bd,ab,cd->", dg, g, N, N) + 2 * np.einsum("ac,bd,ab,cd->", g, g, dN, N))
        assert abs(ds) < 1e-7 * (1 + abs(s))
