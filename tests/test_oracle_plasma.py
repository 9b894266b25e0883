"""Pins of the oracle's grid sampling, plasma state, tetrad and thermal
coefficients (structure and limits; the fitting formulas themselves are not
printed in the paper, so their physical values are parity-unpinned)."""
import math

import numpy as np
import pytest
from scipy.special import kve

C_LIGHT = 2.99792458e10
H_PLANCK = 6.62607015e-27
K_B = 1.380649e-16
M_E = 9.1093837015e-28
M_P = 1.67262192369e-24
Q_E = 4.80320471e-10


@pytest.mark.parametrize("n", [0, 1, 2])
def test_bessel_vs_scipy(oracle, n):
    for x in np.logspace(-3, 2.5, 40):
        ref = kve(n, x)
        assert abs(oracle.bessel_k_scaled(n, x) - ref) < 2e-14 * ref


def planck(nu, thetae):
    return 2 * H_PLANCK * nu ** 3 / C_LIGHT ** 2 / math.expm1(H_PLANCK * nu / (thetae * M_E * C_LIGHT ** 2))


CASES = [(1e6, 10.0, 30.0, 230e9, 0.3), (5e5, 3.0, 80.0, 86e9, -0.7), (2e7, 40.0, 5.0, 690e9, 0.95),
         (1e4, 1.0, 200.0, 1e10, 0.01)]


@pytest.mark.parametrize("ne,th,B,nu,c", CASES)
def test_kirchhoff_and_field_reversal(oracle, ne, th, B, nu, c):
    co = oracle.thermal_coeffs(ne, th, B, nu, c)
    bnu = planck(nu, th)
    for jj, aa in [(0, 3), (1, 4), (2, 5)]:
        assert co[aa] == pytest.approx(co[jj] / bnu, rel=1e-13)
    rev = oracle.thermal_coeffs(ne, th, B, nu, -c)
    # reversing B (cos theta -> -cos theta) flips exactly the circular terms
    for m in (0, 1, 3, 4, 6):
        assert rev[m] == pytest.approx(co[m], rel=1e-14)
    for m in (2, 5, 7):
        assert rev[m] == pytest.approx(-co[m], rel=1e-14)
    assert co[0] > 0 and co[3] > 0


def test_polarization_fractions_bounded(oracle):
    for th in [1.0, 3.0, 10.0, 30.0, 100.0]:
        for B in [1.0, 10.0, 100.0]:
            for c in [0.05, 0.5, 0.9]:
                for nu in [86e9, 230e9, 690e9]:
                    co = oracle.thermal_coeffs(1e6, th, B, nu, c)
                    nuc = 1.5 * Q_E * B / (2 * math.pi * M_E * C_LIGHT) * math.sqrt(1 - c * c) * th * th
                    if nu / nuc < 1.0:
                        continue   # fits are meant for x = nu/nu_c >~ 1
                    assert 0 <= co[1] <= co[0]
                    assert abs(co[2]) <= co[0]


def test_zero_field_and_high_frequency_limit(oracle):
    assert np.all(oracle.thermal_coeffs(1e6, 10.0, 0.0, 230e9, 0.5) == 0)
    assert np.all(oracle.thermal_coeffs(1e6, 10.0, 10.0, 230e9, 1.0) == 0)   # k parallel to B
    # large x: the emissivity approaches the ultra-relativistic thermal form
    # sqrt(2) pi e^2 n nu_s (X^1/2 + 2^(11/12) X^1/6)^2 exp(-X^1/3) / (3 K2(1/Theta) c)
    # (Leung et al. 2011, X = nu/nu_s, nu_s = 2/9 nu_B Theta^2 sin(theta)) within a few percent
    ne, th, B, c = 1e6, 20.0, 10.0, 0.4
    s = math.sqrt(1 - c * c)
    nuB = Q_E * B / (2 * math.pi * M_E * C_LIGHT)
    for x in [10.0, 100.0, 1000.0]:
        nu = x * 1.5 * nuB * s * th * th
        nus = 2.0 / 9.0 * nuB * th * th * s
        X = nu / nus
        k2 = kve(2, 1 / th) * math.exp(-1 / th)
        ref = (math.sqrt(2) * math.pi * Q_E ** 2 * ne * nus * (X ** 0.5 + 2 ** (11 / 12) * X ** (1 / 6)) ** 2
               * math.exp(-X ** (1 / 3)) / (3 * k2 * C_LIGHT))
        assert oracle.thermal_coeffs(ne, th, B, nu, c)[0] == pytest.approx(ref, rel=0.05)


def test_faraday_rotativity_cold_plasma_limit(oracle):
    """As Theta_e -> 0 the thermal Faraday rotativity must reduce to the
    cold-plasma one, rho_V = omega_p^2 omega_B cos(theta) / (c omega^2): the
    plane of polarization turns by d chi / ds = rho_V / 2 =
    2 pi e^3 n B cos(theta) / (m^2 c^2 omega^2) (Rybicki & Lightman, Faraday
    rotation in a cold magnetized plasma).  The relativistic corrections of
    the fit (the Bessel ratio and the X correction) are O(Theta_e)."""
    for ne, B, nu, c in [(1e6, 10.0, 230e9, 0.6), (3e4, 80.0, 86e9, -0.3), (1e7, 2.0, 690e9, 0.95)]:
        omega = 2 * math.pi * nu
        chi_rate = 2 * math.pi * Q_E ** 3 * ne * B * c / (M_E ** 2 * C_LIGHT ** 2 * omega ** 2)
        wp2 = 4 * math.pi * ne * Q_E ** 2 / M_E
        wb = Q_E * B / (M_E * C_LIGHT)
        cold = wp2 * wb * c / (C_LIGHT * omega ** 2)
        assert cold == pytest.approx(2 * chi_rate, rel=1e-12)
        prev = None
        for th in [3e-3, 1e-3, 3e-4]:
            rv = oracle.thermal_coeffs(ne, th, B, nu, c)[7]
            assert abs(rv / cold - 1.0) <= 3.0 * th, (th, rv / cold)
            # hotter electrons rotate less (relativistic suppression)
            if prev is not None:
                assert abs(rv) > abs(prev)
            prev = rv


# ------------------------------------------------------------------ grid
def _block_grid(nb_cells=(6, 5, 4), bounds=(-3, 3, -2, 3, -1, 1), f=None):
    nx, ny, nz = nb_cells
    prims = np.zeros((1, nz, ny, nx, 8))
    x0, x1, y0, y1, z0, z1 = bounds
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                xc = x0 + (i + 0.5) * (x1 - x0) / nx
                yc = y0 + (j + 0.5) * (y1 - y0) / ny
                zc = z0 + (k + 0.5) * (z1 - z0) / nz
                prims[0, k, j, i] = f(xc, yc, zc)
    return dict(bounds=np.array([bounds], float), prims=prims, rho_unit=1e-17)


def test_trilinear_reproduces_linear_fields(oracle):
    lin = lambda x, y, z: np.array([1 + 0.3 * x - 0.2 * y + 0.7 * z + 0.1 * m for m in range(8)])
    g = _block_grid(f=lin)
    rng = np.random.default_rng(1)
    for _ in range(50):
        # stay half a cell inside the faces, where no clamping happens
        p = np.array([rng.uniform(-2.5, 2.5), rng.uniform(-1.5, 2.5), rng.uniform(-0.75, 0.75)])
        b, v = oracle.grid_sample(g, p, interp=1)
        assert b == 0
        assert np.abs(v - lin(*p)).max() < 1e-13
    # within half a cell of a face the value is held at the face cell centre
    b, v = oracle.grid_sample(g, np.array([-2.9, 0.0, 0.0]), interp=1)
    assert np.abs(v - lin(-2.5, 0.0, 0.0)).max() < 1e-13
    # outside: vacuum
    assert oracle.grid_sample(g, np.array([3.0, 0.0, 0.0]))[0] == -1
    assert oracle.grid_sample(g, np.array([0.0, -2.01, 0.0]))[0] == -1


def test_nearest_cell(oracle):
    g = _block_grid(f=lambda x, y, z: np.array([x, y, z, 0, 0, 0, 0, 0]))
    b, v = oracle.grid_sample(g, np.array([0.99, 2.99, -0.49]), interp=0)
    assert np.allclose(v[:3], [0.5, 2.5, -0.25])
    b, v = oracle.grid_sample(g, np.array([-3.0, -2.0, -1.0]), interp=0)   # lower faces belong to the block
    assert b == 0 and np.allclose(v[:3], [-2.5, -1.5, -0.75])


def test_smr_block_search_and_prolongation(oracle):
    """A two-level grid whose fine blocks copy their parent cells returns the
    same nearest-cell values as the uniform coarse grid."""
    from paper_2203_15963_amd import synth
    coarse = synth.smr_grid(root=4, cells=4, half_width=8.0, a=0.5, refine_radius=None)
    fine = synth.smr_grid(root=4, cells=4, half_width=8.0, a=0.5, refine_radius=5.0)
    assert len(fine["bounds"]) > len(coarse["bounds"])
    # overwrite fine data by prolongation of the coarse cells
    for b, bd in enumerate(fine["bounds"]):
        for k in range(4):
            for j in range(4):
                for i in range(4):
                    c = np.array([bd[0] + (i + 0.5) * (bd[1] - bd[0]) / 4, bd[2] + (j + 0.5) * (bd[3] - bd[2]) / 4,
                                  bd[4] + (k + 0.5) * (bd[5] - bd[4]) / 4])
                    _, v = oracle.grid_sample(coarse, c, interp=0)
                    fine["prims"][b, k, j, i] = v
    rng = np.random.default_rng(5)
    for _ in range(200):
        p = rng.uniform(-7.99, 7.99, 3)
        bc, vc = oracle.grid_sample(coarse, p, interp=0)
        bf, vf = oracle.grid_sample(fine, p, interp=0)
        assert bc >= 0 and bf >= 0
        assert np.array_equal(vc, vf)
        bd = fine["bounds"][bf]
        assert bd[0] <= p[0] < bd[1] and bd[2] <= p[1] < bd[3] and bd[4] <= p[2] < bd[5]


# --------------------------------------------------------- plasma state
def _const_grid(prim, half=20.0):
    return dict(bounds=np.array([[-half, half, -half, half, -half, half]]),
                prims=np.tile(np.asarray(prim, float), (1, 2, 2, 2, 1)), rho_unit=1e-17)


PL = dict(mu=0.5, ne_ni=1.0, r_high=20.0, r_low=1.0, sigma_max=1.0, polarized=1, interp=1)


def test_plasma_state_flat_rest_frame(oracle):
    """Flat space, fluid at rest, beta = 10: n_e, Theta_e (the R_high
    prescription inverted by the input recipe), B in gauss, frequency."""
    theta_target, beta = 10.0, 10.0
    rt = (20.0 + 0.01) / 1.01
    rho = 2.0
    p = rho * theta_target * (M_E / M_P) * (1 + rt) / (0.5 * 2)
    Bc = math.sqrt(2 * p / beta)
    gr = _const_grid([rho, p, 0, 0, 0, 0, Bc, 0])
    st = dict(a=0.0, r_in=0.0, flat=1)
    y = np.array([0.0, 1.0, 0.5, -0.3, -1.0, 1.0, 0.0, 0.0])   # k along +x, B along y
    out = oracle.sample_point(st, gr, PL, y, 230e9)
    assert out[28] == 1.0
    assert out[8] == pytest.approx(rho * 1e-17 / M_P, rel=1e-14)
    assert out[9] == pytest.approx(theta_target, rel=1e-13)
    assert out[10] == pytest.approx(Bc * C_LIGHT * math.sqrt(4 * math.pi * 1e-17), rel=1e-14)
    assert out[11] == pytest.approx(230e9, rel=1e-15)
    e = out[12:28].reshape(4, 4)
    assert np.allclose(e[0], [1, 0, 0, 0]) and np.allclose(e[3], [0, 1, 0, 0])
    assert np.allclose(e[2], [0, 0, 1, 0]) and np.allclose(e[1], [0, 0, 0, -1])
    # sigma cut
    gr2 = _const_grid([rho, p, 0, 0, 0, 0, 10 * math.sqrt(rho), 0])
    assert oracle.sample_point(st, gr2, PL, y, 230e9)[28] == 0.0


def test_doppler_and_tetrad_in_kerr(oracle):
    a = 0.7
    st = dict(a=a, r_in=0.0, flat=0)
    rng = np.random.default_rng(2)
    for _ in range(10):
        ut = rng.normal(size=3) * 0.5
        B = rng.normal(size=3) * 0.05
        gr = _const_grid([1.0, 0.01, *ut, *B])
        x = np.concatenate([[0.0], rng.uniform(-10, 10, 3)])
        if np.linalg.norm(x[1:]) < 4:
            continue
        k = np.concatenate([[-1.0], rng.normal(size=3)])
        g, gi = oracle.metric(a, x)
        # make k null by solving for k_t
        A, Bq, Cq = gi[0, 0], gi[0, 1:] @ k[1:], k[1:] @ gi[1:, 1:] @ k[1:]
        k[0] = (-Bq + math.sqrt(Bq * Bq - A * Cq)) / A
        y = np.concatenate([x, k])
        out = oracle.sample_point(st, gr, dict(PL, sigma_max=1e30), y, 1e11)
        e = out[12:28].reshape(4, 4)
        G = e @ g @ e.T
        assert np.abs(G - np.diag([-1.0, 1, 1, 1])).max() < 1e-12
        ku = gi @ k
        omega = -(k @ e[0])
        assert out[11] == pytest.approx(1e11 * omega, rel=1e-13)
        # e3 is the photon direction in the fluid frame; e1, e2 span the screen
        assert np.allclose(ku, omega * (e[0] + e[3]), rtol=1e-12, atol=1e-12 * np.abs(ku).max())
        # right-handed screen basis (e1 x e2 = e3): det(e^a_(b)) = +1 / sqrt(-g) = +1
        assert np.linalg.det(e) == pytest.approx(1.0, abs=1e-10)
