"""Whole-pixel pins of the oracle in flat spacetime (paper section 4.2): a
uniform cube of plasma at rest must give the slab solutions of the transfer
equations along each chord, with the camera-frame polarization conventions."""
import math

import numpy as np
import pytest
from scipy.linalg import expm

M_E, M_P, C_LIGHT = 9.1093837015e-28, 1.67262192369e-24, 2.99792458e10
HALF = 10.0


def _setup(polarized, bdir=(0.0, 1.0, 0.0), n=8):
    theta, beta = 10.0, 10.0
    rt = (20.0 + 0.01) / 1.01
    rho = 1.0
    p = rho * theta * (M_E / M_P) * (1 + rt) / (0.5 * 2)
    B = math.sqrt(2 * p / beta) * np.asarray(bdir) / np.linalg.norm(bdir)
    prim = np.array([rho, p, 0, 0, 0, *B])
    grid = dict(bounds=np.array([[-HALF, HALF] * 3]).reshape(1, 6),
                prims=np.tile(prim, (1, 4, 4, 4, 1)), rho_unit=1e-17)
    cam = dict(r=100.0, theta=math.pi / 2, phi=0.0, width=30.0, n=n, nu_hz=230e9)
    st = dict(a=0.0, r_in=0.0, flat=1, mass_msun=4.152e6)
    integ = dict(f_abs=1e-8, f_rel=1e-8, ds_max=0.05)
    pl = dict(mu=0.5, ne_ni=1.0, r_high=20.0, r_low=1.0, sigma_max=1.0, polarized=polarized, interp=1)
    return cam, st, integ, grid, pl


def _pixel_offsets(n, w=30.0):
    return [((i - n / 2 + 0.5) * w / n, (j - n / 2 + 0.5) * w / n) for j in range(n) for i in range(n)]


def test_flat_unpolarized_cube(oracle):
    cam, st, integ, grid, pl = _setup(0)
    img, aux = oracle.render(cam, st, integ, grid, pl)
    # coefficients of the (uniform) plasma at any interior sample
    y, n = oracle.camera_ray(cam, st, 4, 4)
    yc = y.copy()
    yc[1] = 0.0
    c = oracle.sample_point(st, grid, pl, yc, n)
    jI, aI = c[0], c[3]
    L = 6.6743e-8 * 4.152e6 * 1.98841e33 / C_LIGHT ** 2
    nu3 = 230e9 ** 3
    for p, (ap, bp) in enumerate(_pixel_offsets(8)):
        j, i = divmod(p, 8)
        inside = abs(ap) < HALF and abs(bp) < HALF
        tau = aux[3, j, i]
        if not inside:
            assert img[0, j, i] == 0.0 and tau == 0.0
            continue
        # plasma length along the chord = 2 HALF up to one transfer piece
        Lp = tau / aI / L * n
        assert abs(Lp - 2 * HALF) <= integ["ds_max"] * 1.0001
        # composition of exact segment solutions with constant j, alpha
        assert img[0, j, i] == pytest.approx(nu3 * jI / aI * -math.expm1(-tau), rel=1e-12)
        assert aux[4, j, i] == pytest.approx(nu3 * jI * tau / aI, rel=1e-12)
        # flat-space light-crossing time and proper length from the pixel to the far side
        assert aux[0, j, i] == pytest.approx(aux[1, j, i], rel=1e-12)


@pytest.mark.parametrize("bdir,qsign", [((0.0, 1.0, 0.0), 1.0), ((0.0, 0.0, 1.0), -1.0)])
def test_flat_polarized_cube(oracle, bdir, qsign):
    """B along the horizontal H: thin synchrotron emission is polarized
    perpendicular to B, i.e. along the vertical V, so Q > 0 (and Q < 0 for B
    along V).  The Stokes vector equals the constant-coefficient solution over
    the plasma length, computed independently with scipy's expm."""
    cam, st, integ, grid, pl = _setup(1, bdir)
    img, aux = oracle.render(cam, st, integ, grid, pl)
    y, n = oracle.camera_ray(cam, st, 4, 4)
    yc = y.copy()
    yc[1] = 0.0
    c = oracle.sample_point(st, grid, pl, yc, n)
    jI, jQ, jV, aI, aQ, aV, rQ, rV = c[:8]
    M = np.array([[aI, aQ, 0, aV], [aQ, aI, rV, 0], [0, -rV, aI, rQ], [aV, 0, -rQ, aI]])
    J = np.array([jI, jQ, 0, jV])
    L = 6.6743e-8 * 4.152e6 * 1.98841e33 / C_LIGHT ** 2
    nu3 = 230e9 ** 3
    checked = 0
    for p, (ap, bp) in enumerate(_pixel_offsets(8)):
        j, i = divmod(p, 8)
        if not (abs(ap) < HALF and abs(bp) < HALF):
            assert np.all(img[:, j, i] == 0.0)
            continue
        s = aux[3, j, i] / aI            # physical plasma length
        A = np.zeros((5, 5))
        A[:4, :4] = -M * s
        A[:4, 4] = J * s
        S = expm(A)[:4, 4]
        # the fluid screen basis is (e1, e2) = (-z, y) for B along y; the camera
        # basis is (V, -H) = (z, -y): both vectors flip, leaving Q, U, V unchanged
        if bdir[2] != 0.0:   # B along z: fluid basis (e1, e2) = (y, z) vs camera (z, -y)
            S = np.array([S[0], -S[1], -S[2], S[3]])
        got = img[:, j, i] / nu3
        assert np.abs(got - S).max() < 1e-10 * S[0]
        assert np.sign(got[1]) == qsign
        checked += 1
    assert checked == 36
