"""Pins of the oracle's averaged quantities (paper section 4.6, Auxiliary
Images): <q>_lambda, <q>_Ij and <q>_tau for q = rho, n_e, p, Theta_e, B,
sigma, beta^-1, on a uniform cube of plasma at rest in flat spacetime, where
they have closed forms: along a ray q is constant, so <q>_Ij = q,
<q>_tau = q (1 - e^-tau) (the relaxation d<q>/dtau = q - <q> from 0), and
<q>_lambda lambda = q times the affine length inside the plasma, which tau
fixes through the constant absorptivity.  The q are computed here from the
cube's defining constants (not from the oracle), which pins the order of the
21 maps as well."""
import math

import numpy as np
import pytest

from test_oracle_pipeline import C_LIGHT, HALF, M_P, _pixel_offsets, _setup


def _quantities(grid, pl):
    prim = grid["prims"][0, 0, 0, 0]
    rho, p = prim[0], prim[1]
    b2 = float(np.dot(prim[5:8], prim[5:8]))   # plasma at rest in flat spacetime: b = B
    ne = rho * grid["rho_unit"] / (pl["mu"] * M_P) / (1.0 + 1.0 / pl["ne_ni"])
    B = math.sqrt(b2) * C_LIGHT * math.sqrt(4.0 * math.pi * grid["rho_unit"])
    return [rho, ne, p, 10.0, B, b2 / rho, b2 / (2.0 * p)]   # Theta_e = 10 by construction


@pytest.mark.parametrize("polarized", [0, 1])
def test_averages_on_a_uniform_cube(oracle, polarized):
    cam, st, integ, grid, pl = _setup(polarized)
    img, aux, avg = oracle.render(cam, st, integ, grid, pl, averages=True)
    q = _quantities(grid, pl)
    y, n = oracle.camera_ray(cam, st, 4, 4)
    yc = y.copy()
    yc[1] = 0.0
    c = oracle.sample_point(st, grid, pl, yc, n)
    aI = c[3]
    assert c[9] == pytest.approx(10.0, rel=1e-12)   # the cube's Theta_e
    L = 6.6743e-8 * 4.152e6 * 1.98841e33 / C_LIGHT ** 2
    for p, (ap, bp) in enumerate(_pixel_offsets(8)):
        j, i = divmod(p, 8)
        tau, lam = aux[3, j, i], aux[2, j, i]
        if not (abs(ap) < HALF and abs(bp) < HALF):
            assert np.all(avg[:, j, i] == 0.0)
            continue
        _, ni = oracle.camera_ray(cam, st, i, j)
        lp = tau / aI / L * ni   # affine length inside the plasma
        for k in range(7):
            assert avg[7 + k, j, i] == pytest.approx(q[k], rel=1e-12), ("Ij", k)
            assert avg[14 + k, j, i] == pytest.approx(q[k] * -math.expm1(-tau), rel=1e-11), ("tau", k)
            assert avg[k, j, i] * lam == pytest.approx(q[k] * lp, rel=1e-11), ("lambda", k)


def test_averages_do_not_change_the_image(oracle):
    cam, st, integ, grid, pl = _setup(1)
    i0, a0 = oracle.render(cam, st, integ, grid, pl)
    i1, a1, _ = oracle.render(cam, st, integ, grid, pl, averages=True)
    assert np.array_equal(i0, i1) and np.array_equal(a0, a1)
