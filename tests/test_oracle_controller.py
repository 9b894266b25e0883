"""Pins of the oracle's step-size control (paper section 2.2, Geodesics: the
embedded RK5(4) error estimate accepts or rejects each trial step; the
controller follows Numerical Recipes, whose constants the paper does not
print).  The readings under test: accept iff eps <= 1; after an accepted
trial the step is multiplied by min(10, max(0.2, 0.9 eps^-1/5)) (10 when eps
is exactly 0), after a rejected one by max(0.2, 0.9 eps^-1/5), an accepted
trial right after a rejection may not grow the step, every factor is rounded
to a multiple of 1/4096, and the first trial is h0 = -0.1 rint(1024 r_pix) /
1024.

The error norm of every logged trial is recomputed here from the paper's
definition -- the fifth- and fourth-order solutions formed separately from
the tableau as printed (golden file) and differenced -- rather than from the
weighted difference of the stages that the oracle sums, so a wrong weight, a
dropped stage or a wrong scale in the oracle fails the comparison."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "dp_tableau.txt")


def _tableau():
    rows, w = [], {}
    for line in open(GOLDEN):
        line = line.split("#")[0].strip()
        if not line:
            continue
        tag, rest = line.split(None, 1)
        if tag == "c":
            parts = rest.split("|")
            rows.append([float(Fraction(x)) for x in parts[1].split()] if len(parts) > 1 else [])
        else:
            w[tag] = np.array([float(Fraction(x)) for x in rest.split()])
    A = np.zeros((7, 7))
    for i, r in enumerate(rows):
        A[i, :len(r)] = r
    return A, w["b5"], w["b4"]


def _ks_r(a, x, y, z):
    R2 = x * x + y * y + z * z
    return math.sqrt(0.5 * (R2 - a * a + math.sqrt((R2 - a * a) ** 2 + 4 * a * a * z * z)))


def _eps_by_definition(oracle, a, flat, y, h, f_abs, f_rel):
    """eps of one trial: y5 and y4 each formed from the stages, then
    differenced (paper: eps = max_m |y5 - y4| / (f_abs + f_rel max(|y|, |y5|)))."""
    A, b5, b4 = _tableau()
    k = np.zeros((7, 8))
    k[0] = oracle.geodesic_rhs(a, y, flat=flat)
    for i in range(1, 7):
        k[i] = oracle.geodesic_rhs(a, y + h * (A[i, :i] @ k[:i]), flat=flat)
    y5 = y + h * (b5 @ k)
    y4 = y + h * (b4 @ k)
    sc = f_abs + f_rel * np.maximum(np.abs(y), np.abs(y5))
    return float(np.max(np.abs(y5 - y4) / sc)), y5


def _law(eps, accepted, after_reject):
    if accepted:
        f = 10.0 if eps == 0.0 else min(10.0, max(0.2, 0.9 * eps ** -0.2))
    else:
        f = max(0.2, 0.9 * eps ** -0.2)
    f = round(f * 4096.0) / 4096.0
    if accepted and after_reject:
        f = min(f, 1.0)
    return f


INTEG = dict(f_abs=1e-8, f_rel=1e-8, ds_max=0.5, h0_frac=0.1, max_steps=100000)


def test_flat_space_steps_grow_tenfold(oracle):
    """Minkowski metric: every stage of a trial is the same constant vector, so
    the two solutions coincide, eps is (up to the rounding of the weight sums)
    zero, every trial is accepted and each step is exactly ten times the last,
    starting from h0 = -0.1 rint(1024 r_pix) / 1024."""
    cam = dict(r=100.0, theta=math.radians(30), width=30.0, n=5)
    st = dict(a=0.0, r_in=0.0, flat=1)
    for i, j in [(0, 0), (2, 2), (4, 1)]:
        t = oracle.trace_trials(cam, st, INTEG, i, j)
        tr = t["trials"]
        assert t["n_rej"] == 0 and t["status"] == oracle.ESCAPED and len(tr) >= 3
        y0 = tr[0, :8]
        r_pix = math.sqrt(y0[1] ** 2 + y0[2] ** 2 + y0[3] ** 2)
        assert tr[0, 8] == -0.1 * (round(1024.0 * r_pix) / 1024.0)
        assert np.all(tr[:, 9] < 1e-6) and np.all(tr[:, 10] == 1.0)
        for q in range(1, len(tr)):
            assert tr[q, 8] == 10.0 * tr[q - 1, 8]


@pytest.mark.parametrize("a,theta_deg,pixels", [
    (0.9, 17.0, [(8, 8), (3, 12), (0, 0), (15, 7)]),
    (0.98, 80.0, [(6, 8), (9, 8), (8, 2)]),
])
def test_controller_law_in_kerr(oracle, a, theta_deg, pixels):
    cam = dict(r=100.0, theta=math.radians(theta_deg), width=30.0, n=16)
    st = dict(a=a, r_in=1.01 * (1.0 + math.sqrt(1.0 - a * a)))
    n_rej = n_mid = 0
    for i, j in pixels:
        t = oracle.trace_trials(cam, st, INTEG, i, j)
        tr = t["trials"]
        assert len(tr) == t["n_acc"] + t["n_rej"] > 10
        y0 = tr[0, :8]
        assert tr[0, 8] == -0.1 * (round(1024.0 * _ks_r(a, *y0[1:4])) / 1024.0)
        for q in range(len(tr)):
            y, h, eps, acc = tr[q, :8], tr[q, 8], tr[q, 9], tr[q, 10]
            eps_def, y5 = _eps_by_definition(oracle, a, 0, y, h, INTEG["f_abs"], INTEG["f_rel"])
            assert abs(eps_def - eps) <= 1e-6 * max(1.0, eps), (i, j, q, eps, eps_def)
            assert acc == (1.0 if eps <= 1.0 else 0.0)
            if q + 1 == len(tr):
                break
            after_reject = q > 0 and tr[q - 1, 10] == 0.0
            fac = tr[q + 1, 8] / h
            # every factor is a multiple of 1/4096 within [0.2, 10] (the ratio
            # of the stored steps carries the rounding of h * factor)
            assert abs(fac * 4096.0 - round(fac * 4096.0)) <= 1e-9 and 0.2 - 1e-12 <= fac <= 10.0 + 1e-12
            assert tr[q + 1, 8] == h * _law(eps, acc == 1.0, after_reject), (i, j, q, eps, fac)
            if acc == 1.0:
                # the next trial starts from this trial's fifth-order solution
                assert np.abs(tr[q + 1, :8] - y5).max() <= 1e-12 * (1.0 + np.abs(y5).max())
                if after_reject:
                    assert fac <= 1.0
                if 0.2 < fac < 10.0 and not after_reject:
                    n_mid += 1
            else:
                n_rej += 1
                assert np.array_equal(tr[q + 1, :8], y)   # a rejected trial leaves the state
                assert fac < 1.0
    # the sample exercises rejections and factors strictly inside the clamps
    assert n_rej >= 3 and n_mid >= 50
