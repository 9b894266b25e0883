"""Pins of the oracle's adaptive ray tracing (paper section 4.4, Adaptive Ray
Tracing): the five refinement criteria against closed forms of smooth
intensity fields (linear, quadratic, exponential), the edge rules, the
critical-fraction and region rules at their boundaries, the level geometry
against the oracle camera (a pixel's four children are centred on it), and a
whole adaptive render of a uniform cube in flat spacetime, whose refined
blocks follow from where the cube's face projects on the image plane."""
import math

import numpy as np
import pytest

from oracle import adaptive as A
from test_oracle_pipeline import HALF, _setup

B = 6
II, JJ = np.meshgrid(np.arange(B, dtype=float), np.arange(B, dtype=float))   # II[j][i] = i


def test_linear_field_gradient_is_exact_everywhere():
    I = 3.0 + 0.25 * II - 0.5 * JJ
    g = A.criterion_map(I, A.GRAD_ABS)
    assert np.allclose(g, math.hypot(0.25, 0.5), rtol=1e-14, atol=0)   # edges too: one-sided is exact
    assert np.allclose(A.criterion_map(I, A.LAP_ABS), 0.0, atol=1e-13)
    assert np.array_equal(A.criterion_map(I, A.VALUE), I)


def test_quadratic_field_laplacian_and_central_gradient():
    I = II ** 2 + 2.0 * JJ ** 2
    # every three-point second difference of a quadratic is exact: 2 + 4
    assert np.allclose(A.criterion_map(I, A.LAP_ABS), 6.0, rtol=1e-14)
    g = A.criterion_map(I, A.GRAD_ABS)
    # interior: central differences of a quadratic are exact derivatives
    for j in range(1, B - 1):
        for i in range(1, B - 1):
            assert g[j, i] == pytest.approx(math.hypot(2 * i, 4 * j), rel=1e-14)
    # corner (0, 0): one-sided differences I[1] - I[0] = 1 and 2
    assert g[0, 0] == pytest.approx(math.hypot(1.0, 2.0), rel=1e-14)
    # corner (B-1, B-1): I[B-1] - I[B-2] = 2B - 3 and 2 (2B - 3)
    assert g[B - 1, B - 1] == pytest.approx(math.hypot(2 * B - 3, 2 * (2 * B - 3)), rel=1e-14)


@pytest.mark.parametrize("al", [0.3, -1.1])
def test_exponential_field_relative_criteria(al):
    # I = e^(al i): the 1-2-1 normalised differences are 2 tanh(al/2) and
    # 4 tanh^2(al/2), independent of i (along j the field is constant)
    I = np.exp(al * II)
    g = A.criterion_map(I, A.GRAD_REL)
    lap = A.criterion_map(I, A.LAP_REL)
    t = math.tanh(al / 2)
    assert np.allclose(g[:, 1:B - 1], 2 * abs(t), rtol=1e-13)
    assert np.allclose(lap, 4 * t * t, rtol=1e-12)
    # one-sided at the edges: 2 (e^al - 1) / (1 + e^al) = 2 tanh(al/2) as well
    assert np.allclose(g[:, 0], 2 * abs(t), rtol=1e-13)
    assert np.allclose(g[:, B - 1], 2 * abs(t), rtol=1e-13)
    # scale invariance of the relative criteria
    assert np.allclose(A.criterion_map(7.5 * I, A.GRAD_REL), g, rtol=1e-14)


def test_degenerate_blocks():
    z = np.zeros((4, 4))
    for k in range(A.N_CRIT):
        assert np.array_equal(A.criterion_map(z, k), z)   # relative forms of I = 0 are 0, not NaN
    one = np.array([[5.0]])
    assert A.criterion_map(one, A.GRAD_ABS)[0, 0] == 0.0
    assert A.criterion_map(one, A.LAP_ABS)[0, 0] == 0.0
    two = np.array([[1.0, 4.0], [2.0, 8.0]])
    assert np.array_equal(A.criterion_map(two, A.LAP_ABS), np.zeros((2, 2)))
    g = A.criterion_map(two, A.GRAD_ABS)
    assert g[0, 0] == pytest.approx(math.hypot(3.0, 1.0)) and g[1, 1] == pytest.approx(math.hypot(6.0, 4.0))


def test_critical_fraction_boundary():
    I = np.zeros((4, 4))
    I[0, :3] = 1.0                      # three pixels above 0.5
    ad = dict(thr=[0.5, None, None, None, None], frac=3 / 16)
    assert A.refines(I, 0, (0.0, 0.0), ad)
    assert not A.refines(I, 0, (0.0, 0.0), dict(ad, frac=3.0001 / 16))
    assert not A.refines(I, 0, (0.0, 0.0), dict(ad, thr=[1.0, None, None, None, None]))   # strict
    assert not A.refines(I, 0, (0.0, 0.0), dict(ad, thr=[None] * 5))


def test_region_rule():
    I = np.zeros((2, 2))
    ad = dict(thr=[None] * 5, frac=1.0, regions=[(-1.0, 1.0, 0.0, 2.0, 2)])
    assert A.refines(I, 0, (1.0, 0.0), ad)          # closed rectangle
    assert A.refines(I, 1, (0.0, 2.0), ad)
    assert not A.refines(I, 2, (0.0, 1.0), ad)      # at its minimum level
    assert not A.refines(I, 0, (1.0 + 1e-12, 1.0), ad)
    # centres: a 2 x 2 block grid of a 4-pixel root with width 8 has centres at +-2
    assert A.block_center(4, 2, 8.0, 0, 0, 0) == (-2.0, -2.0)
    assert A.block_center(4, 2, 8.0, 1, 3, 0) == (3.0, -3.0)


def test_children_order():
    out = A.children([(1, 0, 0), (1, 3, 2), (1, 1, 1)], [True, False, True])
    assert out == [(2, 0, 0), (2, 1, 0), (2, 0, 1), (2, 1, 1), (2, 2, 2), (2, 3, 2), (2, 2, 3), (2, 3, 3)]


def test_children_pixels_are_centred_on_their_parent(oracle):
    cam, st, _, _, _ = _setup(0, n=6)
    cam = dict(cam, theta=1.1, phi=0.4, r=50.0)
    for stx in (dict(st, a=0.9, flat=0), st):
        for (i, j) in [(0, 0), (5, 2), (3, 4)]:
            y0, _ = oracle.camera_ray(cam, stx, i, j)
            kids = [oracle.camera_ray(dict(cam, n=12), stx, 2 * i + di, 2 * j + dj)[0]
                    for dj in (0, 1) for di in (0, 1)]
            mean = np.mean([k[:4] for k in kids], axis=0)
            assert np.allclose(mean, y0[:4], rtol=0, atol=1e-12)
            if stx["flat"]:
                # flat space: the children sit half a child pixel off the
                # parent centre along each image axis
                d = kids[3][1:4] - kids[0][1:4]
                assert np.linalg.norm(d) == pytest.approx(math.sqrt(2) * cam["width"] / 12, rel=1e-12)


def _expected_cube_blocks(n_root, b, width, max_level):
    """Blocks refined by the value criterion (I > 0 in one pixel) on the face-on
    cube: a pixel is lit iff its centre projects inside the cube's face."""
    inside = lambda c: abs(c) < HALF
    blocks = [(0, bx, by) for by in range(n_root // b) for bx in range(n_root // b)]
    levels = [blocks]
    for level in range(max_level):
        nl = n_root * 2 ** level
        ctr = lambda p: (p - nl / 2 + 0.5) * width / nl
        flags = [any(inside(ctr(bx * b + i)) and inside(ctr(by * b + j)) for j in range(b) for i in range(b))
                 for (_, bx, by) in blocks]
        blocks = A.children(blocks, flags)
        levels.append(blocks)
    return levels


def test_cube_render_refines_where_the_cube_is(oracle):
    cam, st, integ, grid, pl = _setup(0, n=4)
    cam = dict(cam, width=60.0)
    ad = dict(block=2, max_level=2, thr=[0.0, None, None, None, None], frac=1 / 4)
    levels = A.render_adaptive(cam, st, integ, grid, pl, ad)
    want = _expected_cube_blocks(4, 2, cam["width"], 2)
    assert [len(l[0]) for l in levels] == [len(w) for w in want] == [4, 16, 16]
    for (blk, img, aux), w in zip(levels, want):
        assert [tuple(r) for r in blk] == w
        assert img.shape == (len(w), 4, 2, 2)
    # the level-2 pixels are those of a uniform 16 x 16 render
    blk, img, _ = levels[2]
    full, _ = oracle.render(dict(cam, n=16), st, integ, grid, pl)
    for k, (_, bx, by) in enumerate(blk):
        assert np.array_equal(img[k], full[:, 2 * by:2 * by + 2, 2 * bx:2 * bx + 2])
