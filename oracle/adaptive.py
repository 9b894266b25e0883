"""Adaptive ray tracing (paper section 4.4, Adaptive Ray Tracing): plain
reference of the refinement criteria and of the level-by-level render.

TEST INFRASTRUCTURE ONLY: imported by the test suite, never by the product
library.  Written from the definitions in plain Python loops; the pixels
themselves come from the oracle's own render (oracle.render_pixels).

Geometry.  A pixel is a square of the image plane sampled by a ray through
its centre.  Level 0 is the root image of N x N pixels, cut into blocks of
B x B pixels (B divides N).  Refining a block of level l splits each of its
pixels into four, giving four blocks of level l + 1 with B x B pixels each.
A level-l pixel is therefore pixel (i, j) of a uniform image of N 2^l pixels
per side with the same camera width, and block (bx, by) of level l holds its
pixels i = bx B .. bx B + B - 1, j = by B .. by B + B - 1.  The children of
block (bx, by) are (2bx, 2by), (2bx+1, 2by), (2bx, 2by+1), (2bx+1, 2by+1), in
that order; the blocks of a level are listed in the order of their parents
(level 0 row by row).

Criteria, on the intensity I (Stokes I at the rendered frequency) of the
pixels of one block, with no information from other blocks:
  VALUE     I itself
  GRAD_ABS  (Di^2 + Dj^2)^(1/2), Di = (I[i+1] - I[i-1]) / 2
  GRAD_REL  (Di^2 + Dj^2)^(1/2), Di = 2 (I[i+1] - I[i-1]) / (I[i-1] + 2 I[i] + I[i+1])
  LAP_ABS   |Di + Dj|, Di = I[i-1] - 2 I[i] + I[i+1]
  LAP_REL   |Di + Dj|, Di = 4 (I[i-1] - 2 I[i] + I[i+1]) / (I[i-1] + 2 I[i] + I[i+1])
(Dj alike along the column).  Readings where the paper is silent or garbled:
  - the relative Laplacian divides the second difference by the same
    1-2-1 weighted sum as the relative gradient (the printed quotient has the
    numerator's expression in its denominator as well);
  - one-sided differences at block edges: the gradient uses the two-point
    difference I[1] - I[0] (relative: divided by (I[0] + I[1]) / 2), the
    Laplacian the three-point second difference of the nearest interior
    pixel; along a direction with one pixel (two for the Laplacian) the
    difference is 0;
  - a relative difference whose weighted sum is 0 (I = 0 on all its points,
    as intensities are non-negative) is 0;
  - a block is refined if, for any enabled criterion, the number of its
    pixels whose value exceeds the threshold (strictly) is at least
    frac B^2, or if its centre lies in an image-plane region (closed
    rectangle) whose minimum level exceeds the block's level.
"""
import math

import numpy as np

from . import oracle as _o

VALUE, GRAD_ABS, GRAD_REL, LAP_ABS, LAP_REL = range(5)
N_CRIT = 5


def _grad_1d(v, k, rel):
    n = len(v)
    if n < 2:
        return 0.0
    if 0 < k < n - 1:
        a, b, c = v[k - 1], v[k], v[k + 1]
        if rel:
            s = a + 2.0 * b + c
            return 0.0 if s == 0.0 else 2.0 * (c - a) / s
        return 0.5 * (c - a)
    lo, hi = (v[0], v[1]) if k == 0 else (v[n - 2], v[n - 1])
    if rel:
        s = lo + hi
        return 0.0 if s == 0.0 else 2.0 * (hi - lo) / s
    return hi - lo


def _lap_1d(v, k, rel):
    n = len(v)
    if n < 3:
        return 0.0
    m = min(max(k, 1), n - 2)
    a, b, c = v[m - 1], v[m], v[m + 1]
    d2 = a - 2.0 * b + c
    if rel:
        s = a + 2.0 * b + c
        return 0.0 if s == 0.0 else 4.0 * d2 / s
    return d2


def criterion_map(I, kind):
    """Per-pixel value of one criterion over a block I[j][i] (row j along
    the image plane's vertical axis, column i along its horizontal one)."""
    I = np.asarray(I, dtype=np.float64)
    nj, ni = I.shape
    out = np.zeros((nj, ni))
    for j in range(nj):
        for i in range(ni):
            row, col = list(I[j, :]), list(I[:, i])
            if kind == VALUE:
                out[j, i] = I[j, i]
            elif kind in (GRAD_ABS, GRAD_REL):
                rel = kind == GRAD_REL
                di, dj = _grad_1d(row, i, rel), _grad_1d(col, j, rel)
                out[j, i] = math.sqrt(di * di + dj * dj)
            else:
                rel = kind == LAP_REL
                out[j, i] = abs(_lap_1d(row, i, rel) + _lap_1d(col, j, rel))
    return out


def block_center(n_root, b, width, level, bx, by):
    """Image-plane coordinates (along the horizontal and vertical axes, in
    units of the camera width) of the centre of block (bx, by) of a level."""
    nl = n_root * 2 ** level
    return ((bx * b + 0.5 * b - 0.5 * nl) * width / nl, (by * b + 0.5 * b - 0.5 * nl) * width / nl)


def refines(I_block, level, center, ad):
    """Refinement decision for one block.  ad: dict with 'thr' (5 thresholds,
    None = criterion off), 'frac' and 'regions' (list of (x0, x1, y0, y1,
    min_level))."""
    cx, cy = center
    for (x0, x1, y0, y1, lmin) in ad.get("regions", []):
        if x0 <= cx <= x1 and y0 <= cy <= y1 and level < lmin:
            return True
    nb = np.asarray(I_block).size
    for kind, thr in enumerate(ad.get("thr", [None] * N_CRIT)):
        if thr is None:
            continue
        count = int(np.sum(criterion_map(I_block, kind) > thr))
        if count >= ad["frac"] * nb:
            return True
    return False


def children(blocks, flags):
    """Blocks of the next level from the blocks of a level and their flags."""
    out = []
    for (lev, bx, by), f in zip(blocks, flags):
        if f:
            for dy in (0, 1):
                for dx in (0, 1):
                    out.append((lev + 1, 2 * bx + dx, 2 * by + dy))
    return out


def block_pixels(n_root, b, level, bx, by):
    """Pixel indices i + N_l j (N_l = N 2^level) of a block, row by row."""
    nl = n_root * 2 ** level
    return [(bx * b + i) + nl * (by * b + j) for j in range(b) for i in range(b)]


def render_adaptive(cam, st, integ, gr, pl, ad, n_threads=None):
    """Level-by-level render.  ad: 'block' (B), 'max_level', and the criteria
    of `refines`.  Returns a list over levels of (blocks [n][3] = (level, bx,
    by), image [n][4][B][B], aux [n][NAUX][B][B])."""
    n_root, b = int(cam["n"]), int(ad["block"])
    nbk = n_root // b
    blocks = [(0, bx, by) for by in range(nbk) for bx in range(nbk)]
    levels = []
    for level in range(int(ad["max_level"]) + 1):
        if not blocks:
            break
        cl = dict(cam, n=n_root * 2 ** level)
        pix = [p for (_, bx, by) in blocks for p in block_pixels(n_root, b, level, bx, by)]
        img, aux = _o.render_pixels(cl, st, integ, gr, pl, pix, n_threads)
        nblk = len(blocks)
        img = img.reshape(nblk, b, b, 4).transpose(0, 3, 1, 2)
        aux = aux.reshape(nblk, b, b, -1).transpose(0, 3, 1, 2)
        levels.append((np.array(blocks, dtype=np.int32).reshape(-1, 3), img, aux))
        if level == int(ad["max_level"]):
            break
        flags = [refines(img[k, 0], level, block_center(n_root, b, cam["width"], level, bx, by), ad)
                 for k, (_, bx, by) in enumerate(blocks)]
        blocks = children(blocks, flags)
    return levels
