"""Plain CPU oracle of the octree initialisation of the primitives and of the
SSIM term of the photometric loss (test infrastructure only; shares no code
with the library).

Octree (the appendix's initialisation algorithm): starting from the root cube,
every node holding more than m points is split into its 8 equal sub-cubes
(recursively); D_max is the deepest leaf's depth and d_stop = floor((D_max +
1) / 2); then for d = 0 .. d_stop - 1 every leaf at depth d is split into its
non-empty sub-cubes.  Each final leaf gives one primitive: centre the
centroid of its points, radius half the cube's diagonal (sqrt(3)/2 times its
side).

Readings where the algorithm leaves a choice open:
  * the root is the axis-aligned cube centred on the points' bounding box,
    with side the box's largest extent;
  * a point belongs to the lower half of an axis when its coordinate is below
    the cube's midpoint, else to the upper half;
  * empty sub-cubes are dropped (they hold no points to take a centroid of);
  * a leaf whose points all coincide is not split further (its cubes would
    shrink without separating them).

SSIM (Sec. 3.5's photometric objective, as 3D Gaussian splatting computes it):
per channel, local means, variances and covariance under an 11 x 11 Gaussian
window of standard deviation 1.5 (weights normalised to sum 1), the image
padded with zeros, then SSIM = mean over pixels and channels of
(2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(s_x^2 + s_y^2 + C2)),
C1 = 0.01^2, C2 = 0.03^2.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["octree_leaves", "octree_primitives", "ssim"]


def _split(pts, lo, side):
    """The non-empty sub-cubes of the cube [lo, lo + side)^3 with their points."""
    mid = lo + side / 2.0
    out = []
    for ix in (0, 1):
        for iy in (0, 1):
            for iz in (0, 1):
                sel = np.ones(len(pts), bool)
                for a, ia in enumerate((ix, iy, iz)):
                    below = pts[:, a] < mid[a]
                    sel &= below if ia == 0 else ~below
                if sel.any():
                    clo = lo + np.array([ix, iy, iz], np.float64) * side / 2.0
                    out.append((pts[sel], clo, side / 2.0))
    return out


def octree_leaves(points, m: int):
    """Leaves (points, cube corner, side, depth) of the initialisation octree."""
    pts = np.asarray(points, np.float64)
    bmin, bmax = pts.min(0), pts.max(0)
    side = float((bmax - bmin).max())
    side = side if side > 0 else 1.0
    lo = (bmin + bmax) / 2.0 - side / 2.0
    leaves = []

    def build(p, clo, s, depth):
        if len(p) > m and not np.all(p == p[0]):
            for cp, cl, cs in _split(p, clo, s):
                build(cp, cl, cs, depth + 1)
        else:
            leaves.append((p, clo, s, depth))

    build(pts, lo, side, 0)
    d_max = max(d for _, _, _, d in leaves)
    d_stop = (d_max + 1) // 2
    for d in range(d_stop):
        nxt = []
        for p, clo, s, depth in leaves:
            if depth == d and not np.all(p == p[0]):
                nxt.extend((cp, cl, cs, depth + 1) for cp, cl, cs in _split(p, clo, s))
            else:
                nxt.append((p, clo, s, depth))
        leaves = nxt
    return leaves


def octree_primitives(points, m: int):
    """(centres [N,3], radii [N]) of the final leaves, sorted by centre
    (x, then y, then z) so that two implementations can be compared."""
    leaves = octree_leaves(points, m)
    c = np.array([p.mean(0) for p, _, _, _ in leaves])
    r = np.array([math.sqrt(3.0) / 2.0 * s for _, _, s, _ in leaves])
    order = np.lexsort((c[:, 2], c[:, 1], c[:, 0]))
    return c[order], r[order]


def _gauss_window(size=11, sigma=1.5):
    x = np.arange(size) - size // 2
    g = np.exp(-(x * x) / (2.0 * sigma * sigma))
    g /= g.sum()
    return np.outer(g, g)


def ssim(x, y, size=11, sigma=1.5):
    """Mean SSIM of two images [H, W, C] (float64, pixel loops over the
    window: slow, for small images)."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    h, w, nc = x.shape
    win = _gauss_window(size, sigma)
    r = size // 2
    c1, c2 = 0.01 ** 2, 0.03 ** 2
    total = 0.0
    for ch in range(nc):
        for i in range(h):
            for j in range(w):
                mx = my = sxx = syy = sxy = 0.0
                for a in range(size):
                    for b in range(size):
                        ii, jj = i + a - r, j + b - r
                        if 0 <= ii < h and 0 <= jj < w:
                            wt = win[a, b]
                            xv, yv = x[ii, jj, ch], y[ii, jj, ch]
                            mx += wt * xv
                            my += wt * yv
                            sxx += wt * xv * xv
                            syy += wt * yv * yv
                            sxy += wt * xv * yv
                vx, vy, cxy = sxx - mx * mx, syy - my * my, sxy - mx * my
                total += ((2 * mx * my + c1) * (2 * cxy + c2)) / ((mx * mx + my * my + c1) * (vx + vy + c2))
    return total / (h * w * nc)
