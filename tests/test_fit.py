"""The fitting module's host-side pieces: the octree initialisation and the
SSIM term, the oracle's versions pinned by hand-computed cases and
invariants, and the library's (vectorised, torch) versions against them."""
import math

import numpy as np
import pytest
import torch

import oracle


def test_octree_root_leaf_when_few_points():
    pts = np.array([[0.0, 0.0, 0.0], [1.0, 0.5, 0.25], [0.5, 1.0, 0.0]])
    c, r = oracle.octree_primitives(pts, 3)
    # one leaf: the root cube, side = largest extent 1
    np.testing.assert_allclose(c, [pts.mean(0)])
    np.testing.assert_allclose(r, [math.sqrt(3) / 2])


def test_octree_two_clusters_by_hand():
    """Six points, three near each of two opposite corners of the unit cube:
    with m = 3 the root (6 points) splits once; the clusters fall in octants
    (0,0,0) and (1,1,1), depth 1 = D_max, d_stop = 1, and no leaf lies at
    depth 0, so the refinement changes nothing."""
    a = np.array([[0.0, 0.0, 0.0], [0.1, 0.0, 0.0], [0.0, 0.1, 0.0]])
    b = np.array([[1.0, 1.0, 1.0], [0.9, 1.0, 1.0], [1.0, 1.0, 0.9]])
    c, r = oracle.octree_primitives(np.concatenate([a, b]), 3)
    np.testing.assert_allclose(c, [a.mean(0), b.mean(0)])
    np.testing.assert_allclose(r, [math.sqrt(3) / 4] * 2)


def test_octree_refines_shallow_leaves():
    """A dense cluster near one corner forces deep leaves (D_max = 8, so
    d_stop = 4).  The far pair (0.9, 0.9, 0.9), (1, 1, 1) is a depth-1 leaf
    of the first pass (2 <= m points); the refinement splits it at depths
    1, 2 and 3: both stay in the upper child ([0.5,1), [0.75,1), [0.875,1))
    until the midpoint 0.9375 separates them, leaving each alone in a
    depth-4 cube of side 1/16."""
    rng = np.random.default_rng(3)
    dense = 0.05 + 0.01 * rng.random((40, 3))
    lone = np.array([[0.9, 0.9, 0.9]])
    corner = np.array([[0.0, 0.0, 0.0], [1.0, 1.0, 1.0]])
    pts = np.concatenate([dense, lone, corner])
    leaves = oracle.octree_leaves(pts, 10)
    dmax_first = max(d for _, _, _, d in leaves)
    for p, lo, s, d in leaves:
        assert np.all(p >= lo - 1e-12) and np.all(p < lo + s + 1e-12)   # the cube holds its points
        assert len(p) <= 10
    sizes = sorted(len(p) for p, _, _, _ in leaves)
    assert sum(sizes) == len(pts)                                          # a partition
    assert dmax_first == 8
    for q in (lone[0], corner[1]):
        leaf = [x for x in leaves if len(x[0]) == 1 and np.allclose(x[0][0], q)][0]
        assert leaf[3] == 4 and math.isclose(leaf[2], 1 / 16)


def test_octree_invariants_and_library_agrees():
    from paper_2606_03877_amd.fit import octree_init
    for seed, n, m in [(0, 400, 10), (1, 1500, 5), (2, 200, 20), (5, 60, 1)]:
        rng = np.random.default_rng(seed)
        pts = np.concatenate([rng.random((n, 3)), 0.02 * rng.standard_normal((n // 2, 3)) + 0.3])
        leaves = oracle.octree_leaves(pts, m)
        assert sum(len(p) for p, _, _, _ in leaves) == len(pts)
        dmax = max(d for _, _, _, d in leaves)
        for p, lo, s, d in leaves:
            assert len(p) <= m or np.all(p == p[0]) or d > 0
            assert np.all(p >= lo - 1e-12) and np.all(p < lo + s + 1e-12)
        c1, r1 = oracle.octree_primitives(pts, m)
        c2, r2 = octree_init(pts, m)
        np.testing.assert_allclose(c2, c1, rtol=0, atol=1e-12)
        np.testing.assert_array_equal(r2, r1)


def test_ssim_pins():
    rng = np.random.default_rng(0)
    x = rng.random((6, 6, 3))
    assert oracle.ssim(x, x) == pytest.approx(1.0, abs=1e-12)
    y = np.clip(x + 0.1 * rng.standard_normal(x.shape), 0, 1)
    assert oracle.ssim(x, y) == pytest.approx(oracle.ssim(y, x), abs=1e-12)
    z = np.clip(x + 0.3 * rng.standard_normal(x.shape), 0, 1)
    assert oracle.ssim(x, z) < oracle.ssim(x, y) < 1.0
    # a single pixel: only the window's centre weight w0 = g0^2 sees the image
    # (zero padding), g0 = 1 / sum_k exp(-k^2 / 4.5) over k = -5..5
    g0 = 1.0 / sum(math.exp(-k * k / 4.5) for k in range(-5, 6))
    w0 = g0 * g0
    a, b = 0.7, 0.4
    mx, my = w0 * a, w0 * b
    vx, vy, cxy = w0 * a * a - mx * mx, w0 * b * b - my * my, w0 * a * b - mx * my
    c1, c2 = 1e-4, 9e-4
    want = ((2 * mx * my + c1) * (2 * cxy + c2)) / ((mx * mx + my * my + c1) * (vx + vy + c2))
    assert oracle.ssim(np.full((1, 1, 1), a), np.full((1, 1, 1), b)) == pytest.approx(want, rel=1e-12)


def test_library_ssim_matches_oracle():
    from paper_2606_03877_amd.fit import ssim_tiles
    rng = np.random.default_rng(1)
    x = rng.random((3, 8, 8, 3))
    y = np.clip(x + 0.2 * rng.standard_normal(x.shape), 0, 1)
    want = np.mean([oracle.ssim(x[i], y[i]) for i in range(3)])
    t = lambda a: torch.from_numpy(a).permute(0, 3, 1, 2).float()
    got = float(ssim_tiles(t(x), t(y)))
    assert got == pytest.approx(want, abs=2e-6)
