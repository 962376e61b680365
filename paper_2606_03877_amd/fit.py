"""End-to-end fitting of a primitive set to images with the render path.

* ``octree_init``: the initialisation algorithm of the paper's appendix
  (an adaptive octree over a point cloud: nodes holding more than m points
  split into their 8 sub-cubes; then, up to half the deepest leaf depth,
  every shallow leaf split into its non-empty sub-cubes; each final leaf
  one primitive, centred on its points' centroid, radius half the cube's
  diagonal), vectorised over the points level by level.
* ``photometric_loss``: Sec. 3.5's (1 - lambda) L1 + lambda (1 - SSIM),
  SSIM with the 11 x 11 Gaussian window (standard deviation 1.5) of 3D
  Gaussian splatting, evaluated per 8 x 8 tile (zero padding).
* ``fit``: Adam with the learning rates of Sec. 4.1 (1e-2 for log-scales,
  1e-4 for positions, 1e-3 for everything else) over mini-batches of the
  appendix's tile-based training: each iteration takes 4 images and a
  quarter of each image's 8 x 8 tiles.

Rendering and its gradients run in the HIP library; this module holds the
training loop around it (torch for the loss and the optimiser).
"""
from __future__ import annotations

import math
from typing import List, Optional, Sequence

import numpy as np
import torch

from .render import NetSpec, RenderOpts, Renderer, render

__all__ = ["octree_init", "init_primitives", "ssim_tiles", "photometric_loss", "TileBatches", "fit"]

TILE = 8


def octree_init(points, m: int = 10):
    """(centres [N,3], radii [N]) of the initialisation octree's final leaves,
    sorted by centre (x, then y, then z).  The root is the cube centred on the
    points' bounding box with its largest extent as side; a point takes the
    upper half of an axis from the cube's midpoint on; empty cubes are
    dropped and a node whose points all coincide is not split."""
    pts = np.asarray(points, np.float64)
    n = len(pts)
    bmin, bmax = pts.min(0), pts.max(0)
    side0 = float((bmax - bmin).max())
    side0 = side0 if side0 > 0 else 1.0
    lo0 = (bmin + bmax) / 2.0 - side0 / 2.0

    def split(cell, lo, side, depth, idx):
        """Child cells of the points idx of the given cells (per point)."""
        mid = lo[idx] + (side[idx] / 2.0)[:, None]
        bits = (pts[idx] >= mid).astype(np.int64)
        child = bits[:, 0] * 4 + bits[:, 1] * 2 + bits[:, 2]
        key = cell[idx] * 8 + child
        uniq, inv = np.unique(key, return_inverse=True)
        new_lo = lo[idx] + bits * (side[idx] / 2.0)[:, None]
        return uniq, inv, new_lo, side[idx] / 2.0, depth[idx] + 1

    # per point: its current leaf (a unique id per cell), cube corner, side, depth
    cell = np.zeros(n, np.int64)
    lo = np.tile(lo0, (n, 1))
    side = np.full(n, side0)
    depth = np.zeros(n, np.int64)
    ids = np.zeros(n, np.int64)          # dense leaf id per point

    def regroup():
        _, d = np.unique(cell, return_inverse=True)
        return d

    def spread(ids):
        """Per leaf: points, and whether they are not all the same point."""
        cnt = np.bincount(ids)
        mn = np.full((len(cnt), 3), np.inf)
        mx = np.full((len(cnt), 3), -np.inf)
        np.minimum.at(mn, ids, pts)
        np.maximum.at(mx, ids, pts)
        return cnt, (mx > mn).any(1)

    while True:
        ids = regroup()
        cnt, distinct = spread(ids)
        want = (cnt > m) & distinct
        sel = want[ids]
        if not sel.any():
            break
        idx = np.nonzero(sel)[0]
        uniq, inv, nlo, nside, ndep = split(cell, lo, side, depth, idx)
        cell[idx] = (cell.max() + 1) + inv          # fresh ids for the children
        lo[idx], side[idx], depth[idx] = nlo, nside, ndep
    d_stop = (int(depth.max()) + 1) // 2
    for d in range(d_stop):
        ids = regroup()
        _, distinct = spread(ids)
        sel = (depth == d) & distinct[ids]
        if not sel.any():
            continue
        idx = np.nonzero(sel)[0]
        uniq, inv, nlo, nside, ndep = split(cell, lo, side, depth, idx)
        cell[idx] = (cell.max() + 1) + inv
        lo[idx], side[idx], depth[idx] = nlo, nside, ndep
    ids = regroup()
    cnt = np.bincount(ids)
    cen = np.zeros((len(cnt), 3))
    np.add.at(cen, ids, pts)
    cen /= cnt[:, None]
    rad = np.zeros(len(cnt))
    rad[ids] = math.sqrt(3.0) / 2.0 * side
    order = np.lexsort((cen[:, 2], cen[:, 1], cen[:, 0]))
    return cen[order], rad[order]


def init_primitives(centres, radii, spec: NetSpec, seed: int = 0, device="cuda"):
    """Initial parameters of the primitives of the octree's leaves: centre at
    the leaf's centroid, isotropic semi-axes equal to its radius (for the
    contact-point primitive a third of it, so that the 3-sigma support is the
    leaf's circumscribed sphere), identity rotation; each network
    Kaiming-uniform with zero biases except the density's, set for an opacity
    of about one half along a mean chord.  Returns (center, log_scale, quat,
    mlp) float32 tensors on ``device``."""
    rng = np.random.default_rng(seed)
    P = len(centres)
    contact = spec.primitive == "contact"
    s = np.asarray(radii, np.float64) / (3.0 if contact else 1.0)
    in_dim = 12 * spec.pe_freqs if contact else 3 + 6 * spec.pe_freqs
    dims = [in_dim] + [spec.hidden_width] * spec.hidden_layers + [spec.out_dim]
    n_params = sum(dims[i] * dims[i + 1] + dims[i + 1] for i in range(len(dims) - 1))
    mlp = np.zeros((P, n_params))
    for p in range(P):
        off = 0
        for li in range(len(dims) - 1):
            fi, fo = dims[li], dims[li + 1]
            bnd = math.sqrt(6.0 / fi)
            mlp[p, off:off + fi * fo] = rng.uniform(-bnd, bnd, fi * fo)
            off += fi * fo
            if li == len(dims) - 2:
                length = math.sqrt(2.0 * math.pi) * s[p] if contact else (4.0 / 3.0) * s[p]
                mlp[p, off + 3] = math.log(math.expm1(math.log(2.0) / length))
            off += fo
    quat = np.zeros((P, 4))
    quat[:, 0] = 1.0
    t = lambda a: torch.tensor(a, dtype=torch.float32, device=device)
    return t(centres), t(np.log(np.repeat(s[:, None], 3, 1))), t(quat), t(mlp)


def _gauss(size=11, sigma=1.5, device="cpu"):
    x = torch.arange(size, dtype=torch.float32, device=device) - size // 2
    g = torch.exp(-(x * x) / (2 * sigma * sigma))
    g = g / g.sum()
    return (g[:, None] * g[None, :])[None, None]


def ssim_tiles(x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    """Mean SSIM of image tiles x, y [T, C, h, w] (each tile padded with
    zeros, 11 x 11 Gaussian window of standard deviation 1.5)."""
    t, c, h, w = x.shape
    win = _gauss(device=x.device)
    f = lambda z: torch.nn.functional.conv2d(z.reshape(t * c, 1, h, w), win, padding=5).reshape(t, c, h, w)
    mx, my = f(x), f(y)
    vx = f(x * x) - mx * mx
    vy = f(y * y) - my * my
    cxy = f(x * y) - mx * my
    c1, c2 = 0.01 ** 2, 0.03 ** 2
    s = ((2 * mx * my + c1) * (2 * cxy + c2)) / ((mx * mx + my * my + c1) * (vx + vy + c2))
    return s.mean()


def photometric_loss(pred: torch.Tensor, target: torch.Tensor, lam: float = 0.2) -> torch.Tensor:
    """(1 - lam) mean |pred - target| + lam (1 - SSIM) over tiles [T, 3, 8, 8]."""
    return (1 - lam) * (pred - target).abs().mean() + lam * (1 - ssim_tiles(pred, target))


class TileBatches:
    """Mini-batches of tile-based training: ``views`` is a list of (ray_o,
    ray_d) device tensors of whole images given tile by tile (64 rays per
    8 x 8 tile, the image sides multiples of 8), ``targets`` their colours.
    Each batch takes ``images`` of the views and a ``frac`` of each one's
    tiles at random."""

    def __init__(self, views, targets, images: int = 4, frac: float = 0.25, seed: int = 0):
        self.views, self.targets = views, targets
        self.images, self.frac = images, frac
        self.gen = torch.Generator().manual_seed(seed)

    def sample(self):
        dev = self.views[0][0].device
        vs = torch.randperm(len(self.views), generator=self.gen)[:self.images].tolist()
        os_, ds_, ts_ = [], [], []
        for v in vs:
            o, d = self.views[v]
            nt = o.shape[0] // (TILE * TILE)
            k = max(1, int(round(nt * self.frac)))
            tiles = torch.randperm(nt, generator=self.gen)[:k].to(dev)
            idx = (tiles[:, None] * (TILE * TILE) + torch.arange(TILE * TILE, device=dev)[None]).reshape(-1)
            os_.append(o[idx])
            ds_.append(d[idx])
            ts_.append(self.targets[v][idx])
        return torch.cat(os_), torch.cat(ds_), torch.cat(ts_)


def _tiles(rgb: torch.Tensor) -> torch.Tensor:
    """[T*64, 3] rays in tile order -> [T, 3, 8, 8]."""
    return rgb.reshape(-1, TILE, TILE, 3).permute(0, 3, 1, 2)


def fit(renderer: Renderer, params, batches: TileBatches, iters: int, lam: float = 0.2,
        lrs=(1e-2, 1e-4, 1e-3), log_every: int = 0) -> List[float]:
    """Optimise params = (center, log_scale, quat, mlp) (leaf tensors) with
    Adam for ``iters`` mini-batches; returns the loss of every iteration."""
    center, log_scale, quat, mlp = params
    opt = torch.optim.Adam([{"params": [log_scale], "lr": lrs[0]},
                            {"params": [center], "lr": lrs[1]},
                            {"params": [quat, mlp], "lr": lrs[2]}])
    hist = []
    for it in range(iters):
        ro, rd, tgt = batches.sample()
        opt.zero_grad(set_to_none=True)
        rgb, _, _ = render(renderer, center, log_scale.exp(), quat, mlp, ro, rd)
        loss = photometric_loss(_tiles(rgb), _tiles(tgt), lam)
        loss.backward()
        opt.step()
        hist.append(float(loss.detach()))
        if log_every and it % log_every == 0:
            print(f"iteration {it}: loss {hist[-1]:.5f}", flush=True)
    return hist
