"""Seeded synthetic inputs for the MLP-Splatting render path.

This module only draws inputs: primitive parameters (center, scale, quaternion,
per-primitive MLP weights), pinhole cameras and their rays, and upstream
gradients.  It contains none of the rendering arithmetic, so that the FP64
oracle (``oracle/``) and the HIP library (``paper_2606_03877_amd``) can both be
fed the very same arrays without sharing any code.

Workload shapes follow the paper's setting (Sec. 3.1 primitives with a centre,
scale vector and unit quaternion, each owning an MLP; Sec. 4.1 pinhole
rendering of full frames) at the five synthetic configurations listed in
``CONFIGS``.  The paper's own scenes (Replica, ScanNet) are not available;
these seeded scenes stand in for them.

Weight layout per primitive (flat float32 vector): for every layer, first the
weight matrix W[out, in] in row-major order, then the bias b[out].  Layers are
input -> hidden (x hidden_layers) -> output.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

__all__ = [
    "Config", "CONFIGS", "layer_dims", "num_params", "make_scene",
    "make_camera", "camera_rays", "make_rays", "make_batch_rays",
    "upstream_grads", "tile_order",
]


@dataclasses.dataclass(frozen=True)
class Config:
    idx: int
    name: str
    num_prims: int
    pe_freqs: int
    hidden_width: int
    hidden_layers: int
    out_dim: int
    center_law: str                 # "uniform" | "clusters"
    scale_law: Tuple                # ("loguniform", lo, hi) | ("lognormal", mu, sigma)
    views: Tuple[Tuple[int, int], ...]   # (width, height) per camera
    camera_radius: float
    samples_fixed: int              # K per hit; 0 = proportional to chord length
    samples_min: int = 8
    samples_max: int = 128
    samples_per_unit: float = 128.0
    t_stop: float = 0.0             # 0 = no early termination
    batch_rays: int = 0             # >0: random batch over the views' pixels
    jitter: int = 1                 # 1 = stratified (hashed) offsets, 0 = midpoints
    fov_deg: float = 50.0
    # "chord": K samples of the hit chord, input the local position (3 + 6L
    # encoded values); "contact": the paper's primitive, one interaction at
    # the contact point, input [d; delta] (12 L encoded values), scale = the
    # Gaussian support's standard deviations
    primitive: str = "chord"

    @property
    def in_dim(self) -> int:
        return 12 * self.pe_freqs if self.primitive == "contact" else 3 + 6 * self.pe_freqs

    @property
    def num_rays(self) -> int:
        if self.batch_rays:
            return self.batch_rays
        return sum(w * h for w, h in self.views)


CONFIGS: List[Config] = [
    Config(0, "tiny-fp32", 8, 4, 32, 2, 4, "uniform", ("loguniform", 0.1, 0.4),
           ((64, 64),), 3.0, 32, t_stop=0.0),
    Config(1, "frame-800", 64, 6, 64, 3, 4, "uniform", ("loguniform", 0.05, 0.3),
           ((800, 800),), 3.0, 64, t_stop=1e-4),
    Config(2, "train-batch", 64, 6, 64, 3, 4, "uniform", ("loguniform", 0.05, 0.3),
           tuple([(800, 800)] * 8), 3.0, 64, t_stop=1e-4, batch_rays=65536),
    Config(3, "large-1080p", 256, 6, 128, 4, 20, "clusters", ("lognormal", math.log(0.08), 0.5),
           ((1920, 1080),), 4.0, 96, t_stop=1e-4),
    Config(4, "multiview", 512, 6, 64, 3, 4, "uniform", ("loguniform", 0.02, 0.5),
           tuple([(256, 256)] * 4 + [(512, 512)] * 4 + [(800, 800)] * 4 + [(1024, 768)] * 4),
           3.0, 0, t_stop=1e-4),
    # the 64-wide network with 16 identity feature channels (39-64x3-20, a
    # compiled shape no workload above uses): a parity-test case
    Config(5, "features-64", 64, 6, 64, 3, 20, "uniform", ("loguniform", 0.05, 0.3),
           ((800, 800),), 3.0, 64, t_stop=1e-4),
    # the paper's own primitive (Sec. 3.2, Sec. 4.1): 72-32-32-4 networks on
    # the encoded [d; delta], one interaction per hit; 2048 primitives (the
    # paper's octree gives 1,344-3,862 on Replica) of Gaussian standard
    # deviations 0.02-0.08, an 800x800 frame
    Config(6, "contact-800", 2048, 6, 32, 2, 4, "uniform", ("loguniform", 0.02, 0.08),
           ((800, 800),), 3.0, 1, t_stop=1e-4, jitter=0, primitive="contact"),
]


def layer_dims(cfg_or_dims) -> List[Tuple[int, int]]:
    """(in, out) for every layer of one primitive's MLP."""
    if isinstance(cfg_or_dims, Config):
        c = cfg_or_dims
        dims = [c.in_dim] + [c.hidden_width] * c.hidden_layers + [c.out_dim]
    else:
        dims = list(cfg_or_dims)
    return [(dims[i], dims[i + 1]) for i in range(len(dims) - 1)]


def num_params(cfg: Config) -> int:
    return sum(i * o + o for i, o in layer_dims(cfg))


def _draw_centers(rng, cfg: Config, n: int) -> np.ndarray:
    if cfg.center_law == "uniform":
        return rng.uniform(-1.0, 1.0, size=(n, 3))
    # mixture of 8 isotropic Gaussian clusters, clipped to [-2, 2]^3
    means = rng.uniform(-1.5, 1.5, size=(8, 3))
    which = rng.integers(0, 8, size=n)
    pts = means[which] + 0.3 * rng.standard_normal(size=(n, 3))
    return np.clip(pts, -2.0, 2.0)


def _draw_scales(rng, cfg: Config, n: int) -> np.ndarray:
    law = cfg.scale_law
    if law[0] == "loguniform":
        return np.exp(rng.uniform(math.log(law[1]), math.log(law[2]), size=(n, 3)))
    return np.exp(law[1] + law[2] * rng.standard_normal(size=(n, 3)))


def make_scene(cfg: Config, seed: Optional[int] = None) -> dict:
    """Draw one scene.  Order of draws: all centres, all scales, all
    quaternions, then each primitive's weights layer by layer.

    Weights are Kaiming-uniform U(-sqrt(6/fan_in), +sqrt(6/fan_in)); biases are
    zero except the density output's bias, set to softplus^-1(ln 2 / Lbar) with
    Lbar = 4/3 * (s_x s_y s_z)^(1/3) (mean chord of the volume-equivalent
    sphere), so a hit's opacity is about one half on average.  For the
    contact-point primitive it is softplus^-1(2 / (sqrt(2 pi) sbar)),
    sbar = (s_x s_y s_z)^(1/3): a ray through the centre sees optical depth 2.
    """
    if seed is None:
        seed = 1000 * cfg.idx
    rng = np.random.default_rng(seed)
    n = cfg.num_prims
    center = _draw_centers(rng, cfg, n)
    scale = _draw_scales(rng, cfg, n)
    q = rng.standard_normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    dims = layer_dims(cfg)
    mlp = np.zeros((n, num_params(cfg)), dtype=np.float64)
    for p in range(n):
        off = 0
        for li, (fi, fo) in enumerate(dims):
            bound = math.sqrt(6.0 / fi)
            mlp[p, off:off + fi * fo] = rng.uniform(-bound, bound, size=fi * fo)
            off += fi * fo
            if li == len(dims) - 1:
                if cfg.primitive == "contact":
                    # optical depth 2 for a ray through the centre: density
                    # times the Gaussian's length sqrt(2 pi) sbar along a ray
                    target = 2.0 / (math.sqrt(2.0 * math.pi) * float(np.prod(scale[p])) ** (1.0 / 3.0))
                else:
                    lbar = (4.0 / 3.0) * float(np.prod(scale[p])) ** (1.0 / 3.0)
                    target = math.log(2.0) / lbar
                mlp[p, off + 3] = math.log(math.expm1(target))
            off += fo
    return {
        "center": center.astype(np.float32),
        "scale": scale.astype(np.float32),
        "quat": q.astype(np.float32),
        "mlp": mlp.astype(np.float32),
    }


def make_camera(rng, width: int, height: int, radius: float, fov_deg: float = 50.0) -> dict:
    """Pinhole camera on a seeded point of the sphere of the given radius,
    looking at the origin, +z up (+y if the view is nearly vertical)."""
    v = rng.standard_normal(3)
    eye = radius * v / np.linalg.norm(v)
    fwd = -eye / np.linalg.norm(eye)
    up = np.array([0.0, 0.0, 1.0])
    if abs(float(fwd @ up)) > 0.99:
        up = np.array([0.0, 1.0, 0.0])
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    true_up = np.cross(right, fwd)
    f = 0.5 * height / math.tan(0.5 * math.radians(fov_deg))
    return {"eye": eye, "fwd": fwd, "right": right, "up": true_up, "focal": f,
            "width": width, "height": height}


def tile_order(width: int, height: int, tile: int = 8) -> np.ndarray:
    """Pixel indices (row-major y*width+x) listed tile by tile (tiles in
    row-major order, pixels row-major inside a tile), so 64 consecutive rays
    of an 8x8 tile form one coherent packet.  Ragged edge tiles are kept."""
    ys, xs = [], []
    for ty in range(0, height, tile):
        for tx in range(0, width, tile):
            yy, xx = np.meshgrid(np.arange(ty, min(ty + tile, height)),
                                 np.arange(tx, min(tx + tile, width)), indexing="ij")
            ys.append(yy.ravel())
            xs.append(xx.ravel())
    y = np.concatenate(ys)
    x = np.concatenate(xs)
    return (y * width + x).astype(np.int64)


def _pixel_dirs(cam: dict, pix: np.ndarray) -> np.ndarray:
    w = cam["width"]
    y = (pix // w).astype(np.float64)
    x = (pix % w).astype(np.float64)
    u = (x + 0.5 - 0.5 * cam["width"]) / cam["focal"]
    v = (y + 0.5 - 0.5 * cam["height"]) / cam["focal"]
    d = cam["fwd"][None, :] + u[:, None] * cam["right"][None, :] - v[:, None] * cam["up"][None, :]
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def camera_rays(cam: dict, tiled: bool = True) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """All rays of one camera: (origin [N,3] f32, direction [N,3] f32 (unit
    in f64 before rounding), pixel index [N])."""
    n = cam["width"] * cam["height"]
    pix = tile_order(cam["width"], cam["height"]) if tiled else np.arange(n)
    d = _pixel_dirs(cam, pix)
    o = np.ascontiguousarray(np.broadcast_to(cam["eye"], d.shape), dtype=np.float32)
    return o, np.ascontiguousarray(d, dtype=np.float32), pix


def packet_tile_rays(cam: dict, packet: int = 64) -> np.ndarray:
    """Per packet of ``packet`` consecutive rays of the camera's tile-ordered
    rays: the ray from the eye through the centre of the packet's pixel
    bounding box on the image plane -- for an 8x8 tile (view sides multiples
    of 8), the tile's centre.  Returns float32 [n_packets, 6] (origin xyz,
    unit direction xyz)."""
    n = cam["width"] * cam["height"]
    pix = tile_order(cam["width"], cam["height"])
    out = np.empty(((n + packet - 1) // packet, 6), np.float64)
    for k, s in enumerate(range(0, n, packet)):
        p = pix[s:s + packet]
        y, x = p // cam["width"], p % cam["width"]
        xc = 0.5 * (x.min() + x.max() + 1)   # (pixel i spans [i, i + 1))
        yc = 0.5 * (y.min() + y.max() + 1)
        u = (xc - 0.5 * cam["width"]) / cam["focal"]
        v = (yc - 0.5 * cam["height"]) / cam["focal"]
        d = cam["fwd"] + u * cam["right"] - v * cam["up"]
        out[k, :3] = cam["eye"]
        out[k, 3:] = d / np.linalg.norm(d)
    return out.astype(np.float32)


def make_rays(cfg: Config, seed: Optional[int] = None):
    """Rays of the configuration: full frames of every view, tile-ordered, or
    (batch_rays > 0) a uniform random batch over (view, pixel) with
    replacement.  Returns (origin, direction, info)."""
    if seed is None:
        seed = 1000 * cfg.idx + 1
    rng = np.random.default_rng(seed)
    cams = [make_camera(rng, w, h, cfg.camera_radius, cfg.fov_deg) for (w, h) in cfg.views]
    if cfg.batch_rays:
        brng = np.random.default_rng(1000 * cfg.idx + 2)
        view = brng.integers(0, len(cams), size=cfg.batch_rays)
        sizes = np.array([c["width"] * c["height"] for c in cams])
        pix = (brng.random(cfg.batch_rays) * sizes[view]).astype(np.int64)
        o = np.empty((cfg.batch_rays, 3), np.float32)
        d = np.empty((cfg.batch_rays, 3), np.float32)
        for vi, cam in enumerate(cams):
            m = view == vi
            dd = _pixel_dirs(cam, pix[m])
            d[m] = dd.astype(np.float32)
            o[m] = cam["eye"].astype(np.float32)
        return o, d, {"cams": cams, "view": view, "pix": pix}
    os_, ds_, views, pixs = [], [], [], []
    for vi, cam in enumerate(cams):
        o, d, pix = camera_rays(cam)
        os_.append(o)
        ds_.append(d)
        views.append(np.full(len(pix), vi))
        pixs.append(pix)
    return (np.concatenate(os_), np.concatenate(ds_),
            {"cams": cams, "view": np.concatenate(views), "pix": np.concatenate(pixs)})


def make_batch_rays(cfg: Config, n: int, seed: int):
    """A seeded random subset of n rays of the configuration's views (used to
    time or check a bounded sample of a full workload)."""
    o, d, info = make_rays(cfg)
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(len(o), size=min(n, len(o)), replace=False))
    return o[idx], d[idx], idx


def upstream_grads(cfg: Config, num_rays: int, seed: Optional[int] = None):
    """Seeded N(0,1)/R upstream gradients for RGB (and features)."""
    if seed is None:
        seed = 1000 * cfg.idx + 4
    rng = np.random.default_rng(seed)
    g_rgb = (rng.standard_normal((num_rays, 3)) / num_rays).astype(np.float32)
    cf = cfg.out_dim - 4
    g_feat = (rng.standard_normal((num_rays, cf)) / num_rays).astype(np.float32) if cf > 0 else None
    return g_rgb, g_feat
