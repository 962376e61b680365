"""FP64 CPU oracle of the paper's own primitive: one ray-primitive interaction
per hit, at the soft contact point (test infrastructure only; shares no code
with the HIP library).

Sec. 3.2: the contact depth t* = max(0, d^T Lambda (mu - o) / d^T Lambda d)
(Eq. 2, the minimiser of Eq. 1 over t >= 0), the contact point
p* = o + t* d, the residual delta = mu - p*, and the 6-D network input
x = [d; delta] encoded component by component with L frequency levels
(12 L values: 72 for L = 6) and no identity term.  The network maps the
encoding to raw (c~, sigma~); c = sigmoid(c~), sigma = softplus(sigma~).
Sec. 3.3: C = sum_i T_i alpha_i c_i with alpha_i = 1 - exp(-sigma_i delta_i).

Readings taken where the paper leaves a choice open:
  * the Gaussian support N(mu, R diag(s^2) R^T) interacts with a ray when the
    ray passes within KAPPA = 3 Mahalanobis units of mu (the 3-sigma extent
    3DGS also culls at) and that part of the ray lies in front of the origin
    (t_c + eta > 0 on the ellipsoid of semi-axes KAPPA s);
  * hits are ordered by the unclamped minimiser t_c of Eq. 1 (equal to the
    clamped t* wherever t* > 0), ties by primitive index;
  * the Gaussian falloff multiplies the density by G = exp(-1/2 |M delta|^2),
    M = diag(s)^-1 R^T, the support's Gaussian at the contact point;
  * the scalar thickness is delta_i = sqrt(2 pi) / |M d|, the length a
    unit-height Gaussian of this covariance spans along the ray (its line
    integral), so that for t* = t_c the optical depth sigma G delta_i is the
    line integral of the density sigma exp(-1/2 |M (x - mu)|^2);
  * the encoding of a vector concatenates the per-component encodings:
    index 2L c + 2 l (+1 for the cosine) holds sin (cos) of 2^l pi x_c;
  * early termination stops after the first hit whose transmittance falls
    below the threshold (one interaction per hit).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import torch

from .render import Opts, intersect, local_frame, mlp_apply, packet_centres, _softplus, _where

__all__ = ["KAPPA", "ContactModel", "encode_vec", "contact_terms", "render_contact"]

KAPPA = 3.0


@dataclasses.dataclass(frozen=True)
class ContactModel:
    """Network of the contact-point primitive: 12 L inputs (Sec. 4.1: 72 for
    L = 6), hidden ReLU layers, out_dim outputs (RGB and density)."""
    pe_freqs: int = 6
    hidden_width: int = 32
    hidden_layers: int = 2
    out_dim: int = 4

    @property
    def in_dim(self) -> int:
        return 12 * self.pe_freqs

    def layer_dims(self):
        dims = [self.in_dim] + [self.hidden_width] * self.hidden_layers + [self.out_dim]
        return [(dims[i], dims[i + 1]) for i in range(len(dims) - 1)]

    @property
    def num_params(self) -> int:
        return sum(i * o + o for i, o in self.layer_dims())


def encode_vec(x: torch.Tensor, n_freqs: int) -> torch.Tensor:
    """gamma of each component of x [..., n] (Sec. 3.2), concatenated:
    [sin(2^0 pi x_0), cos(2^0 pi x_0), ..., cos(2^(L-1) pi x_0), sin(2^0 pi x_1), ...]."""
    feats = []
    for c in range(x.shape[-1]):
        for lvl in range(n_freqs):
            arg = (2.0 ** lvl) * math.pi * x[..., c]
            feats.append(torch.sin(arg))
            feats.append(torch.cos(arg))
    return torch.stack(feats, dim=-1)


def contact_terms(ray_o, ray_d, center, scale, quat, rr, pp, tc):
    """Per hit (ray rr, primitive pp, unclamped contact depth tc): the clamped
    depth t* (Eq. 2), the residual delta = mu - (o + t* d), the falloff
    G = exp(-|M delta|^2 / 2) and the thickness sqrt(2 pi) / |M d|."""
    o = ray_o[rr].to(center.dtype)
    d = ray_d[rr].to(center.dtype)
    mu = center[pp]
    m = local_frame(scale, quat)[pp]                         # [H,3,3], 1-sigma frame
    tstar = _where(tc.real > 0, tc, torch.zeros_like(tc))
    delta = mu - o - tstar[:, None] * d
    y = torch.einsum("hij,hj->hi", m, delta)
    falloff = torch.exp(-0.5 * (y * y).sum(-1))
    e = torch.einsum("hij,hj->hi", m, d)
    thick = math.sqrt(2.0 * math.pi) / torch.sqrt((e * e).sum(-1))
    return tstar, delta, falloff, thick


def render_contact(center, scale, quat, mlp, ray_o, ray_d, model: ContactModel, opts: Opts,
                   centre=None) -> dict:
    """Render every ray with one interaction per hit primitive (Sec. 3.2-3.3).
    Parameters float64 (or complex128) tensors, rays float64.  ``opts`` uses
    t_stop, background and order (sample counts and jitter do not apply).
    With opts.order == 1 hits follow tile order: each packet of 64 rays takes
    the order of the contact depths along its virtual ray (``centre`` as in
    the chord renderer)."""
    dt = center.dtype
    nr = ray_o.shape[0]
    isx = intersect(ray_o, ray_d, center, KAPPA * scale, quat)
    hit = isx["hit"]
    rr, pp = torch.nonzero(hit, as_tuple=True)
    rr = rr.numpy()
    pp = pp.numpy()
    if opts.order == 1:
        oc, dc = packet_centres(ray_o.real, ray_d.real) if centre is None else centre
        key_all = intersect(torch.from_numpy(np.asarray(oc, np.float64)),
                            torch.from_numpy(np.asarray(dc, np.float64)),
                            center.real.detach(), scale.real.detach(), quat.real.detach())["tc"]
    else:
        key_all = isx["tc"]
    key = key_all.real.detach()[rr, pp].numpy() if len(rr) else np.zeros(0)
    order = np.lexsort((pp, key, rr))
    rr, pp = rr[order], pp[order]
    nh = len(rr)
    counts = np.bincount(rr, minlength=nr)
    ray_off = np.zeros(nr + 1, np.int64)
    ray_off[1:] = np.cumsum(counts)
    rank = np.arange(nh) - ray_off[rr]
    rr_t, pp_t = torch.from_numpy(rr), torch.from_numpy(pp)
    tc = isx["tc"][rr_t, pp_t]
    tstar, delta, falloff, thick = contact_terms(ray_o, ray_d, center, scale, quat, rr_t, pp_t, tc)
    x = torch.cat([ray_d[rr_t].to(dt), delta], dim=-1)
    gam = encode_vec(x, model.pe_freqs)
    raw = torch.zeros((nh, model.out_dim), dtype=dt)
    rows = []
    for p in np.unique(pp):
        idx = torch.from_numpy(np.nonzero(pp == p)[0])
        rows.append((idx, mlp_apply(mlp[int(p)], gam[idx], model, opts.gate_form)))
    if rows:
        raw = raw.index_put((torch.cat([i for i, _ in rows]),), torch.cat([v for _, v in rows]))
    col = torch.sigmoid(raw[:, :3])
    sig = _softplus(raw[:, 3])
    tau = sig * falloff * thick
    bg = torch.tensor(list(opts.background), dtype=dt)
    if nh == 0:
        return {"rgb": torch.zeros((nr, 3), dtype=dt) + bg, "trans": torch.ones(nr, dtype=dt),
                "n_used": np.zeros(nr, np.int64), "ray_off": ray_off, "prim": pp, "t_c": tc,
                "t_star": tstar, "delta": delta, "tau": tau, "hit_used": np.zeros(0, bool)}
    hmax = int(counts.max())
    idx2 = (rr_t, torch.from_numpy(rank))
    tau_pad = torch.zeros((nr, hmax), dtype=dt).index_put(idx2, tau)
    t_before = torch.exp(-(torch.cumsum(tau_pad, 1) - tau_pad))
    valid = torch.zeros((nr, hmax), dtype=torch.bool)
    valid[idx2] = True
    used = valid & (t_before.real >= opts.t_stop) if opts.t_stop > 0 else valid
    alpha = 1 - torch.exp(-tau_pad)
    w = _where(used, t_before * alpha, torch.zeros_like(alpha))
    c_pad = torch.zeros((nr, hmax, 3), dtype=dt).index_put(idx2, col)
    rgb = (w[..., None] * c_pad).sum(1)
    trans = torch.exp(-_where(used, tau_pad, torch.zeros_like(tau_pad)).sum(1))
    rgb = rgb + trans[:, None] * bg
    return {"rgb": rgb, "trans": trans, "n_used": used.sum(1).numpy(), "ray_off": ray_off, "prim": pp,
            "t_c": tc, "t_star": tstar, "delta": delta, "tau": tau, "hit_used": used[idx2].numpy(),
            "raw": raw, "falloff": falloff, "thick": thick, "gamma": gam}


def contact_margins(center, scale, quat, mlp, ray_o, ray_d, model: ContactModel, opts: Opts):
    """Per ray, the smallest ReLU margin (relu_margin: distance of a gate from
    switching in units of its rounding noise) over the ray's hits."""
    from .render import relu_margin
    out = render_contact(center, scale, quat, mlp, ray_o, ray_d, model, opts)
    nr = ray_o.shape[0]
    m = np.full(nr, np.inf)
    if len(out["prim"]):
        rr = np.repeat(np.arange(nr), np.diff(out["ray_off"]))
        gam = out["gamma"].detach().real
        hm = np.full(len(rr), np.inf)
        for p in np.unique(out["prim"]):
            idx = np.nonzero(out["prim"] == p)[0]
            hm[idx] = relu_margin(mlp[int(p)], gam[torch.from_numpy(idx)], model, opts.gate_form)
        np.minimum.at(m, rr, hm)
    return out, m


def contact_loss_and_grads(scene: dict, ray_o, ray_d, model: ContactModel, opts: Opts, grad_rgb,
                           grad_trans=None, chunk: int = 4096, centre=None):
    """L = sum(grad_rgb * rgb) (+ sum(grad_trans * trans)) and its gradient
    with respect to the scene's center, scale, quat and mlp (reverse-mode
    autodiff of render_contact, discrete decisions held fixed)."""
    prm = {k: torch.from_numpy(np.asarray(scene[k], np.float64)).requires_grad_(True)
           for k in ("center", "scale", "quat", "mlp")}
    o = torch.from_numpy(np.asarray(ray_o, np.float64))
    d = torch.from_numpy(np.asarray(ray_d, np.float64))
    rgbs, trs = [], []
    for s in range(0, o.shape[0], chunk):
        e = min(o.shape[0], s + chunk)
        out = render_contact(prm["center"], prm["scale"], prm["quat"], prm["mlp"], o[s:e], d[s:e], model, opts,
                             centre=None if centre is None else (centre[0][s:e], centre[1][s:e]))
        loss = (out["rgb"] * torch.from_numpy(np.asarray(grad_rgb[s:e], np.float64))).sum()
        if grad_trans is not None:
            loss = loss + (out["trans"] * torch.from_numpy(np.asarray(grad_trans[s:e], np.float64))).sum()
        if loss.requires_grad:
            loss.backward()
        rgbs.append(out["rgb"].detach())
        trs.append(out["trans"].detach())
    grads = {k: (v.grad if v.grad is not None else torch.zeros_like(v)).numpy() for k, v in prm.items()}
    return torch.cat(rgbs).numpy(), torch.cat(trs).numpy(), grads
