"""FP64 CPU oracle of the MLP-Splatting render path (test infrastructure only).

This is a plain, slow, direct transcription of what the method computes; it is
used only by the tests, by the smoke check and by the benchmark's CPU-baseline
leg.  It shares no code with the HIP library.

Every function works for float64 tensors (with autograd, which gives the
oracle's analytic gradient) and for complex128 tensors (complex-step
differentiation).  All discrete decisions -- hit or miss, depth order, sample
count, ReLU gate, the early-termination cut -- are taken on real parts and are
held fixed under differentiation.

Readings taken where the paper leaves a choice open:
  * quaternion order (w, x, y, z), Hamilton product, normalised before use;
  * the scale vector gives the semi-axes of a hard ellipsoid support; density
    is zero outside it (no Gaussian falloff inside);
  * the MLP input is the scale-normalised local position p of a sample, with
    an identity term in front of the sin/cos encoding;
  * K stratified samples per hit interval, bin width Delta = L / K used as the
    thickness in alpha = 1 - exp(-sigma * Delta);
  * hits are composited one after the other (hit-major), sorted by the
    unclamped contact depth, ties broken by primitive index;
  * tile order (option): every ray of a packet of 64 consecutive rays takes
    the order of the contact depths along one virtual ray of the packet,
    whose origin is the mean of the packet's origins and whose direction is
    the normalised sum of its directions (for an 8x8 pixel tile of a pinhole
    camera, the ray through the tile centre up to a second-order term);
  * early termination stops after the first sample whose transmittance falls
    below the threshold;
  * ReLU gates are decisions a floating-point sum takes: with
    Opts.gate_form "bf16" or "bf16x3" they are taken in that arithmetic
    (``gate_preacts``: operands rounded to bfloat16, or carried as bfloat16
    hi + lo pairs multiplied as hi*hi + hi*lo + lo*hi, sums exact), and the
    network is then evaluated and differentiated in FP64 on the branch those
    gates select (a = z where the gate is open, 0 where it is closed);
  * slot features (option): the local offset u of a hit is taken at the
    unclamped contact point (u = -p_c; the paper's clamp moves the point to the
    ray origin only when the camera is inside the support), the clip to the
    unit cube is inactive for a hit (|p_c| < 1), the directional frame is the
    regular tetrahedron (1,1,1), (1,-1,-1), (-1,1,-1), (-1,-1,1) over sqrt 3,
    and a hit's feature is composited with the hit's total volumetric weight
    (the sum of its samples' weights).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np
import torch

from .pcg import sample_offsets

__all__ = ["Model", "Opts", "quat_to_rotmat", "local_frame", "intersect",
           "encode", "mlp_apply", "bf16_round", "split_bf16", "gate_preacts", "relu_noise", "relu_margin",
           "packet_centres", "render",
           "TETRA", "slot_gates"]

PACKET = 64   # rays per packet (an 8x8 pixel tile)


@dataclasses.dataclass(frozen=True)
class Model:
    pe_freqs: int
    hidden_width: int
    hidden_layers: int
    out_dim: int

    @property
    def in_dim(self) -> int:
        return 3 + 6 * self.pe_freqs

    def layer_dims(self):
        dims = [self.in_dim] + [self.hidden_width] * self.hidden_layers + [self.out_dim]
        return [(dims[i], dims[i + 1]) for i in range(len(dims) - 1)]

    @property
    def num_params(self) -> int:
        return sum(i * o + o for i, o in self.layer_dims())


@dataclasses.dataclass(frozen=True)
class Opts:
    samples_fixed: int = 32          # K per hit; 0 = proportional to chord length
    samples_min: int = 8
    samples_max: int = 128
    samples_per_unit: float = 128.0
    t_stop: float = 0.0              # 0 = no early termination
    jitter: int = 1                  # 1 = hashed stratified offsets, 0 = midpoints
    jitter_seed: int = 0
    background: Sequence[float] = (0.0, 0.0, 0.0)
    order: int = 0                   # 0 = each ray's own contact depth; 1 = tile order
    gate_form: str = "fp64"          # arithmetic of the ReLU gate decisions: fp64 | bf16 | bf16x3


def _where(cond, a, b):
    return torch.where(cond, a, b)


def quat_to_rotmat(q: torch.Tensor) -> torch.Tensor:
    """Rotation matrix R(q) of the normalised quaternion (w, x, y, z), Hamilton
    convention (Sec. 3.1: a unit quaternion gives the primitive's rotation)."""
    n = torch.sqrt((q * q).sum(-1, keepdim=True))
    w, x, y, z = (q / n).unbind(-1)
    r = torch.stack([
        1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
        2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
        2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y),
    ], dim=-1)
    return r.reshape(q.shape[:-1] + (3, 3))


def local_frame(scale: torch.Tensor, quat: torch.Tensor) -> torch.Tensor:
    """M = diag(s)^-1 R(q)^T, so that p = M (x - mu) is the scale-normalised
    local position and (x-mu)^T Lambda (x-mu) = |p|^2 with
    Lambda = R diag(s^-2) R^T (Sec. 3.2, the support metric under Eq. 1)."""
    r = quat_to_rotmat(quat)
    return r.transpose(-1, -2) / scale[..., :, None]


def intersect(ray_o, ray_d, center, scale, quat):
    """Ray/support test for every (ray, primitive) pair.

    With o_l = M(o - mu), d_l = M d and a = |d_l|^2 the contact depth is
    t_c = -(o_l . d_l) / a, which is the unclamped minimiser of Eq. 1 (its
    clamped form is Eq. 2).  The chord of the ellipsoid |p| <= 1 is
    [t_c - eta, t_c + eta] with g = 1 - |o_l + t_c d_l|^2 and eta = sqrt(g/a).
    A pair is a hit iff g > 0 and t_c + eta > 0; the interval starts at
    max(t_c - eta, 0) (the clamp of Eq. 2).
    Returns dict of [R, P] tensors.
    """
    m = local_frame(scale, quat)                                  # [P,3,3]
    rel = ray_o[:, None, :].to(m.dtype) - center[None, :, :]     # [R,P,3]
    ol = torch.einsum("pij,rpj->rpi", m, rel)
    dl = torch.einsum("pij,rj->rpi", m, ray_d.to(m.dtype))
    a = (dl * dl).sum(-1)
    tc = -(ol * dl).sum(-1) / a
    pc = ol + tc[..., None] * dl
    g = 1 - (pc * pc).sum(-1)
    gpos = g.real > 0
    eta = torch.sqrt(_where(gpos, g, torch.ones_like(g)) / a)
    eta = _where(gpos, eta, torch.zeros_like(eta))
    hit = gpos & ((tc + eta).real > 0)
    ta_raw = tc - eta
    ta = _where(ta_raw.real > 0, ta_raw, torch.zeros_like(ta_raw))
    tb = tc + eta
    return {"ol": ol, "dl": dl, "a": a, "tc": tc, "g": g, "eta": eta,
            "hit": hit, "ta": ta, "tb": tb}


def encode(p: torch.Tensor, n_freqs: int) -> torch.Tensor:
    """gamma(p) = [p, then per level l: sin(2^l pi p), cos(2^l pi p)] (Sec. 3.2
    positional encoding, applied per coordinate, with an identity term)."""
    feats = [p]
    for lvl in range(n_freqs):
        arg = (2.0 ** lvl) * math.pi * p
        feats.append(torch.sin(arg))
        feats.append(torch.cos(arg))
    return torch.cat(feats, dim=-1)


def bf16_round(v) -> np.ndarray:
    """Nearest bfloat16 value of each float32 value (ties to even), as float64:
    bfloat16 keeps the sign, the 8 exponent bits and the top 7 fraction bits
    of a float32, so the low 16 bits are rounded away."""
    f = np.ascontiguousarray(np.asarray(v, np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def split_bf16(v):
    """(hi, lo) = (bf16(v), bf16(v - hi)) of the float32 values of v."""
    f = np.asarray(v, np.float64).astype(np.float32).astype(np.float64)
    hi = bf16_round(f)
    return hi, bf16_round(f - hi)


def _gate_dot(a, w, form):
    """a @ w.T with both operands in the given bfloat16 form; sums exact."""
    if form == "bf16":
        return bf16_round(a) @ bf16_round(w).T
    ah, al = split_bf16(a)
    wh, wl = split_bf16(w)
    return ah @ wh.T + al @ wh.T + ah @ wl.T


def gate_preacts(theta, x, model: Model, form: str):
    """Pre-activations of the hidden layers as the gate decisions see them in
    the bfloat16 forms: each layer's input (float32 values) and weights are
    rounded to bfloat16 (form "bf16") or split into hi + lo pairs ("bf16x3"),
    products summed without further rounding; the first layer's bias enters
    as the weight of a constant input 1 (in the same form), the other biases
    as float32 values.  Returns [z] per hidden layer, float64 [rows, width]."""
    th = np.asarray(theta.detach().real if torch.is_tensor(theta) else theta, np.float64)
    h = np.asarray(x.detach().real if torch.is_tensor(x) else x, np.float64).astype(np.float32).astype(np.float64)
    out = []
    off = 0
    for li, (fi, fo) in enumerate(model.layer_dims()[:-1]):
        w = th[off:off + fi * fo].reshape(fo, fi)
        off += fi * fo
        b = th[off:off + fo].astype(np.float32).astype(np.float64)
        off += fo
        if li == 0:
            z = _gate_dot(np.concatenate([h, np.ones((h.shape[0], 1))], 1), np.concatenate([w, b[:, None]], 1), form)
        else:
            z = _gate_dot(h, w, form) + b
        out.append(z)
        h = np.maximum(z, 0.0).astype(np.float32).astype(np.float64)
    return out


def mlp_apply(theta: torch.Tensor, x: torch.Tensor, model: Model, gate_form: str = "fp64") -> torch.Tensor:
    """One primitive's MLP: ReLU hidden layers, linear output (raw values).
    gate_form other than "fp64": the ReLU gates are taken from
    ``gate_preacts`` in that form, and a = z where open, 0 where closed."""
    off = 0
    h = x
    dims = model.layer_dims()
    gates = None
    if gate_form != "fp64":
        gates = [torch.from_numpy(z > 0) for z in gate_preacts(theta, x, model, gate_form)]
    for li, (fi, fo) in enumerate(dims):
        w = theta[off:off + fi * fo].reshape(fo, fi)
        off += fi * fo
        b = theta[off:off + fo]
        off += fo
        h = h @ w.transpose(0, 1) + b
        if li < len(dims) - 1:
            open_ = h.real > 0 if gates is None else gates[li]
            h = _where(open_, h, torch.zeros_like(h))
    return h


def relu_noise(theta, x, model: Model):
    """Pre-activations of the hidden layers and the rounding noise they carry.

    Model (the standard probabilistic model of rounding error): every
    product W_ji h_i and every bias b_j of the forward pass carries an
    independent relative error of standard deviation u.  To first order in u
    the noise of z = W h + b then has standard deviation u e with
        e^(1) = sqrt(W1^2 x^2 + b1^2)
        e^(l) = sqrt(Wl^2 (a^(l-1) (e^(l-1))^2 + (h^(l-1))^2) + bl^2),
    squares elementwise, a^(l-1) the 0/1 ReLU gates of the layer input (a
    closed gate stops the noise), covariances between units neglected (exact
    for the first two hidden layers).  Returns [(z, e)] per hidden layer,
    each [rows, width].  Float64, no autograd.
    """
    th = np.asarray(theta.detach().real if torch.is_tensor(theta) else theta, np.float64)
    h = np.asarray(x.detach().real if torch.is_tensor(x) else x, np.float64)
    e2 = np.zeros_like(h)
    act = np.zeros_like(h)
    out = []
    off = 0
    for fi, fo in model.layer_dims()[:-1]:
        w = th[off:off + fi * fo].reshape(fo, fi)
        off += fi * fo
        b = th[off:off + fo]
        off += fo
        z = h @ w.T + b
        e2 = (act * e2 + h * h) @ (w * w).T + b * b
        out.append((z, np.sqrt(e2)))
        act = (z > 0).astype(np.float64)
        h = np.maximum(z, 0.0)
    return out


def relu_margin(theta, x, model: Model, gate_form: str = "fp64") -> np.ndarray:
    """Distance of each row's closest ReLU gate from its switching point in
    units of its rounding noise: min over hidden units of |z| / e
    (``relu_noise``).  An implementation with unit roundoff u takes a gate
    whose margin is within a small multiple of u either way with appreciable
    probability: such gates are decisions that two correct implementations
    may take differently, and the gradient jumps there.  With a bfloat16
    gate_form, z is that form's pre-activation (``gate_preacts``)."""
    m = np.full(np.shape(x)[0], np.inf)
    noise = relu_noise(theta, x, model)
    if gate_form != "fp64":
        noise = [(zg, e) for zg, (_, e) in zip(gate_preacts(theta, x, model, gate_form), noise)]
    for z, e in noise:
        with np.errstate(divide="ignore", invalid="ignore"):
            r = np.where(e > 0, np.abs(z) / e, np.inf)
        m = np.minimum(m, r.min(1))
    return m


def _softplus(o):
    pos = o.real > 0
    return _where(pos, o + torch.log1p(torch.exp(-o)), torch.log1p(torch.exp(o)))


TETRA = np.array([[1.0, 1.0, 1.0], [1.0, -1.0, -1.0], [-1.0, 1.0, -1.0], [-1.0, -1.0, 1.0]]) / math.sqrt(3.0)


def slot_gates(u: torch.Tensor) -> torch.Tensor:
    """g_k = softmax_k(a_k . u) over the four directions of the tetrahedral
    frame (Sec. 3.4, the feature-embedding equation); u [..., 3] -> [..., 4]."""
    s = u @ torch.from_numpy(TETRA.T).to(u.dtype)
    s = s - s.real.max(-1, keepdim=True).values.detach()
    e = torch.exp(s)
    return e / e.sum(-1, keepdim=True)


def packet_centres(ray_o, ray_d, packet: int = PACKET):
    """Virtual ray of every packet of ``packet`` consecutive rays (the last one
    may be shorter), repeated for each of its rays: origin = mean of the
    packet's origins, direction = normalised sum of its directions, (0, 0, 1)
    if that sum vanishes.  The tile-order variant of the depth sort (Sec. 3.3,
    after Eq. 2; App. on tile-based rendering) solves Eq. 1 along this ray.
    Returns float64 numpy arrays ([R,3], [R,3])."""
    o = np.asarray(ray_o, np.float64)
    d = np.asarray(ray_d, np.float64)
    oc = np.empty_like(o)
    dc = np.empty_like(d)
    for s in range(0, len(o), packet):
        e = min(len(o), s + packet)
        oc[s:e] = o[s:e].mean(0)
        v = d[s:e].sum(0)
        n = np.linalg.norm(v)
        dc[s:e] = v / n if n > 0 else np.array([0.0, 0.0, 1.0])
    return oc, dc


def render(center, scale, quat, mlp, ray_o, ray_d, model: Model, opts: Opts,
           ray_index_base: int = 0, keep_samples: bool = False, ray_ids=None,
           centre=None, slots=None) -> dict:
    """Render every ray (Sec. 3.3 front-to-back compositing over the depth-
    sorted hits, each hit sampled at K stratified points of its chord).

    Parameters are float64 (or complex128) tensors; rays are float64.
    ``ray_index_base`` offsets the ray index fed to the sample-offset hash, so a
    subset of a batch can be rendered with the batch's own offsets; ``ray_ids``
    (one index per ray) overrides it for scattered subsets.  With
    ``opts.order == 1`` hits are ordered along each ray's packet virtual ray:
    ``centre`` = (origins, directions) per ray, by default
    ``packet_centres(ray_o, ray_d)`` (rays given from a packet boundary).
    With ``slots`` ([P, 4, C] slot embeddings) the result also holds
    ``slot_feat`` [R, C]: every hit's feature f = sum_k g_k e_k with gates
    g = slot_gates(u) of its local offset u = -p_c, composited with the hit's
    total volumetric weight (Sec. 3.4, F = sum_i T_i alpha_i f_i).
    """
    dt = center.dtype
    nr = ray_o.shape[0]
    npr = center.shape[0]
    isx = intersect(ray_o, ray_d, center, scale, quat)
    hit = isx["hit"]
    # --- depth order: ascending (key, primitive index) per ray, the key being
    # the contact depth along the ray itself or along its packet's virtual ray
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
    tcr = key_all.real.detach()[rr, pp].numpy() if len(rr) else np.zeros(0)
    order = np.lexsort((pp, tcr, rr))
    rr, pp = rr[order], pp[order]
    nh = len(rr)
    counts = np.bincount(rr, minlength=nr)
    ray_off = np.zeros(nr + 1, np.int64)
    ray_off[1:] = np.cumsum(counts)
    rank = np.arange(nh) - ray_off[rr]
    rr_t = torch.from_numpy(rr)
    pp_t = torch.from_numpy(pp)
    tc = isx["tc"][rr_t, pp_t]
    eta = isx["eta"][rr_t, pp_t]
    ta = isx["ta"][rr_t, pp_t]
    tb = isx["tb"][rr_t, pp_t]
    ol = isx["ol"][rr_t, pp_t]
    dl = isx["dl"][rr_t, pp_t]
    length = tb - ta
    # --- samples per hit ---
    if opts.samples_fixed > 0:
        kh = np.full(nh, opts.samples_fixed, np.int64)
    else:
        kh = np.ceil(opts.samples_per_unit * length.real.detach().numpy()).astype(np.int64)
        kh = np.clip(kh, opts.samples_min, opts.samples_max)
    delta = length / torch.from_numpy(kh).to(dt)
    # flat samples in (ray, rank, k) order
    hs = np.repeat(np.arange(nh), kh)
    hoff = np.zeros(nh + 1, np.int64)
    hoff[1:] = np.cumsum(kh)
    kk = np.arange(len(hs)) - hoff[hs]
    if opts.jitter:
        gid = (np.asarray(ray_ids, np.int64)[rr[hs]] if ray_ids is not None
               else rr[hs] + ray_index_base)
        u = sample_offsets(opts.jitter_seed, gid, rank[hs], kk)
    else:
        u = np.full(len(hs), 0.5)
    hs_t = torch.from_numpy(hs)
    tk = ta[hs_t] + (torch.from_numpy(kk).to(dt) + torch.from_numpy(u).to(dt)) * delta[hs_t]
    pk = ol[hs_t] + tk[:, None] * dl[hs_t]
    # --- per-primitive MLPs ---
    gam = encode(pk, model.pe_freqs)
    raw = torch.zeros((len(hs), model.out_dim), dtype=dt)
    sprim = pp[hs]
    out_rows = []
    for p in np.unique(sprim):
        idx = torch.from_numpy(np.nonzero(sprim == p)[0])
        out_rows.append((idx, mlp_apply(mlp[int(p)], gam[idx], model, opts.gate_form)))
    if out_rows:
        raw = raw.index_put(tuple([torch.cat([i for i, _ in out_rows])]),
                            torch.cat([v for _, v in out_rows]))
    col = torch.sigmoid(raw[:, :3])
    sig = _softplus(raw[:, 3])
    feat = raw[:, 4:]
    tau = sig * delta[hs_t]
    # --- compositing (padded per ray, hit-major sample order) ---
    sray = rr[hs]
    sc = np.bincount(sray, minlength=nr) if len(hs) else np.zeros(nr, np.int64)
    soff = np.zeros(nr + 1, np.int64)
    soff[1:] = np.cumsum(sc)
    smax = int(sc.max()) if nr and len(hs) else 0
    pos = np.arange(len(hs)) - soff[sray]
    cf = model.out_dim - 4
    bg = torch.tensor(list(opts.background), dtype=dt)
    if smax == 0:
        rgb = torch.zeros((nr, 3), dtype=dt) + bg
        out = _pack(rgb, torch.ones(nr, dtype=dt), torch.zeros((nr, cf), dtype=dt),
                    np.zeros(nr, np.int64), ray_off, pp, tc, eta, ta, tb, kh, isx, None)
        if slots is not None:
            out["slot_feat"] = torch.zeros((nr, slots.shape[-1]), dtype=dt)
        return out
    tau_pad = torch.zeros((nr, smax), dtype=dt)
    idx2 = (torch.from_numpy(sray), torch.from_numpy(pos))
    tau_pad = tau_pad.index_put(idx2, tau)
    s_incl = torch.cumsum(tau_pad, dim=1)
    s_excl = s_incl - tau_pad
    t_before = torch.exp(-s_excl)
    valid = torch.zeros((nr, smax), dtype=torch.bool)
    valid[idx2] = True
    if opts.t_stop > 0:
        used = valid & (t_before.real >= opts.t_stop)
    else:
        used = valid
    alpha = 1 - torch.exp(-tau_pad)
    w = _where(used, t_before * alpha, torch.zeros_like(alpha))
    c_pad = torch.zeros((nr, smax, 3), dtype=dt).index_put(idx2, col)
    rgb = (w[..., None] * c_pad).sum(1)
    s_used = _where(used, tau_pad, torch.zeros_like(tau_pad)).sum(1)
    trans = torch.exp(-s_used)
    rgb = rgb + trans[:, None] * bg
    if cf > 0:
        f_pad = torch.zeros((nr, smax, cf), dtype=dt).index_put(idx2, feat)
        fout = (w[..., None] * f_pad).sum(1)
    else:
        fout = torch.zeros((nr, 0), dtype=dt)
    n_used = used.sum(1).numpy()
    slot_feat = None
    if slots is not None:
        # the hit's weight: the sum of its samples' compositing weights
        w_hit = torch.zeros(nh, dtype=dt).index_add(0, hs_t, w[idx2])
        u_loc = -(ol + tc[:, None] * dl)                   # -p_c, inside the unit ball
        assert nh == 0 or float(u_loc.real.detach().abs().max()) < 1.0
        g = slot_gates(u_loc)                               # [nh, 4]
        f_hit = (g[:, :, None] * slots[pp_t]).sum(1)        # [nh, C]
        slot_feat = torch.zeros((nr, slots.shape[-1]), dtype=dt).index_add(
            0, rr_t, w_hit[:, None] * f_hit)
    samples = None
    if keep_samples:
        margin = np.full(len(hs), np.inf)
        for p in np.unique(sprim):
            idx = np.nonzero(sprim == p)[0]
            margin[idx] = relu_margin(mlp[int(p)], gam[torch.from_numpy(idx)], model, opts.gate_form)
        samples = {"hit": hs, "k": kk, "u": u, "t": tk, "p": pk, "c": col, "sigma": sig,
                   "f": feat, "tau": tau, "ray": sray, "relu_margin": margin}
    out = _pack(rgb, trans, fout, n_used, ray_off, pp, tc, eta, ta, tb, kh, isx, samples)
    if slot_feat is not None:
        out["slot_feat"] = slot_feat
    return out


def _pack(rgb, trans, fout, n_used, ray_off, pp, tc, eta, ta, tb, kh, isx, samples):
    g = isx["g"].real.detach()
    front = (isx["tc"] + isx["eta"]).real.detach() > 0
    cand = g[front] if front.any() else g.flatten()
    return {
        "rgb": rgb, "trans": trans, "feat": fout, "n_used": n_used,
        "ray_off": ray_off, "prim": pp, "t_c": tc, "eta": eta, "t_a": ta, "t_b": tb,
        "K": kh, "min_abs_g": float(cand.abs().min()) if cand.numel() else float("inf"),
        "samples": samples,
    }
