"""Oracle gradients (test infrastructure only).

The analytic gradient of the oracle's forward is taken by reverse-mode
automatic differentiation of ``render`` in float64 (a library step standing in
for the adjoint the paper does not print); it is pinned independently by
complex-step differentiation (Squire and Trapp 1998), which needs no autograd,
and by central differences.  Discrete decisions (hit set, order, sample counts,
termination cut, ReLU gates) are held fixed, as in the HIP adjoint.
"""
from __future__ import annotations

import numpy as np
import torch

from .render import Model, Opts, render

__all__ = ["to_tensors", "loss_and_grads", "complex_step"]


def to_tensors(scene: dict, dtype=torch.float64, requires_grad=False) -> dict:
    out = {}
    for k in ("center", "scale", "quat", "mlp", "slots"):
        if k not in scene:
            continue
        t = torch.from_numpy(np.asarray(scene[k], dtype=np.float64)).to(dtype)
        if requires_grad:
            t.requires_grad_(True)
        out[k] = t
    return out


def loss_and_grads(scene: dict, ray_o, ray_d, model: Model, opts: Opts,
                   grad_rgb=None, grad_feat=None, target_rgb=None, chunk: int = 4096,
                   grad_trans=None, ray_ids=None, centre=None, grad_slot=None):
    """Vector-Jacobian product of the render with upstream gradients.

    Either ``grad_rgb`` ([R,3], optionally ``grad_feat``) is given, giving
    L = sum(grad_rgb * rgb) + sum(grad_feat * feat), or ``target_rgb`` is
    given, giving the mean-squared error L = mean((rgb - target)^2) over all
    R x 3 values.  Rays are processed in chunks and gradients accumulated.
    ``centre`` (per-ray virtual rays for tile order, as in ``render``) is
    sliced with the rays; by default chunks start on packet boundaries.  A
    scene with ``slots`` renders slot features; ``grad_slot`` [R, C] adds
    sum(grad_slot * slot_feat) to the loss.
    Returns (rgb, trans, feat, grads) with grads keyed like the scene.
    """
    prm = to_tensors(scene, requires_grad=True)
    o = torch.from_numpy(np.asarray(ray_o, np.float64))
    d = torch.from_numpy(np.asarray(ray_d, np.float64))
    nr = o.shape[0]
    rgbs, trs, fts = [], [], []
    loss_total = 0.0
    for s in range(0, nr, chunk):
        e = min(nr, s + chunk)
        out = render(prm["center"], prm["scale"], prm["quat"], prm["mlp"], o[s:e], d[s:e],
                     model, opts, ray_index_base=s,
                     ray_ids=None if ray_ids is None else ray_ids[s:e],
                     centre=None if centre is None else (centre[0][s:e], centre[1][s:e]),
                     slots=prm.get("slots"))
        if target_rgb is not None:
            tgt = torch.from_numpy(np.asarray(target_rgb[s:e], np.float64))
            loss = ((out["rgb"] - tgt) ** 2).sum() / (3.0 * nr)
        else:
            g = torch.from_numpy(np.asarray(grad_rgb[s:e], np.float64))
            loss = (out["rgb"] * g).sum()
            if grad_feat is not None and out["feat"].shape[1] > 0:
                gf = torch.from_numpy(np.asarray(grad_feat[s:e], np.float64))
                loss = loss + (out["feat"] * gf).sum()
            if grad_trans is not None:
                gt = torch.from_numpy(np.asarray(grad_trans[s:e], np.float64))
                loss = loss + (out["trans"] * gt).sum()
            if grad_slot is not None:
                gs = torch.from_numpy(np.asarray(grad_slot[s:e], np.float64))
                loss = loss + (out["slot_feat"] * gs).sum()
        if loss.requires_grad:
            loss.backward()
        loss_total += float(loss.detach())
        rgbs.append(out["rgb"].detach())
        trs.append(out["trans"].detach())
        fts.append(out["feat"].detach())
    grads = {k: (v.grad if v.grad is not None else torch.zeros_like(v)).numpy()
             for k, v in prm.items()}
    return (torch.cat(rgbs).numpy(), torch.cat(trs).numpy(), torch.cat(fts).numpy(),
            grads, loss_total)


def complex_step(scene: dict, ray_o, ray_d, model: Model, opts: Opts, key: str, index,
                 weights_rgb, weights_feat=None, h: float = 1e-30) -> float:
    """d/dx of L = sum(weights_rgb * rgb) (+ features) for the single
    parameter scene[key][index], by complex step: Im L(x + i h) / h."""
    prm = to_tensors(scene, dtype=torch.complex128)
    prm[key] = prm[key].clone()
    prm[key][index] += 1j * h
    o = torch.from_numpy(np.asarray(ray_o, np.float64))
    d = torch.from_numpy(np.asarray(ray_d, np.float64))
    out = render(prm["center"], prm["scale"], prm["quat"], prm["mlp"], o, d, model, opts)
    w = torch.from_numpy(np.asarray(weights_rgb, np.float64)).to(torch.complex128)
    loss = (out["rgb"] * w).sum()
    if weights_feat is not None and out["feat"].shape[1] > 0:
        wf = torch.from_numpy(np.asarray(weights_feat, np.float64)).to(torch.complex128)
        loss = loss + (out["feat"] * wf).sum()
    return float(loss.imag) / h
