"""Python binding of the msplat C ABI: argument marshalling only.

Every function named msplat_* forwards torch tensors (device memory and the
current stream) to the C entry point of the same name.  ``Renderer`` keeps a
context and grows the workspace when the library reports it too small;
``MLPSplat`` is the autograd Function over the forward and backward entry
points.  All arithmetic runs in the HIP kernels of libmsplat.so.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import MsplatError, load

__all__ = ["NetSpec", "RenderOpts", "Context", "Renderer", "MLPSplat", "render",
           "msplat_render_forward", "msplat_render_backward", "msplat_get_stats",
           "msplat_debug_hits", "msplat_workspace_size", "msplat_num_params",
           "msplat_render_forward_f64", "msplat_profile_enable", "msplat_profile_read",
           "msplat_slot_forward", "msplat_render_backward_slots", "msplat_autotune"]


@dataclasses.dataclass(frozen=True)
class NetSpec:
    num_prims: int
    pe_freqs: int
    hidden_width: int
    hidden_layers: int
    out_dim: int
    precision: str = "fp32"          # "fp32" | "bf16" | "bf16x3"
    primitive: str = "chord"         # "chord" (samples of the support's chord) | "contact" (the paper's
                                     # contact-point primitive: one interaction per hit)

    def c(self) -> _lib.Model:
        prec = {"fp32": _lib.MSPLAT_FP32, "bf16": _lib.MSPLAT_BF16,
                "bf16x3": _lib.MSPLAT_BF16X3}[self.precision]
        kind = {"chord": _lib.MSPLAT_CHORD, "contact": _lib.MSPLAT_CONTACT}[self.primitive]
        return _lib.Model(self.num_prims, self.pe_freqs, self.hidden_width, self.hidden_layers,
                          self.out_dim, prec, kind)


@dataclasses.dataclass(frozen=True)
class RenderOpts:
    samples_fixed: int = 32
    samples_min: int = 8
    samples_max: int = 128
    samples_per_unit: float = 128.0
    t_stop: float = 0.0
    jitter: int = 1
    jitter_seed: int = 0
    background: Sequence[float] = (0.0, 0.0, 0.0)
    order: int = 0   # 0: each ray's own contact depth; 1: tile order (packet virtual ray)
    hits_per_item: int = 0   # work-item size of the network kernels: 16, 32, 64; 0 = autotuned (64 untuned)
    items_per_group: int = 0   # work items per workgroup of the network kernels: 1, 2, 4, 8; 0 = autotuned (else a rule)
    # order 1: optional [ceil(R / 64), 6] float32 device tensor, per 64-ray packet the virtual ray (origin,
    # direction) its hits are ordered along (e.g. through its 8x8 tile's centre); None = mean origin and
    # normalised direction sum
    tile_rays: Optional[torch.Tensor] = None

    def c(self) -> _lib.Opts:
        bg = (ctypes.c_float * 3)(*[float(b) for b in self.background])
        return _lib.Opts(self.samples_fixed, self.samples_min, self.samples_max,
                         float(self.samples_per_unit), float(self.t_stop), self.jitter,
                         self.jitter_seed & 0xFFFFFFFF, bg, self.order, self.hits_per_item,
                         self.items_per_group, None if self.tile_rays is None else self.tile_rays.data_ptr())


def _p(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _check(t: torch.Tensor, name: str, shape, dtype=torch.float32):
    if t.dtype != dtype or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous {dtype} device tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")


class Context:
    """An msplat context bound to one HIP device."""

    def __init__(self, device: int = 0):
        self.lib = load()
        self.device = device
        h = ctypes.c_void_p()
        st = self.lib.msplat_create(device, ctypes.byref(h))
        if st != _lib.MSPLAT_OK:
            raise MsplatError(st, "msplat_create")
        self.handle = h

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                self.lib.msplat_destroy(self.handle)
                self.handle = None
        except Exception:
            pass


def msplat_num_params(spec: NetSpec) -> int:
    return int(load().msplat_num_params(ctypes.byref(spec.c())))


def msplat_workspace_size(spec: NetSpec, num_rays: int, max_hits: int) -> int:
    out = ctypes.c_uint64()
    st = load().msplat_workspace_size(ctypes.byref(spec.c()), num_rays, max_hits, ctypes.byref(out))
    if st != _lib.MSPLAT_OK:
        raise MsplatError(st, "msplat_workspace_size")
    return int(out.value)


def msplat_render_forward(ctx: Context, spec: NetSpec, opts: RenderOpts, center, scale, quat, mlp,
                          ray_o, ray_d, rgb, trans, feat, ws: torch.Tensor, stream=None):
    """Returns (status, need_bytes)."""
    need = ctypes.c_uint64(0)
    st = ctx.lib.msplat_render_forward(
        ctx.handle, ctypes.byref(spec.c()), ctypes.byref(opts.c()), _p(center), _p(scale), _p(quat),
        _p(mlp), _p(ray_o), _p(ray_d), int(ray_o.shape[0]), _p(rgb), _p(trans), _p(feat), _p(ws),
        ws.numel(), ctypes.byref(need), _stream(stream))
    return st, int(need.value)


def msplat_render_backward(ctx: Context, spec: NetSpec, opts: RenderOpts, center, scale, quat, mlp,
                           ray_o, ray_d, grad_rgb, grad_trans, grad_feat, ws, g_center, g_scale,
                           g_quat, g_mlp, stream=None) -> int:
    return ctx.lib.msplat_render_backward(
        ctx.handle, ctypes.byref(spec.c()), ctypes.byref(opts.c()), _p(center), _p(scale), _p(quat),
        _p(mlp), _p(ray_o), _p(ray_d), int(ray_o.shape[0]), _p(grad_rgb), _p(grad_trans),
        _p(grad_feat), _p(ws), ws.numel(), _p(g_center), _p(g_scale), _p(g_quat), _p(g_mlp),
        _stream(stream))


def msplat_get_stats(ctx: Context, ws: torch.Tensor, stream=None) -> dict:
    s = _lib.Stats()
    st = ctx.lib.msplat_get_stats(ctx.handle, _p(ws), ws.numel(), ctypes.byref(s), _stream(stream))
    if st != _lib.MSPLAT_OK:
        raise MsplatError(st, "msplat_get_stats")
    return {f: getattr(s, f) for f, _ in _lib.Stats._fields_}


def msplat_autotune(ctx: Context, spec: NetSpec, opts: RenderOpts, center, scale, quat, mlp, ray_o, ray_d,
                    rgb, trans, feat, grad_rgb, ws, g_center, g_scale, g_quat, g_mlp, stream=None):
    """Returns (status, chosen hits per work item, chosen backward work items per workgroup)."""
    chosen = ctypes.c_int32(0)
    chosen_group = ctypes.c_int32(0)
    st = ctx.lib.msplat_autotune(
        ctx.handle, ctypes.byref(spec.c()), ctypes.byref(opts.c()), _p(center), _p(scale), _p(quat), _p(mlp),
        _p(ray_o), _p(ray_d), int(ray_o.shape[0]), _p(rgb), _p(trans), _p(feat), _p(grad_rgb), _p(ws), ws.numel(),
        _p(g_center), _p(g_scale), _p(g_quat), _p(g_mlp), ctypes.byref(chosen), ctypes.byref(chosen_group),
        _stream(stream))
    return st, int(chosen.value), int(chosen_group.value)


def msplat_profile_enable(ctx: Context, enable: bool = True) -> None:
    st = ctx.lib.msplat_profile_enable(ctx.handle, 1 if enable else 0)
    if st != _lib.MSPLAT_OK:
        raise MsplatError(st, "msplat_profile_enable")


def msplat_profile_read(ctx: Context) -> dict:
    """{stage: (total_ms, launches)} of the event-timed launches so far."""
    n = ctypes.c_int(0)
    cap = 32
    names = (ctypes.c_char_p * cap)()
    tot = (ctypes.c_double * cap)()
    cnt = (ctypes.c_int64 * cap)()
    st = ctx.lib.msplat_profile_read(ctx.handle, cap, names, tot, cnt, ctypes.byref(n))
    if st != _lib.MSPLAT_OK:
        raise MsplatError(st, "msplat_profile_read")
    return {names[i].decode(): (tot[i], cnt[i]) for i in range(min(n.value, cap))}


def msplat_debug_hits(ctx: Context, ws: torch.Tensor, num_rays: int, num_hits: int, stream=None):
    """Depth-sorted hit lists on the host: (ray_off int64, prim int32, t_c f64, n_used int32)."""
    off = np.zeros(num_rays + 1, np.int64)
    prim = np.zeros(max(num_hits, 1), np.int32)
    tc = np.zeros(max(num_hits, 1), np.float64)
    nu = np.zeros(max(num_hits, 1), np.int32)
    st = ctx.lib.msplat_debug_hits(ctx.handle, _p(ws), ws.numel(), num_rays,
                                   off.ctypes.data_as(ctypes.c_void_p), prim.ctypes.data_as(ctypes.c_void_p),
                                   tc.ctypes.data_as(ctypes.c_void_p), nu.ctypes.data_as(ctypes.c_void_p),
                                   len(prim), _stream(stream))
    if st != _lib.MSPLAT_OK:
        raise MsplatError(st, "msplat_debug_hits")
    return off, prim[:num_hits], tc[:num_hits], nu[:num_hits]


def msplat_render_forward_f64(ctx: Context, spec: NetSpec, opts: RenderOpts, center, scale, quat, mlp,
                              ray_o, ray_d, rgb, trans, feat, ws, decisions=None, stream=None):
    need = ctypes.c_uint64(0)
    st = ctx.lib.msplat_render_forward_f64(
        ctx.handle, ctypes.byref(spec.c()), ctypes.byref(opts.c()), _p(center), _p(scale), _p(quat),
        _p(mlp), _p(ray_o), _p(ray_d), int(ray_o.shape[0]), _p(rgb), _p(trans), _p(feat),
        _p(decisions), _p(ws), ws.numel(), ctypes.byref(need), _stream(stream))
    return st, int(need.value)


def msplat_slot_forward(ctx: Context, spec: NetSpec, slots, out, ws: torch.Tensor, stream=None) -> int:
    return ctx.lib.msplat_slot_forward(ctx.handle, ctypes.byref(spec.c()), _p(slots), int(slots.shape[-1]),
                                       int(out.shape[0]), _p(out), _p(ws), ws.numel(), _stream(stream))


def msplat_render_backward_slots(ctx: Context, spec: NetSpec, opts: RenderOpts, center, scale, quat, mlp,
                                 ray_o, ray_d, grad_rgb, grad_trans, grad_feat, slots, grad_slot, ws,
                                 g_center, g_scale, g_quat, g_mlp, g_slots, stream=None) -> int:
    return ctx.lib.msplat_render_backward_slots(
        ctx.handle, ctypes.byref(spec.c()), ctypes.byref(opts.c()), _p(center), _p(scale), _p(quat),
        _p(mlp), _p(ray_o), _p(ray_d), int(ray_o.shape[0]), _p(grad_rgb), _p(grad_trans),
        _p(grad_feat), _p(slots), int(slots.shape[-1]), _p(grad_slot), _p(ws), ws.numel(), _p(g_center),
        _p(g_scale), _p(g_quat), _p(g_mlp), _p(g_slots), _stream(stream))


class Renderer:
    """Context + workspace management around the forward/backward entry points."""

    def __init__(self, spec: NetSpec, opts: RenderOpts, device: int = 0):
        self.spec = spec
        self.opts = opts
        self.device = torch.device("cuda", device)
        self.ctx = Context(device)
        self.n_params = msplat_num_params(spec)
        self._bytes_hint = {}

    def new_workspace(self, num_rays: int, hits: Optional[int] = None) -> torch.Tensor:
        h = hits if hits is not None else num_rays // 2 + 1024
        nbytes = max(msplat_workspace_size(self.spec, num_rays, h), self._bytes_hint.get(num_rays, 0))
        ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        assert ws.data_ptr() % 256 == 0
        return ws

    def check_inputs(self, center, scale, quat, mlp, ray_o, ray_d):
        P = self.spec.num_prims
        _check(center, "center", (P, 3))
        _check(scale, "scale", (P, 3))
        _check(quat, "quat", (P, 4))
        _check(mlp, "mlp", (P, self.n_params))
        R = ray_o.shape[0]
        _check(ray_o, "ray_o", (R, 3))
        _check(ray_d, "ray_d", (R, 3))
        if self.opts.tile_rays is not None:
            _check(self.opts.tile_rays, "tile_rays", ((R + 63) // 64, 6))

    def forward(self, center, scale, quat, mlp, ray_o, ray_d, ws: Optional[torch.Tensor] = None):
        """Returns (rgb [R,3], trans [R], feat [R,C] or None, workspace)."""
        self.check_inputs(center, scale, quat, mlp, ray_o, ray_d)
        R = ray_o.shape[0]
        cf = self.spec.out_dim - 4
        rgb = torch.empty((R, 3), dtype=torch.float32, device=self.device)
        trans = torch.empty((R,), dtype=torch.float32, device=self.device)
        feat = torch.empty((R, cf), dtype=torch.float32, device=self.device) if cf > 0 else None
        if ws is None:
            ws = self.new_workspace(R)
        for _ in range(4):
            st, need = msplat_render_forward(self.ctx, self.spec, self.opts, center, scale, quat, mlp,
                                             ray_o, ray_d, rgb, trans, feat, ws)
            if st == _lib.MSPLAT_OK:
                break
            if st != _lib.MSPLAT_E_CAPACITY:
                raise MsplatError(st, "msplat_render_forward")
            ws = torch.empty(int(need * 1.25) + 4096, dtype=torch.uint8, device=self.device)
        else:
            raise MsplatError(_lib.MSPLAT_E_CAPACITY, "msplat_render_forward")
        # remember the size this ray count needed, with slack for other views
        self._bytes_hint[R] = max(self._bytes_hint.get(R, 0), int(need * 1.1) + 4096)
        return rgb, trans, feat, ws

    def backward(self, ws, center, scale, quat, mlp, ray_o, ray_d, grad_rgb, grad_trans=None,
                 grad_feat=None):
        P = self.spec.num_prims
        g_center = torch.empty((P, 3), dtype=torch.float32, device=self.device)
        g_scale = torch.empty((P, 3), dtype=torch.float32, device=self.device)
        g_quat = torch.empty((P, 4), dtype=torch.float32, device=self.device)
        g_mlp = torch.empty((P, self.n_params), dtype=torch.float32, device=self.device)
        self.check_inputs(center, scale, quat, mlp, ray_o, ray_d)
        grad_rgb, grad_trans, grad_feat = self._upstream(ray_o.shape[0], grad_rgb, grad_trans, grad_feat)
        st = msplat_render_backward(self.ctx, self.spec, self.opts, center, scale, quat, mlp, ray_o,
                                    ray_d, grad_rgb, grad_trans, grad_feat, ws, g_center, g_scale,
                                    g_quat, g_mlp)
        if st != _lib.MSPLAT_OK:
            raise MsplatError(st, "msplat_render_backward")
        return g_center, g_scale, g_quat, g_mlp

    def _upstream(self, R: int, grad_rgb, grad_trans, grad_feat):
        """Upstream gradients as contiguous float32 tensors of the shapes the
        kernels index ([R,3], [R], [R, out_dim - 4])."""
        grad_rgb = grad_rgb.contiguous().float()
        _check(grad_rgb, "grad_rgb", (R, 3))
        if grad_trans is not None:
            grad_trans = grad_trans.contiguous().float()
            _check(grad_trans, "grad_trans", (R,))
        if grad_feat is not None:
            grad_feat = grad_feat.contiguous().float()
            _check(grad_feat, "grad_feat", (R, self.spec.out_dim - 4))
        return grad_rgb, grad_trans, grad_feat

    def slot_forward(self, ws, slots, num_rays: int):
        """Slot features [R, C] of the forward that last wrote ``ws``; slots [P, 4, C]."""
        if slots.dim() != 3:
            raise ValueError(f"slots: expected shape ({self.spec.num_prims}, 4, C), got {tuple(slots.shape)}")
        _check(slots, "slots", (self.spec.num_prims, 4, slots.shape[-1]))
        out = torch.empty((num_rays, slots.shape[-1]), dtype=torch.float32, device=self.device)
        st = msplat_slot_forward(self.ctx, self.spec, slots, out, ws)
        if st != _lib.MSPLAT_OK:
            raise MsplatError(st, "msplat_slot_forward")
        return out

    def backward_slots(self, ws, center, scale, quat, mlp, ray_o, ray_d, grad_rgb, slots, grad_slot,
                       grad_trans=None, grad_feat=None):
        """backward() of a loss that also depends on slot_forward()'s features;
        returns (g_center, g_scale, g_quat, g_mlp, g_slots)."""
        P = self.spec.num_prims
        R = ray_o.shape[0]
        self.check_inputs(center, scale, quat, mlp, ray_o, ray_d)
        if slots.dim() != 3:
            raise ValueError(f"slots: expected shape ({P}, 4, C), got {tuple(slots.shape)}")
        C = slots.shape[-1]
        slots = slots.contiguous().float()
        _check(slots, "slots", (P, 4, C))
        grad_slot = grad_slot.contiguous().float()
        _check(grad_slot, "grad_slot", (R, C))
        g = [torch.empty(sh, dtype=torch.float32, device=self.device)
             for sh in ((P, 3), (P, 3), (P, 4), (P, self.n_params), (P, 4, C))]
        grad_rgb, grad_trans, grad_feat = self._upstream(R, grad_rgb, grad_trans, grad_feat)
        st = msplat_render_backward_slots(self.ctx, self.spec, self.opts, center, scale, quat, mlp, ray_o,
                                          ray_d, grad_rgb, grad_trans, grad_feat, slots, grad_slot, ws, *g)
        if st != _lib.MSPLAT_OK:
            raise MsplatError(st, "msplat_render_backward_slots")
        return tuple(g)

    def autotune(self, center, scale, quat, mlp, ray_o, ray_d, grad_rgb=None) -> dict:
        """Time the work-item sizes on this workload (forward, and backward
        with ``grad_rgb``), then the work items per workgroup; later renders
        of it with hits_per_item = 0 (and items_per_group = 0) use the
        fastest.  Returns the choices: {"hits_per_item", "items_per_group"}."""
        self.check_inputs(center, scale, quat, mlp, ray_o, ray_d)
        R = ray_o.shape[0]
        P = self.spec.num_prims
        cf = self.spec.out_dim - 4
        rgb, trans, feat, ws = self.forward(center, scale, quat, mlp, ray_o, ray_d)
        g = [torch.empty(sh, dtype=torch.float32, device=self.device)
             for sh in ((P, 3), (P, 3), (P, 4), (P, self.n_params))]
        if grad_rgb is not None:
            grad_rgb = grad_rgb.contiguous().float()
            _check(grad_rgb, "grad_rgb", (R, 3))
        st, chosen, group = msplat_autotune(self.ctx, self.spec, self.opts, center, scale, quat, mlp, ray_o,
                                            ray_d, rgb, trans, feat, grad_rgb, ws, *g)
        if st != _lib.MSPLAT_OK:
            raise MsplatError(st, "msplat_autotune")
        return {"hits_per_item": chosen, "items_per_group": group}

    def stats(self, ws) -> dict:
        return msplat_get_stats(self.ctx, ws)

    def hits(self, ws, num_rays: int):
        st = self.stats(ws)
        return msplat_debug_hits(self.ctx, ws, num_rays, int(st["num_hits"]))


class MLPSplat(torch.autograd.Function):
    """Differentiable render: (center, scale, quat, mlp) -> (rgb, trans, feat)."""

    @staticmethod
    def forward(ctx, renderer: Renderer, center, scale, quat, mlp, ray_o, ray_d):
        rgb, trans, feat, ws = renderer.forward(center, scale, quat, mlp, ray_o, ray_d)
        ctx.renderer = renderer
        ctx.ws = ws
        ctx.has_feat = feat is not None
        ctx.save_for_backward(center, scale, quat, mlp, ray_o, ray_d)
        if feat is None:
            feat = torch.zeros((ray_o.shape[0], 0), dtype=torch.float32, device=ray_o.device)
        return rgb, trans, feat

    @staticmethod
    def backward(ctx, g_rgb, g_trans, g_feat):
        center, scale, quat, mlp, ray_o, ray_d = ctx.saved_tensors
        if g_rgb is None:
            g_rgb = torch.zeros((ray_o.shape[0], 3), dtype=torch.float32, device=ray_o.device)
        gf = g_feat if (ctx.has_feat and g_feat is not None) else None
        gc, gs, gq, gm = ctx.renderer.backward(ctx.ws, center, scale, quat, mlp, ray_o, ray_d,
                                               g_rgb, g_trans, gf)
        return None, gc, gs, gq, gm, None, None


def render(renderer: Renderer, center, scale, quat, mlp, ray_o, ray_d):
    """(rgb, trans, feat) with autograd support for the primitive parameters."""
    return MLPSplat.apply(renderer, center, scale, quat, mlp, ray_o, ray_d)
