"""MLP-Splatting render path on AMD MI355X (gfx950).

The HIP library libmsplat.so (built by ``paper_2606_03877_amd.build``) does all
the work; this package is its ctypes binding plus an autograd Function.
"""
from .render import (NetSpec, RenderOpts, Context, Renderer, MLPSplat, render,
                     msplat_render_forward, msplat_render_backward, msplat_get_stats,
                     msplat_debug_hits, msplat_workspace_size, msplat_num_params,
                     msplat_render_forward_f64, msplat_profile_enable, msplat_profile_read,
                     msplat_slot_forward, msplat_render_backward_slots, msplat_autotune)
from ._lib import load, MsplatError, LIB_PATH, EXPORTS

__all__ = ["NetSpec", "RenderOpts", "Context", "Renderer", "MLPSplat", "render",
           "msplat_render_forward", "msplat_render_backward", "msplat_get_stats",
           "msplat_debug_hits", "msplat_workspace_size", "msplat_num_params",
           "msplat_render_forward_f64", "msplat_profile_enable", "msplat_profile_read",
           "msplat_slot_forward", "msplat_render_backward_slots", "msplat_autotune", "load", "MsplatError", "LIB_PATH", "EXPORTS"]
