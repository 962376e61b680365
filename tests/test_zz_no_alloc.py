"""msplat_render_forward_noalloc (the forward into the library's own device
scratch array, for callers that cannot allocate) against
msplat_render_forward into a caller workspace, through the C ABI: two calls
in a row, the second with fewer rays, and a workload beyond the array."""
import ctypes

import numpy as np
import pytest
import torch

import synth
from gpu_cases import opts_of, scene, spec_of, to_dev, view_rays

pytestmark = pytest.mark.gpu


def _noalloc(ctx, spec, opts, t, to, td, R, cf):
    rgb = torch.full((R, 3), 9.0, device="cuda")
    trans = torch.full((R,), 9.0, device="cuda")
    feat = torch.full((R, cf), 9.0, device="cuda") if cf else None
    need = ctypes.c_uint64(0)
    p = lambda x: None if x is None else ctypes.c_void_p(x.data_ptr())
    st = ctx.lib.msplat_render_forward_noalloc(
        ctx.handle, ctypes.byref(spec.c()), ctypes.byref(opts.c()), p(t["center"]), p(t["scale"]), p(t["quat"]),
        p(t["mlp"]), p(to), p(td), R, p(rgb), p(trans), p(feat), ctypes.byref(need),
        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    return st, int(need.value), rgb, trans, feat


@pytest.mark.parametrize("ci,precision", [(1, "bf16x3"), (5, "fp32")])
def test_noalloc_forward_matches_workspace_forward(ci, precision):
    from paper_2606_03877_amd import Renderer, _lib
    cfg = synth.CONFIGS[ci]
    sc = scene(ci)
    opts = opts_of(cfg)
    r = Renderer(spec_of(cfg, precision), opts)
    cf = cfg.out_dim - 4
    for w, h in ((160, 120), (48, 40)):      # the second call is smaller
        o, d = view_rays(ci, w, h)
        R = len(o)
        t, to, td = to_dev(sc, o, d)
        st, need, rgb, trans, feat = _noalloc(r.ctx, r.spec, opts, t, to, td, R, cf)
        assert st == _lib.MSPLAT_OK, st
        assert 0 < need <= (256 << 20)
        ref_rgb, ref_tr, ref_ft, _ = r.forward(t["center"], t["scale"], t["quat"], t["mlp"], to, td)
        torch.cuda.synchronize()
        tol = 1e-5 if precision == "fp32" else 2e-3
        assert float((rgb - ref_rgb).abs().max()) <= tol
        assert float((trans - ref_tr).abs().max()) <= tol
        if cf:
            assert float((feat - ref_ft).abs().max()) <= 4 * tol * max(1.0, float(ref_ft.abs().max()))
        print(f"config {ci} {w}x{h}: {R} rays, rgb max diff {float((rgb - ref_rgb).abs().max()):.3g}")


def test_noalloc_refuses_a_workload_beyond_its_array():
    from paper_2606_03877_amd import Renderer, _lib
    ci = 4
    cfg = synth.CONFIGS[ci]
    sc = scene(ci)
    o, d, _ = synth.make_rays(cfg)
    r = Renderer(spec_of(cfg, "bf16x3"), opts_of(cfg))
    t, to, td = to_dev(sc, o, d)
    st, need, rgb, _, _ = _noalloc(r.ctx, r.spec, r.opts, t, to, td, len(o), 0)
    assert st == _lib.MSPLAT_E_CAPACITY
    assert need > (256 << 20)
    assert float(rgb[:1000].min()) == 9.0      # outputs untouched
