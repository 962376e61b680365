"""GPU parity on the 65,536-ray training batch (config 2: rays drawn at random
over 8 views, so the 64-ray packets are incoherent and every packet tests
every primitive), and of the float64 checker's forward, against the FP64
oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_cases import (gpu_render, gradient_mask, opts_of, oracle_model, oracle_opts, oracle_render, ray_nused,
                       scene, spec_of, view_rays)

pytestmark = pytest.mark.gpu

KEYS = ("center", "scale", "quat", "mlp")
TOL = {"fp32": 1e-5, "bf16x3": 2e-3}


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_batch_hit_lists_rgb_and_gradients(precision):
    """The whole batch in one call (as the benchmark launches it), checked on
    1024 seeded rays: exact-order hit lists bit-exact, RGB within the
    tolerance, and the gradient of those rays' pixels (upstream gradient on
    them only) against the oracle's."""
    ci = 2
    cfg = synth.CONFIGS[ci]
    sc = scene(ci)
    o, d, _ = synth.make_rays(cfg)
    opts = opts_of(cfg)
    g = gpu_render(ci, precision, sc, o, d, opts)
    idx = np.sort(np.random.default_rng(91).choice(len(o), 1024, replace=False))
    ref = oracle_render(ci, sc, o[idx], d[idx], opts, ray_ids=idx, margins=True, precision=precision)
    for n, i in enumerate(idx):
        np.testing.assert_array_equal(g["prim"][g["ray_off"][i]:g["ray_off"][i + 1]],
                                      ref["prim"][ref["ray_off"][n]:ref["ray_off"][n + 1]])
    nu = ray_nused(g)[idx]
    same = nu == ref["n_used"]
    err = float(np.abs(g["rgb"][idx] - ref["rgb"])[same].max())
    print(f"batch {precision}: {len(g['prim'])} hits, rgb max err {err:.3g} on {int(same.sum())} rays")
    assert err <= TOL[precision]
    keep = gradient_mask(nu, ref, precision, len(idx))
    rng = np.random.default_rng(2005)
    g_sub = (rng.standard_normal((len(idx), 3)) / len(idx)).astype(np.float32)
    g_sub[~keep] = 0.0
    g_rgb = np.zeros((len(o), 3), np.float32)
    g_rgb[idx] = g_sub
    t, to, td = g["dev"]
    out = g["renderer"].backward(g["ws"], t["center"], t["scale"], t["quat"], t["mlp"], to, td,
                                 torch.from_numpy(g_rgb).cuda())
    _, _, _, want, _ = oracle.loss_and_grads(sc, o[idx].astype(np.float64), d[idx].astype(np.float64),
                                             oracle_model(cfg), oracle_opts(opts, precision),
                                             grad_rgb=g_sub.astype(np.float64), ray_ids=idx)
    for k, v in zip(KEYS, out):
        rel = float(np.abs(v.cpu().numpy() - want[k]).max() / max(np.abs(want[k]).max(), 1e-30))
        print(f"  {k}: {rel:.2e}")
        assert rel <= TOL[precision], k


@pytest.mark.parametrize("ci,w,h", [(0, 40, 36), (1, 64, 50), (5, 40, 30)])
def test_f64_checker_matches_oracle(ci, w, h):
    """The float64 forward of the finite-difference checker against the
    oracle: the same render to float64 rounding."""
    from paper_2606_03877_amd import Renderer, msplat_render_forward_f64
    cfg = synth.CONFIGS[ci]
    sc = scene(ci)
    o, d = view_rays(ci, w, h)
    opts = opts_of(cfg)
    r = Renderer(spec_of(cfg, "fp32"), opts)
    dev = torch.device("cuda", 0)
    p64 = {k: torch.from_numpy(v.astype(np.float64)).to(dev) for k, v in sc.items()}
    o64 = torch.from_numpy(o.astype(np.float64)).to(dev)
    d64 = torch.from_numpy(d.astype(np.float64)).to(dev)
    R = len(o)
    cf = cfg.out_dim - 4
    rgb = torch.empty((R, 3), dtype=torch.float64, device=dev)
    tr = torch.empty((R,), dtype=torch.float64, device=dev)
    ft = torch.empty((R, cf), dtype=torch.float64, device=dev) if cf else None
    ws = torch.empty(4096, dtype=torch.uint8, device=dev)
    st, _ = msplat_render_forward_f64(r.ctx, r.spec, opts, p64["center"], p64["scale"], p64["quat"], p64["mlp"],
                                      o64, d64, rgb, tr, ft, ws)
    assert st == 0
    ref = oracle_render(ci, sc, o, d, opts)
    e_rgb = float(np.abs(rgb.cpu().numpy() - ref["rgb"]).max())
    e_tr = float(np.abs(tr.cpu().numpy() - ref["trans"]).max())
    print(f"config {ci}: float64 checker vs oracle: rgb {e_rgb:.3g}, trans {e_tr:.3g}")
    assert e_rgb <= 1e-12 and e_tr <= 1e-12
    if cf:
        assert float(np.abs(ft.cpu().numpy() - ref["feat"]).max()) <= 1e-12 * max(1.0, np.abs(ref["feat"]).max())
