"""The work-item autotuner: every work-item size the network kernels can run
with (16, 32, 64 hits of one primitive) and every number of work items a
workgroup of the forward and backward network kernels takes (1, 2, 4, 8: a
run of up to 512 hits of one primitive, dealt to the waves at once) renders
and differentiates within the tolerances of the FP64 oracle, and the tuner's
choices are recorded and used."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_cases import (gpu_render, gradient_mask, opts_of, oracle_model, oracle_opts, oracle_render, ray_nused,
                       scene, view_rays)

pytestmark = pytest.mark.gpu

KEYS = ("center", "scale", "quat", "mlp")
TOL = {"fp32": 1e-5, "bf16x3": 2e-3}


# (hits per item, items per workgroup) per case: every size of each knob, on
# each network width and precision; 16 x 8 puts two or more primitives'
# hits in most workgroups, and 64 x 4 in FP32 (two waves) is cut to the
# 128 hits its workgroup holds
CASES = [(1, 64, 50, "bf16x3", 16, 8), (1, 64, 50, "bf16x3", 64, 1), (4, 44, 40, "bf16x3", 32, 2),
         (4, 44, 40, "bf16x3", 64, 8), (4, 44, 40, "fp32", 16, 1), (4, 44, 40, "fp32", 64, 4),
         (3, 40, 30, "bf16x3", 16, 8), (3, 40, 30, "bf16x3", 32, 4)]


@pytest.mark.parametrize("ci,w,h,precision,hpi,group", CASES)
def test_every_work_item_size_matches_oracle(ci, w, h, precision, hpi, group):
    cfg = synth.CONFIGS[ci]
    sc = scene(ci)
    o, d = view_rays(ci, w, h)
    opts = dataclasses.replace(opts_of(cfg), hits_per_item=hpi, items_per_group=group)
    R = len(o)
    g = gpu_render(ci, precision, sc, o, d, opts)
    assert g["stats"]["hits_per_item"] == hpi
    ref_fwd = oracle_render(ci, sc, o, d, opts, margins=True, precision=precision)
    same = ray_nused(g) == ref_fwd["n_used"]
    err = float(np.abs(g["rgb"] - ref_fwd["rgb"])[same].max())
    assert err <= TOL[precision]
    keep = gradient_mask(ray_nused(g), ref_fwd, precision, R)
    g_rgb = (np.random.default_rng(1000 * ci + 7).standard_normal((R, 3)) / R).astype(np.float32)
    g_rgb[~keep] = 0.0
    cf = cfg.out_dim - 4
    g_ft = None
    if cf > 0:
        g_ft = (np.random.default_rng(1000 * ci + 8).standard_normal((R, cf)) / R).astype(np.float32)
        g_ft[~keep] = 0.0
    _, _, _, ref, _ = oracle.loss_and_grads(sc, o.astype(np.float64), d.astype(np.float64), oracle_model(cfg),
                                            oracle_opts(opts, precision), grad_rgb=g_rgb, grad_feat=g_ft)
    t, to, td = g["dev"]
    out = g["renderer"].backward(g["ws"], t["center"], t["scale"], t["quat"], t["mlp"], to, td,
                                 torch.from_numpy(g_rgb).cuda(), None,
                                 None if g_ft is None else torch.from_numpy(g_ft).cuda())
    assert g["stats"]["items_per_group"] == group
    for k, v in zip(KEYS, out):
        rel = float(np.abs(v.cpu().numpy() - ref[k]).max() / max(np.abs(ref[k]).max(), 1e-30))
        print(f"config {ci} {precision} {hpi} hits per item, {group} per group {k}: {rel:.2e}")
        assert rel <= TOL[precision], k


def test_autotune_records_and_uses_its_choice():
    from paper_2606_03877_amd import NetSpec, RenderOpts, Renderer
    ci = 1
    cfg = synth.CONFIGS[ci]
    sc = scene(ci)
    o, d = view_rays(ci, 200, 160)
    opts = opts_of(cfg)
    assert opts.hits_per_item == 0
    g = gpu_render(ci, "bf16x3", sc, o, d, opts)
    r = g["renderer"]
    assert g["stats"]["hits_per_item"] == 64        # untuned default
    t, to, td = g["dev"]
    grad = torch.full((len(o), 3), 1.0 / len(o), device="cuda")
    chosen = r.autotune(t["center"], t["scale"], t["quat"], t["mlp"], to, td, grad)
    assert chosen["hits_per_item"] in (16, 32, 64)
    assert chosen["items_per_group"] in (1, 2, 4, 8)
    _, _, _, ws = r.forward(t["center"], t["scale"], t["quat"], t["mlp"], to, td)
    assert r.stats(ws)["hits_per_item"] == chosen["hits_per_item"]
    assert r.stats(ws)["items_per_group"] == chosen["items_per_group"]
    # another workload (ray count) is not covered by the choice
    _, _, _, ws2 = r.forward(t["center"], t["scale"], t["quat"], t["mlp"], to[:640], td[:640])
    assert r.stats(ws2)["hits_per_item"] == 64
    # an explicit size wins
    r2 = Renderer(r.spec, dataclasses.replace(opts, hits_per_item=16, items_per_group=2))
    _, _, _, ws3 = r2.forward(t["center"], t["scale"], t["quat"], t["mlp"], to, td)
    assert r2.stats(ws3)["hits_per_item"] == 16
    assert r2.stats(ws3)["items_per_group"] == 2


@pytest.mark.parametrize("field,value", [("hits_per_item", 48), ("items_per_group", 3),
                                         ("items_per_group", 16)])
def test_work_item_options_are_validated(field, value):
    from paper_2606_03877_amd import Renderer, msplat_render_forward, _lib
    from gpu_cases import spec_of, to_dev
    ci = 0
    cfg = synth.CONFIGS[ci]
    sc = scene(ci)
    o, d = view_rays(ci, 16, 8)
    r = Renderer(spec_of(cfg, "fp32"), dataclasses.replace(opts_of(cfg), **{field: value}))
    t, to, td = to_dev(sc, o, d)
    ws = r.new_workspace(len(o))
    rgb = torch.empty((len(o), 3), device="cuda")
    trans = torch.empty((len(o),), device="cuda")
    st, _ = msplat_render_forward(r.ctx, r.spec, r.opts, t["center"], t["scale"], t["quat"], t["mlp"], to, td,
                                  rgb, trans, None, ws)
    assert st == _lib.MSPLAT_E_INVALID


@pytest.mark.parametrize("ci,w,h", [(1, 800, 800), (2, 0, 0)])
def test_untuned_items_per_group_rule(ci, w, h):
    """Without a recorded choice a workgroup takes the most work items (up to
    8) that leave at least 2048 workgroups."""
    cfg = synth.CONFIGS[ci]
    sc = scene(ci)
    if cfg.batch_rays:
        o, d, _ = synth.make_rays(cfg)
    else:
        o, d = view_rays(ci, w, h)
    g = gpu_render(ci, "bf16x3", sc, o, d, opts_of(cfg))
    st = g["stats"]
    items = int(st["num_work_items"])
    want = 1
    while want < 8 and items >= 2048 * 2 * want:
        want *= 2
    print(f"config {ci}: {items} work items, {st['items_per_group']} per workgroup")
    assert st["items_per_group"] == want
