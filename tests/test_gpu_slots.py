"""GPU parity of slot features (four slot embeddings per primitive, gated by
a softmax over a tetrahedral frame of the hit's local offset and composited
with the hit's weight) against the FP64 oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_cases import (MASK_MAX, RELU_AMBIGUOUS, gpu_render, opts_of, oracle_model, oracle_opts, ray_nused, scene,
                       view_rays)

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "bf16x3": 2e-3}


def _slots(ci, C, seed=0):
    P = synth.CONFIGS[ci].num_prims
    return np.random.default_rng(500 + 10 * ci + seed).standard_normal((P, 4, C)).astype(np.float32)


def _oracle(ci, sc, o, d, opts, slots, chunk=4096, precision=None):
    cfg = synth.CONFIGS[ci]
    p = oracle.to_tensors(sc)
    st = torch.from_numpy(slots.astype(np.float64))
    outs, nus = [], []
    for s in range(0, len(o), chunk):
        e = min(len(o), s + chunk)
        r = oracle.render(p["center"], p["scale"], p["quat"], p["mlp"], torch.from_numpy(o[s:e].astype(np.float64)),
                          torch.from_numpy(d[s:e].astype(np.float64)), oracle_model(cfg),
                          oracle_opts(opts, precision), ray_index_base=s, slots=st, keep_samples=True)
        outs.append(r["slot_feat"].numpy())
        m = np.full(e - s, np.inf)
        if r["samples"] is not None:
            np.minimum.at(m, r["samples"]["ray"], r["samples"]["relu_margin"])
        nus.append((r["n_used"], m))
    return (np.concatenate(outs), np.concatenate([a for a, _ in nus]), np.concatenate([b for _, b in nus]))


@pytest.mark.parametrize("ci,w,h", [(0, 64, 64), (1, 100, 75), (4, 90, 70)])
@pytest.mark.parametrize("C", [512, 36, 1040])
@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_slot_forward_matches_oracle(ci, w, h, C, precision):
    sc = scene(ci)
    o, d = view_rays(ci, w, h)
    opts = opts_of(synth.CONFIGS[ci])
    slots = _slots(ci, C)
    g = gpu_render(ci, precision, sc, o, d, opts)
    F = g["renderer"].slot_forward(g["ws"], torch.from_numpy(slots).cuda(), len(o)).cpu().numpy()
    ref, n_used, _ = _oracle(ci, sc, o, d, opts, slots)
    same = ray_nused(g) == n_used
    # the features are bounded by max |e| times the ray's opacity
    err = float(np.abs(F - ref)[same].max())
    scale = float(np.abs(slots).max())
    print(f"config {ci} {w}x{h} C={C} {precision}: max err {err:.3g} (max |e| {scale:.3g}), "
          f"rays with another cut {int((~same).sum())}")
    assert err <= TOL[precision] * scale
    assert np.abs(F[~same] - ref[~same]).max(initial=0.0) <= (opts.t_stop + TOL[precision]) * scale


# slot widths 64 (one 256-channel chunk), 516 (four, the last ragged) and
# 1040 (beyond the register-resident row: streamed per hit, two passes)
@pytest.mark.parametrize("ci,w,h,precision,C", [
    (1, 64, 50, "fp32", 64), (4, 44, 40, "fp32", 64), (1, 64, 50, "bf16x3", 64), (4, 44, 40, "bf16x3", 64),
    (1, 48, 40, "fp32", 516), (0, 40, 40, "fp32", 1040)])
def test_slot_backward_matches_oracle(ci, w, h, precision, C):
    tol = TOL[precision]
    cfg = synth.CONFIGS[ci]
    sc = scene(ci)
    o, d = view_rays(ci, w, h)
    opts = opts_of(cfg)
    slots = _slots(ci, C, seed=1)
    R = len(o)
    rng = np.random.default_rng(1000 * ci + 9)
    g_rgb = (rng.standard_normal((R, 3)) / R).astype(np.float32)
    g_slot = (rng.standard_normal((R, C)) / R).astype(np.float32)
    g = gpu_render(ci, precision, sc, o, d, opts)
    _, n_used, margin = _oracle(ci, sc, o, d, opts, slots, precision=precision)
    keep = (ray_nused(g) == n_used) & (margin >= RELU_AMBIGUOUS[precision])
    print(f"rays left out: {R - int(keep.sum())} of {R}")
    assert R - keep.sum() <= MASK_MAX * R
    g_rgb[~keep] = 0.0
    g_slot[~keep] = 0.0
    scs = dict(sc)
    scs["slots"] = slots
    _, _, _, ref, _ = oracle.loss_and_grads(scs, o.astype(np.float64), d.astype(np.float64), oracle_model(cfg),
                                            oracle_opts(opts, precision), grad_rgb=g_rgb, grad_slot=g_slot)
    t, to, td = g["dev"]
    got = g["renderer"].backward_slots(g["ws"], t["center"], t["scale"], t["quat"], t["mlp"], to, td,
                                       torch.from_numpy(g_rgb).cuda(), torch.from_numpy(slots).cuda(),
                                       torch.from_numpy(g_slot).cuda())
    for k, v in zip(("center", "scale", "quat", "mlp", "slots"), got):
        v = v.cpu().numpy()
        rel = float(np.abs(v - ref[k]).max() / max(np.abs(ref[k]).max(), 1e-30))
        print(f"config {ci} {precision} {k}: rel err {rel:.3g}")
        assert rel <= tol, k
    # without slot gradients the entry point gives the plain backward's results
    zero = torch.zeros((R, C), device="cuda")
    a = g["renderer"].backward_slots(g["ws"], t["center"], t["scale"], t["quat"], t["mlp"], to, td,
                                     torch.from_numpy(g_rgb).cuda(), torch.from_numpy(slots).cuda(), zero)
    b = g["renderer"].backward(g["ws"], t["center"], t["scale"], t["quat"], t["mlp"], to, td,
                               torch.from_numpy(g_rgb).cuda())
    for x, y in zip(a[:4], b):
        np.testing.assert_allclose(x.cpu().numpy(), y.cpu().numpy(), rtol=1e-5,
                                   atol=1e-6 * float(y.abs().max()) + 1e-30)
    assert float(a[4].abs().max()) == 0.0


def test_slot_arguments_are_validated():
    from paper_2606_03877_amd import msplat_slot_forward, _lib
    ci = 0
    sc = scene(ci)
    o, d = view_rays(ci, 16, 8)
    g = gpu_render(ci, "fp32", sc, o, d, opts_of(synth.CONFIGS[ci]))
    r = g["renderer"]
    bad = torch.zeros((synth.CONFIGS[ci].num_prims, 4, 6), device="cuda")   # C not a multiple of 4
    out = torch.empty((len(o), 6), device="cuda")
    assert msplat_slot_forward(r.ctx, r.spec, bad, out, g["ws"]) == _lib.MSPLAT_E_INVALID
    fresh = torch.zeros_like(g["ws"])   # no forward has filled it
    good = torch.zeros((synth.CONFIGS[ci].num_prims, 4, 8), device="cuda")
    out8 = torch.empty((len(o), 8), device="cuda")
    assert msplat_slot_forward(r.ctx, r.spec, good, out8, fresh) == _lib.MSPLAT_E_STATE


def test_calls_on_an_earlier_workspace_check_its_layout():
    """A workspace that is not the context's last one is read through the
    identity its forward recorded: the same ray count works, another is
    refused (the layout would differ)."""
    from paper_2606_03877_amd import msplat_slot_forward, _lib
    ci = 0
    cfg = synth.CONFIGS[ci]
    sc = scene(ci)
    o, d = view_rays(ci, 32, 16)
    g = gpu_render(ci, "fp32", sc, o, d, opts_of(cfg))
    r = g["renderer"]
    t, to, td = g["dev"]
    ws1 = g["ws"]
    # another forward on a second workspace becomes the context's last one
    r.forward(t["center"], t["scale"], t["quat"], t["mlp"], to[:64], td[:64])
    slots = torch.zeros((cfg.num_prims, 4, 8), device="cuda")
    out = torch.empty((len(o), 8), device="cuda")
    assert msplat_slot_forward(r.ctx, r.spec, slots, out, ws1) == _lib.MSPLAT_OK
    more = torch.empty((len(o) + 64, 8), device="cuda")
    assert msplat_slot_forward(r.ctx, r.spec, slots, more, ws1) == _lib.MSPLAT_E_STATE


@pytest.mark.parametrize("fast_path", [True, False])
def test_another_precision_on_the_same_workspace_is_refused(fast_path):
    """The packed operands (whose size depends on the precision) precede the
    hit arrays, so a backward or slot call with another precision than the
    forward's would read the hits at other offsets: refused with
    MSPLAT_E_STATE before any launch, both when the workspace is the
    context's last one and when its recorded identity is read."""
    from paper_2606_03877_amd import (NetSpec, msplat_render_backward, msplat_slot_forward, _lib)
    ci = 0
    cfg = synth.CONFIGS[ci]
    sc = scene(ci)
    o, d = view_rays(ci, 32, 16)
    g = gpu_render(ci, "fp32", sc, o, d, opts_of(cfg))
    r = g["renderer"]
    t, to, td = g["dev"]
    ws1 = g["ws"]
    if not fast_path:
        r.forward(t["center"], t["scale"], t["quat"], t["mlp"], to[:64], td[:64])
    other = NetSpec(cfg.num_prims, cfg.pe_freqs, cfg.hidden_width, cfg.hidden_layers, cfg.out_dim, "bf16x3")
    P, R = cfg.num_prims, len(o)
    gr = torch.zeros((R, 3), device="cuda")
    outs = [torch.full(sh, 7.0, device="cuda") for sh in ((P, 3), (P, 3), (P, 4), (P, r.n_params))]
    st = msplat_render_backward(r.ctx, other, r.opts, t["center"], t["scale"], t["quat"], t["mlp"], to, td,
                                gr, None, None, ws1, *outs)
    assert st == _lib.MSPLAT_E_STATE
    torch.cuda.synchronize()
    assert all(bool((x == 7.0).all()) for x in outs)   # nothing was launched
    slots = torch.zeros((P, 4, 8), device="cuda")
    out = torch.empty((R, 8), device="cuda")
    assert msplat_slot_forward(r.ctx, other, slots, out, ws1) == _lib.MSPLAT_E_STATE
    # the forward's own precision is still accepted
    assert msplat_slot_forward(r.ctx, r.spec, slots, out, ws1) == _lib.MSPLAT_OK


def test_backward_checks_upstream_gradient_shapes():
    ci = 0
    cfg = synth.CONFIGS[ci]
    sc = scene(ci)
    o, d = view_rays(ci, 16, 8)
    g = gpu_render(ci, "fp32", sc, o, d, opts_of(cfg))
    r = g["renderer"]
    t, to, td = g["dev"]
    R = len(o)
    with pytest.raises(ValueError):
        r.backward(g["ws"], t["center"], t["scale"], t["quat"], t["mlp"], to, td, torch.zeros((R - 1, 3),
                                                                                               device="cuda"))
    slots = torch.zeros((cfg.num_prims, 4, 8), device="cuda")
    with pytest.raises(ValueError):
        r.backward_slots(g["ws"], t["center"], t["scale"], t["quat"], t["mlp"], to, td,
                         torch.zeros((R, 3), device="cuda"), slots, torch.zeros((R, 4), device="cuda"))
    with pytest.raises(ValueError):
        r.backward_slots(g["ws"], t["center"], t["scale"], t["quat"], t["mlp"], to, td,
                         torch.zeros((R, 3), device="cuda"), slots[:, 0], torch.zeros((R, 8), device="cuda"))
