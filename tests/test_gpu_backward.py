"""GPU parity of the backward pass (through the C ABI and the autograd
Function) against the oracle's analytic gradient."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_cases import (gpu_render, gradient_mask, opts_of, oracle_model, oracle_opts, oracle_render,
                       ray_nused, scene, spec_of, to_dev, view_rays)

pytestmark = pytest.mark.gpu

CASES = [(0, 40, 36), (1, 64, 50), (4, 44, 40), (3, 40, 30), (5, 48, 40)]
KEYS = ("center", "scale", "quat", "mlp")


def _grads(ci, precision, w, h, with_trans=False, t_stop=None):
    cfg = synth.CONFIGS[ci]
    sc = scene(ci)
    o, d = view_rays(ci, w, h)
    opts = opts_of(cfg, t_stop=t_stop)
    R = len(o)
    rng = np.random.default_rng(1000 * ci + 4)
    g_rgb = (rng.standard_normal((R, 3)) / R).astype(np.float32)
    g_tr = (rng.standard_normal(R) / R).astype(np.float32) if with_trans else None
    cf = cfg.out_dim - 4
    g_ft = (rng.standard_normal((R, cf)) / R).astype(np.float32) if cf > 0 else None
    g = gpu_render(ci, precision, sc, o, d, opts)
    # a termination cut on a neighbouring sample (threshold crossing within
    # rounding) and a ReLU gate within rounding of its switching point (in the
    # form's own arithmetic) are discrete decisions either side may take the
    # other way: such rays carry no upstream gradient on either side
    ref_fwd = oracle_render(ci, sc, o, d, opts, margins=True, precision=precision)
    keep = gradient_mask(ray_nused(g), ref_fwd, precision, R)
    g_rgb[~keep] = 0.0
    if g_tr is not None:
        g_tr[~keep] = 0.0
    if g_ft is not None:
        g_ft[~keep] = 0.0
    _, _, _, ref, _ = oracle.loss_and_grads(sc, o.astype(np.float64), d.astype(np.float64),
                                            oracle_model(cfg), oracle_opts(opts, precision), grad_rgb=g_rgb,
                                            grad_trans=g_tr, grad_feat=g_ft)
    t, to, td = g["dev"]
    gt = None if g_tr is None else torch.from_numpy(g_tr).cuda()
    gf = None if g_ft is None else torch.from_numpy(g_ft).cuda()
    gc, gs, gq, gm = g["renderer"].backward(g["ws"], t["center"], t["scale"], t["quat"], t["mlp"], to, td,
                                            torch.from_numpy(g_rgb).cuda(), gt, gf)
    got = {"center": gc.cpu().numpy(), "scale": gs.cpu().numpy(), "quat": gq.cpu().numpy(),
           "mlp": gm.cpu().numpy()}
    return got, ref, sc


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))


@pytest.mark.parametrize("ci,w,h", CASES)
@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("bf16x3", 2e-3)])
def test_gradients_match_oracle(ci, w, h, precision, tol):
    got, ref, sc = _grads(ci, precision, w, h)
    errs = {k: _rel(got[k], ref[k]) for k in KEYS}
    print(f"config {ci} {precision} rel errors {errs}")
    for k in KEYS:
        assert errs[k] <= tol, (k, errs[k])


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("bf16x3", 2e-3)])
def test_gradients_match_oracle_without_cut(precision, tol):
    ci = 4
    got, ref, sc = _grads(ci, precision, 40, 36, t_stop=0.0)
    errs = {k: _rel(got[k], ref[k]) for k in KEYS}
    print(f"config {ci} {precision} rel errors {errs}")
    for k in KEYS:
        assert errs[k] <= tol, (k, errs[k])


def test_transmittance_gradient_and_quaternion_orthogonality():
    got, ref, sc = _grads(1, "fp32", 48, 40, with_trans=True)
    for k in KEYS:
        assert _rel(got[k], ref[k]) <= 1e-5, k
    dots = np.abs((got["quat"] * sc["quat"]).sum(1))
    assert dots.max() <= 1e-5 * np.abs(got["quat"]).max()


def test_autograd_function_mse_matches_direct_backward():
    from paper_2606_03877_amd import Renderer, render
    ci = 1
    cfg = synth.CONFIGS[ci]
    sc = scene(ci)
    o, d = view_rays(ci, 48, 40)
    R = len(o)
    opts = opts_of(cfg)
    r = Renderer(spec_of(cfg, "fp32"), opts)
    t, to, td = to_dev(sc, o, d)
    target = torch.rand((R, 3), device="cuda", generator=torch.Generator("cuda").manual_seed(5))
    # rays whose cut or ReLU gates are decided within rounding are masked out of the loss
    _, _, _, ws = r.forward(t["center"], t["scale"], t["quat"], t["mlp"], to, td)
    off, _, _, nused = r.hits(ws, R)
    ref_fwd = oracle_render(ci, sc, o, d, opts, margins=True, precision="fp32")
    keep = gradient_mask(ray_nused({"ray_off": off, "hit_nused": nused}), ref_fwd, "fp32", R)
    mask = torch.from_numpy(keep.astype(np.float32)).cuda()[:, None]
    params = {k: t[k].clone().requires_grad_(True) for k in KEYS}
    rgb, trans, feat = render(r, params["center"], params["scale"], params["quat"], params["mlp"], to, td)
    loss = (((rgb - target) ** 2) * mask).sum() / (3 * R)
    loss.backward()
    g_rgb = (2.0 / (3 * R)) * (rgb.detach() - target) * mask
    _, _, _, ws = r.forward(t["center"], t["scale"], t["quat"], t["mlp"], to, td)
    direct = r.backward(ws, t["center"], t["scale"], t["quat"], t["mlp"], to, td, g_rgb)
    for k, dv in zip(KEYS, direct):
        np.testing.assert_allclose(params[k].grad.cpu().numpy(), dv.cpu().numpy(), rtol=1e-4,
                                   atol=1e-6 * float(dv.abs().max()))
    # and against the oracle's gradient of the same masked mean-squared error
    tg = target.cpu().numpy().astype(np.float64)
    g_ref = (2.0 / (3 * R)) * (ref_fwd["rgb"] - tg) * keep[:, None]
    _, _, _, ref, _ = oracle.loss_and_grads(sc, o.astype(np.float64), d.astype(np.float64),
                                            oracle_model(cfg), oracle_opts(opts), grad_rgb=g_ref)
    for k in KEYS:
        assert _rel(params[k].grad.cpu().numpy(), ref[k]) <= 1e-5, k


@pytest.mark.parametrize("ci,precision", [(1, "fp32"), (1, "bf16x3"), (3, "bf16x3"), (4, "fp32"),
                                          (4, "bf16x3")])
def test_full_size_gradient_of_sampled_rays(ci, precision):
    """Full-size backward (all hits and work items of the benchmark's launch)
    with upstream gradient on 256 seeded rays only: the result is the gradient
    of those rays' pixels, which the oracle computes on the subset."""
    tol = {"fp32": 1e-5, "bf16x3": 2e-3}[precision]
    cfg = synth.CONFIGS[ci]
    sc = scene(ci)
    o, d, _ = synth.make_rays(cfg)
    opts = opts_of(cfg)
    g = gpu_render(ci, precision, sc, o, d, opts)
    idx = np.sort(np.random.default_rng(78).choice(len(o), 256, replace=False))
    ref_fwd = oracle_render(ci, sc, o[idx], d[idx], opts, ray_ids=idx, margins=True, precision=precision)
    keep = gradient_mask(ray_nused(g)[idx], ref_fwd, precision, len(idx))
    # hit lists of the sampled rays, bit-exact
    for n, i in enumerate(idx):
        np.testing.assert_array_equal(g["prim"][g["ray_off"][i]:g["ray_off"][i + 1]],
                                      ref_fwd["prim"][ref_fwd["ray_off"][n]:ref_fwd["ray_off"][n + 1]])
    rng = np.random.default_rng(1000 * ci + 5)
    g_sub = rng.standard_normal((len(idx), 3)) / len(idx)
    g_sub[~keep] = 0.0
    cf = cfg.out_dim - 4
    f_sub = rng.standard_normal((len(idx), cf)) / len(idx) if cf > 0 else None
    if f_sub is not None:
        f_sub[~keep] = 0.0
    g_rgb = np.zeros((len(o), 3), np.float32)
    g_rgb[idx] = g_sub
    g_ft = None
    if f_sub is not None:
        g_ft = np.zeros((len(o), cf), np.float32)
        g_ft[idx] = f_sub
    t, to, td = g["dev"]
    out = g["renderer"].backward(g["ws"], t["center"], t["scale"], t["quat"], t["mlp"], to, td,
                                 torch.from_numpy(g_rgb).cuda(), None,
                                 None if g_ft is None else torch.from_numpy(g_ft).cuda())
    got = dict(zip(KEYS, [x.cpu().numpy() for x in out]))
    _, _, _, ref, _ = oracle.loss_and_grads(sc, o[idx].astype(np.float64), d[idx].astype(np.float64),
                                            oracle_model(cfg), oracle_opts(opts, precision),
                                            grad_rgb=g_rgb[idx].astype(np.float64),
                                            grad_feat=None if g_ft is None else g_ft[idx].astype(np.float64),
                                            ray_ids=idx)
    errs = {k: _rel(got[k], ref[k]) for k in KEYS}
    print(f"config {ci} full size {precision}: {int(keep.sum())} of 256 rays kept, rel errors {errs}")
    for k in KEYS:
        assert errs[k] <= tol, (k, errs[k])
