"""Finite-difference check of the GPU gradient on the training batch of
config 2 (65,536 rays from 8 views of the 64-primitive scene, MSE against the
frames of a second seeded scene): central differences of the float64 GPU
forward on 32 parameters against the analytic backward, in FP32 and in the
split-bfloat16 form."""
import numpy as np
import pytest
import torch

import synth
from gpu_cases import opts_of, spec_of

pytestmark = pytest.mark.gpu

KEYS = ("center", "scale", "quat", "mlp")


def _f64_render(ctx, spec, opts, p64, o64, d64):
    from paper_2606_03877_amd import msplat_render_forward_f64
    R = o64.shape[0]
    rgb = torch.empty((R, 3), dtype=torch.float64, device="cuda")
    tr = torch.empty((R,), dtype=torch.float64, device="cuda")
    ws = torch.empty(4096, dtype=torch.uint8, device="cuda")
    st, _ = msplat_render_forward_f64(ctx, spec, opts, p64["center"], p64["scale"], p64["quat"], p64["mlp"],
                                      o64, d64, rgb, tr, None, ws)
    assert st == 0, st
    return rgb


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("bf16x3", 2e-3)])
def test_batch_gradient_matches_central_differences(precision, tol):
    from paper_2606_03877_amd import Renderer, render
    cfg = synth.CONFIGS[2]
    sc = synth.make_scene(cfg)
    sc_t = synth.make_scene(cfg, seed=1000 * cfg.idx + 10)
    o, d, _ = synth.make_rays(cfg)
    opts = opts_of(cfg, t_stop=0.0)       # no cut: the step must not move a discrete decision
    spec = spec_of(cfg, precision)
    r = Renderer(spec, opts)
    dev = torch.device("cuda", 0)
    o64 = torch.from_numpy(o.astype(np.float64)).to(dev)
    d64 = torch.from_numpy(d.astype(np.float64)).to(dev)
    p64 = {k: torch.from_numpy(v.astype(np.float64)).to(dev) for k, v in sc.items()}
    t64 = {k: torch.from_numpy(v.astype(np.float64)).to(dev) for k, v in sc_t.items()}
    target = _f64_render(r.ctx, spec, opts, t64, o64, d64)
    R = o.shape[0]

    def loss64(p):
        rgb = _f64_render(r.ctx, spec, opts, p, o64, d64)
        return float(((rgb - target) ** 2).sum() / (3 * R))

    # analytic gradient through the autograd Function
    leaf = {k: torch.from_numpy(v).to(dev).requires_grad_(True) for k, v in sc.items()}
    ro, rd = torch.from_numpy(o).to(dev), torch.from_numpy(d).to(dev)
    rgb, _, _ = render(r, leaf["center"], leaf["scale"], leaf["quat"], leaf["mlp"], ro, rd)
    loss = ((rgb - target.float()) ** 2).mean()
    loss.backward()
    grads = {k: leaf[k].grad.double().cpu().numpy() for k in KEYS}
    # 16 network parameters spread over the layers, 16 geometry values of hit primitives
    rng = np.random.default_rng(2024)
    _, _, _, ws = r.forward(leaf["center"].detach(), leaf["scale"].detach(), leaf["quat"].detach(),
                            leaf["mlp"].detach(), ro, rd)
    off, prim, _, _ = r.hits(ws, R)
    counts = np.bincount(prim, minlength=cfg.num_prims)
    hit_prims = np.nonzero(counts > 200)[0]
    dims = synth.layer_dims(cfg)
    layer_starts = np.cumsum([0] + [i * o_ + o_ for i, o_ in dims])
    picks = []
    for li in range(len(dims)):
        for _ in range(4):
            p = int(rng.choice(hit_prims))
            picks.append(("mlp", (p, int(rng.integers(layer_starts[li], layer_starts[li + 1])))))
    for key, width in (("center", 3), ("scale", 3), ("quat", 4)):
        n_k = 6 if key != "quat" else 4
        for _ in range(n_k):
            picks.append((key, (int(rng.choice(hit_prims)), int(rng.integers(0, width)))))
    picks = picks[:32]
    scale_g = {k: max(np.abs(grads[k]).max(), 1e-30) for k in KEYS}
    bad = []
    for key, idx in picks:
        h = 1e-4 * max(1.0, abs(float(p64[key][idx])))
        pp = {k: v.clone() for k, v in p64.items()}
        pm = {k: v.clone() for k, v in p64.items()}
        pp[key][idx] += h
        pm[key][idx] -= h
        fd = (loss64(pp) - loss64(pm)) / (2 * h)
        g = grads[key][idx]
        err = abs(fd - g) / scale_g[key]
        # truncation of the central difference: h^2/6 * f''' ~ (h * 2^(L-1) pi / s)^2 / 6
        trunc = (h * 32 * np.pi / 0.05) ** 2 / 6 * abs(fd) / scale_g[key]
        if err > max(tol, trunc) * 3:
            bad.append((key, idx, fd, g, err))
    print(f"{precision}: {len(picks)} parameters, outside tolerance: {bad}")
    assert not bad
