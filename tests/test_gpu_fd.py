"""Finite-difference check of the GPU gradient on the training batch of
config 2 (65,536 rays from 8 views of the 64-primitive scene, MSE against the
frames of a second seeded scene): central differences of the float64 GPU
forward on 32 parameters against the analytic backward, in FP32 and in the
split-bfloat16 form.

A step of a parameter may move a discrete decision of some rays (a ray
entering or leaving a support, two hits swapping depth order, a ReLU gate
switching): the loss is not differentiable there, so for each parameter the
rays whose decisions differ at the two perturbed points (hit lists of the
float32 forward, the decision hash of the float64 forward) are masked out of
the loss, on both sides of the comparison."""
import numpy as np
import pytest
import torch

import synth
from gpu_cases import opts_of, spec_of

pytestmark = pytest.mark.gpu

KEYS = ("center", "scale", "quat", "mlp")


def _f64_render(ctx, spec, opts, p64, o64, d64, with_decisions=False):
    from paper_2606_03877_amd import msplat_render_forward_f64
    R = o64.shape[0]
    rgb = torch.empty((R, 3), dtype=torch.float64, device="cuda")
    tr = torch.empty((R,), dtype=torch.float64, device="cuda")
    dec = torch.empty((R,), dtype=torch.int32, device="cuda") if with_decisions else None
    ws = torch.empty(4096, dtype=torch.uint8, device="cuda")
    st, _ = msplat_render_forward_f64(ctx, spec, opts, p64["center"], p64["scale"], p64["quat"], p64["mlp"],
                                      o64, d64, rgb, tr, None, ws, decisions=dec)
    assert st == 0, st
    return (rgb, dec) if with_decisions else rgb


def _hit_lists(r, p32, ro, rd):
    _, _, _, ws = r.forward(p32["center"], p32["scale"], p32["quat"], p32["mlp"], ro, rd)
    off, prim, _, _ = r.hits(ws, ro.shape[0])
    return off, prim


def _same_lists(a, b):
    """Per ray: True where the depth-ordered primitive lists agree."""
    (oa, pa), (ob, pb) = a, b
    R = len(oa) - 1
    na, nb = np.diff(oa), np.diff(ob)
    same = na == nb
    # compare lists of rays with equal counts via a padded table
    w = int(max(na.max(initial=0), nb.max(initial=0)))
    ta = np.full((R, max(w, 1)), -1, np.int64)
    tb = np.full((R, max(w, 1)), -1, np.int64)
    ra = np.repeat(np.arange(R), na)
    rb = np.repeat(np.arange(R), nb)
    ta[ra, np.arange(len(pa)) - oa[ra]] = pa
    tb[rb, np.arange(len(pb)) - ob[rb]] = pb
    return same & (ta == tb).all(1)


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("bf16x3", 2e-3)])
def test_batch_gradient_matches_central_differences(precision, tol):
    from paper_2606_03877_amd import Renderer
    cfg = synth.CONFIGS[2]
    sc = synth.make_scene(cfg)
    sc_t = synth.make_scene(cfg, seed=1000 * cfg.idx + 10)
    o, d, _ = synth.make_rays(cfg)
    opts = opts_of(cfg, t_stop=0.0)       # no cut: the step must not move a termination decision
    spec = spec_of(cfg, precision)
    r = Renderer(spec, opts)
    dev = torch.device("cuda", 0)
    o64 = torch.from_numpy(o.astype(np.float64)).to(dev)
    d64 = torch.from_numpy(d.astype(np.float64)).to(dev)
    ro, rd = torch.from_numpy(o).to(dev), torch.from_numpy(d).to(dev)
    p64 = {k: torch.from_numpy(v.astype(np.float64)).to(dev) for k, v in sc.items()}
    p32 = {k: torch.from_numpy(v).to(dev) for k, v in sc.items()}
    t64 = {k: torch.from_numpy(v.astype(np.float64)).to(dev) for k, v in sc_t.items()}
    target = _f64_render(r.ctx, spec, opts, t64, o64, d64)
    R = o.shape[0]
    rgb, _, _, ws = r.forward(p32["center"], p32["scale"], p32["quat"], p32["mlp"], ro, rd)
    base = r.hits(ws, R)
    off, prim = base[0], base[1]
    base = (off, prim)
    counts = np.bincount(prim, minlength=cfg.num_prims)
    hit_prims = np.nonzero(counts > 200)[0]
    # 16 network parameters spread over the layers, 16 geometry values of hit primitives
    rng = np.random.default_rng(2024)
    dims = synth.layer_dims(cfg)
    layer_starts = np.cumsum([0] + [i * o_ + o_ for i, o_ in dims])
    picks = []
    for li in range(len(dims)):
        for _ in range(4):
            p = int(rng.choice(hit_prims))
            picks.append(("mlp", (p, int(rng.integers(layer_starts[li], layer_starts[li + 1])))))
    for key, width, n_k in (("center", 3, 6), ("scale", 3, 6), ("quat", 4, 4)):
        for _ in range(n_k):
            picks.append((key, (int(rng.choice(hit_prims)), int(rng.integers(0, width)))))
    bad, masked, ratios = [], [], []
    for key, idx in picks:
        x = float(sc[key][idx])
        # geometry moves samples through an encoding of frequency up to
        # 2^(L-1) pi / s_min per unit of world length: keep that phase step small
        h = (1e-6 if key != "mlp" else 1e-5) * max(1.0, abs(x))
        pp = {k: v.clone() for k, v in p64.items()}
        pm = {k: v.clone() for k, v in p64.items()}
        pp[key][idx] += h
        pm[key][idx] -= h
        keep = np.ones(R, bool)
        for q in (pp, pm):
            q32 = {k: v.float().contiguous() for k, v in q.items()}
            keep &= _same_lists(base, _hit_lists(r, q32, ro, rd))
        # every discrete decision of the float64 forward (hit order, samples,
        # open ReLU gates) must agree at the two points, or the ray is masked
        out_p, dec_p = _f64_render(r.ctx, spec, opts, pp, o64, d64, with_decisions=True)
        out_m, dec_m = _f64_render(r.ctx, spec, opts, pm, o64, d64, with_decisions=True)
        keep &= (dec_p == dec_m).cpu().numpy()
        masked.append(int((~keep).sum()))
        mk = torch.from_numpy(keep.astype(np.float64)).to(dev)[:, None]
        lp = float((((out_p - target) ** 2) * mk).sum() / (3 * R))
        lm = float((((out_m - target) ** 2) * mk).sum() / (3 * R))
        fd = (lp - lm) / (2 * h)
        g_rgb = ((2.0 / (3 * R)) * (rgb.double() - target) * mk).float()
        grads = r.backward(ws, p32["center"], p32["scale"], p32["quat"], p32["mlp"], ro, rd, g_rgb)
        gk = grads[KEYS.index(key)].double().cpu().numpy()
        g = gk[idx]
        scale_g = max(np.abs(gk).max(), 1e-30)
        err = abs(fd - g) / scale_g
        # truncation of the central difference (h^2/6 times the third
        # derivative): for geometry the third derivative is of the order of the
        # gradient scale times the squared phase rate (highest encoding
        # frequency over the smallest scale, 0.05)
        trunc = (h * 32 * np.pi / 0.05) ** 2 / 6 if key != "mlp" else h ** 2
        ratios.append((err / max(tol, trunc), key))
        if err > max(tol, trunc):
            bad.append((key, idx, fd, g, err))
    print(f"{precision}: {len(picks)} parameters, rays masked per parameter {masked}, "
          f"largest error over the bar {max(ratios)}, outside tolerance: {bad}")
    assert not bad
