"""GPU parity in the corners of the option space: rays starting inside a
primitive (chord clipped at t = 0), a non-black background, midpoint samples
(no jitter), chord-proportional sample counts up to the 128 maximum, an
early-termination threshold high enough to cut most rays, and rays with more
hits than a register-sorted group holds."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_cases import (RELU_AMBIGUOUS, compare_rgb, gpu_render, gradient_mask, oracle_model, oracle_opts,
                       oracle_render, ray_nused, scene, spec_of, to_dev)

pytestmark = pytest.mark.gpu

KEYS = ("center", "scale", "quat", "mlp")
TOL = {"fp32": 1e-5, "bf16x3": 2e-3}


def _rays_from_inside(ci, n, seed):
    """n rays from the centre of primitive 0 (so its chord starts at t = 0)
    plus n rays from a camera outside, in seeded random directions."""
    sc = scene(ci)
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((2 * n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = np.empty((2 * n, 3))
    o[:n] = sc["center"][0]
    o[n:] = [0.2, -2.5, 0.4]
    return sc, o.astype(np.float32), d.astype(np.float32)


def _opts(t_stop):
    from paper_2606_03877_amd import RenderOpts
    return RenderOpts(samples_fixed=0, samples_min=8, samples_max=128, samples_per_unit=400.0,
                      t_stop=t_stop, jitter=0, jitter_seed=0, background=(0.3, 0.5, 0.7))


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("t_stop", [0.0, 0.3])
def test_clipped_chords_background_midpoints(precision, t_stop):
    ci = 0
    sc, o, d = _rays_from_inside(ci, 600, seed=31)
    opts = _opts(t_stop)
    g = gpu_render(ci, precision, sc, o, d, opts)
    ref = oracle_render(ci, sc, o, d, opts, margins=True, precision=precision)
    np.testing.assert_array_equal(g["ray_off"], ref["ray_off"])
    np.testing.assert_array_equal(g["prim"], ref["prim"])
    c = compare_rgb(g, ref, TOL[precision], opts.t_stop)
    K = np.asarray(oracle.render(*[oracle.to_tensors(sc)[k] for k in KEYS],
                                 torch.from_numpy(o[:4].astype(np.float64)),
                                 torch.from_numpy(d[:4].astype(np.float64)),
                                 oracle_model(synth.CONFIGS[ci]), oracle_opts(opts))["K"])
    print(f"{precision} t_stop={t_stop}: {c}; K of the first hits {K}")
    assert c["max_err"] <= TOL[precision]
    assert c["cut_mismatch_err"] <= opts.t_stop + TOL[precision]
    # gradients, rays with a cut or gate decided within rounding left out
    keep = gradient_mask(ray_nused(g), ref, precision, len(o))
    g_rgb = (np.random.default_rng(32).standard_normal((len(o), 3)) / len(o)).astype(np.float32)
    g_rgb[~keep] = 0.0
    t, to, td = g["dev"]
    out = g["renderer"].backward(g["ws"], t["center"], t["scale"], t["quat"], t["mlp"], to, td,
                                 torch.from_numpy(g_rgb).cuda())
    got = dict(zip(KEYS, [x.cpu().numpy() for x in out]))
    _, _, _, grads, _ = oracle.loss_and_grads(sc, o.astype(np.float64), d.astype(np.float64),
                                              oracle_model(synth.CONFIGS[ci]), oracle_opts(opts, precision),
                                              grad_rgb=g_rgb)
    for k in KEYS:
        err = float(np.abs(got[k] - grads[k]).max() / max(np.abs(grads[k]).max(), 1e-30))
        print(f"  {k}: {err:.2e}")
        assert err <= TOL[precision], k


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("t_stop", [0.0, 1e-4])
def test_rays_with_more_hits_than_a_sorted_group(precision, t_stop):
    """600 nested supports around the origin and rays from near it: every ray
    hits all 600 primitives, more than the 512 hits the fill sorts in
    registers per group of rays, so every packet takes the per-ray path
    (appended in primitive order, insertion-sorted in the ray's segment).
    Hit lists bit-exact, RGB and gradients within the form's bar (133 rays:
    two full packets and a ragged one)."""
    from paper_2606_03877_amd import Renderer, RenderOpts
    ci = 0
    cfg = dataclasses.replace(synth.CONFIGS[ci], num_prims=600)
    sc = synth.make_scene(cfg, seed=51)
    rng = np.random.default_rng(52)
    sc["center"] = rng.uniform(-0.05, 0.05, (600, 3))
    sc["scale"] = rng.uniform(0.6, 1.0, (600, 3))
    sc = {k: np.ascontiguousarray(v, np.float32) for k, v in sc.items()}
    n = 2 * 64 + 5
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = rng.uniform(-0.02, 0.02, (n, 3))
    o, d = o.astype(np.float32), d.astype(np.float32)
    opts = RenderOpts(samples_fixed=4, t_stop=t_stop, jitter=1, jitter_seed=53)
    r = Renderer(spec_of(cfg, precision), opts)
    t, to, td = to_dev(sc, o, d)
    rgb, trans, _, ws = r.forward(t["center"], t["scale"], t["quat"], t["mlp"], to, td)
    torch.cuda.synchronize()
    off, prim, _, nused = r.hits(ws, n)
    g = {"rgb": rgb.cpu().numpy(), "trans": trans.cpu().numpy(), "ray_off": off, "prim": prim,
         "hit_nused": nused}
    assert np.diff(g["ray_off"]).min() > 512
    ref = oracle_render(ci, sc, o, d, opts)
    np.testing.assert_array_equal(g["ray_off"], ref["ray_off"])
    np.testing.assert_array_equal(g["prim"], ref["prim"])
    c = compare_rgb(g, ref, TOL[precision], opts.t_stop)
    print(f"{precision} t_stop={t_stop}: {len(g['prim'])} hits; {c}")
    assert c["max_err"] <= TOL[precision]
    assert c["cut_mismatch_err"] <= opts.t_stop + TOL[precision]
    if t_stop == 0.0:
        return
    # the gradient through 600 hits per ray (the adjoint walks each ray's
    # chunks from the last hit back).  Rays are left out where the cut falls
    # on another sample or a ReLU gate of a composited sample is within
    # rounding of switching (the samples past the cut carry no gradient).
    p64 = oracle.to_tensors(sc)
    out_s = oracle.render(p64["center"], p64["scale"], p64["quat"], p64["mlp"],
                          torch.from_numpy(o.astype(np.float64)), torch.from_numpy(d.astype(np.float64)),
                          oracle_model(cfg), oracle_opts(opts, precision), keep_samples=True)
    smp = out_s["samples"]
    sray = np.asarray(smp["ray"])
    first = np.searchsorted(sray, np.arange(n))
    composited = np.arange(len(sray)) - first[sray] < out_s["n_used"][sray]
    margin = np.full(n, np.inf)
    np.minimum.at(margin, sray[composited], np.asarray(smp["relu_margin"])[composited])
    keep = (ray_nused(g) == out_s["n_used"]) & (margin >= RELU_AMBIGUOUS[precision])
    print(f"rays left out: {n - int(keep.sum())} of {n}")
    assert n - keep.sum() <= 0.05 * n
    g_rgb = (np.random.default_rng(54).standard_normal((n, 3)) / n).astype(np.float32)
    g_rgb[~keep] = 0.0
    out = r.backward(ws, t["center"], t["scale"], t["quat"], t["mlp"], to, td, torch.from_numpy(g_rgb).cuda())
    got = dict(zip(KEYS, [x.cpu().numpy() for x in out]))
    _, _, _, grads, _ = oracle.loss_and_grads(sc, o.astype(np.float64), d.astype(np.float64),
                                              oracle_model(cfg), oracle_opts(opts, precision), grad_rgb=g_rgb)
    for k in KEYS:
        err = float(np.abs(got[k] - grads[k]).max() / max(np.abs(grads[k]).max(), 1e-30))
        print(f"  {k}: {err:.2e}")
        assert err <= TOL[precision], k
