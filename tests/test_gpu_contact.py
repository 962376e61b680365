"""GPU parity of the paper's contact-point primitive (one interaction per
hit at Eq. 2's contact point, the 72-32-32-4 network on the encoded
[d; delta], Gaussian falloff and line-integral thickness) against the FP64
oracle (oracle/contact.py), through the C ABI."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle.contact import ContactModel, contact_loss_and_grads, contact_margins, render_contact
from gpu_cases import GATE_FORM, MASK_MAX, RELU_AMBIGUOUS, scene, to_dev, view_rays

pytestmark = pytest.mark.gpu

CI = 6
CFG = synth.CONFIGS[CI]
MODEL = ContactModel(CFG.pe_freqs, CFG.hidden_width, CFG.hidden_layers, CFG.out_dim)
KEYS = ("center", "scale", "quat", "mlp")
TOL = {"fp32": 1e-5, "bf16": 2e-3, "bf16x3": 2e-3}


def _renderer(precision, t_stop=1e-4, order=0):
    from paper_2606_03877_amd import NetSpec, RenderOpts, Renderer
    spec = NetSpec(CFG.num_prims, CFG.pe_freqs, CFG.hidden_width, CFG.hidden_layers, CFG.out_dim, precision,
                   primitive="contact")
    return Renderer(spec, RenderOpts(samples_fixed=1, t_stop=t_stop, jitter=0, order=order))


def _oracle_opts(r, precision=None):
    o = oracle.Opts(t_stop=r.opts.t_stop, background=tuple(r.opts.background), order=r.opts.order)
    return dataclasses.replace(o, gate_form=GATE_FORM[precision]) if precision else o


def _oracle(sc, o, d, oo, chunk=2048, centre=None):
    p = oracle.to_tensors(sc)
    outs = []
    for s in range(0, len(o), chunk):
        e = min(len(o), s + chunk)
        outs.append(render_contact(p["center"], p["scale"], p["quat"], p["mlp"],
                                   torch.from_numpy(o[s:e].astype(np.float64)),
                                   torch.from_numpy(d[s:e].astype(np.float64)), MODEL, oo,
                                   centre=None if centre is None else (centre[0][s:e], centre[1][s:e])))
    off = [0]
    for x in outs:
        off.extend((x["ray_off"][1:] + off[-1]).tolist())
    return {"rgb": np.concatenate([x["rgb"].detach().numpy() for x in outs]),
            "trans": np.concatenate([x["trans"].detach().numpy() for x in outs]),
            "n_used": np.concatenate([x["n_used"] for x in outs]),
            "ray_off": np.array(off, np.int64), "prim": np.concatenate([x["prim"] for x in outs])}


def _gpu(r, sc, o, d):
    t, to, td = to_dev(sc, o, d)
    rgb, trans, feat, ws = r.forward(t["center"], t["scale"], t["quat"], t["mlp"], to, td)
    torch.cuda.synchronize()
    off, prim, tc, nused = r.hits(ws, len(o))
    cs = np.concatenate([[0], np.cumsum(nused.astype(np.int64))])
    return {"rgb": rgb.cpu().numpy(), "trans": trans.cpu().numpy(), "ray_off": off, "prim": prim,
            "n_used": cs[off[1:]] - cs[off[:-1]], "ws": ws, "dev": (t, to, td), "stats": r.stats(ws)}


@pytest.mark.parametrize("w,h", [(96, 70), (40, 33)])
def test_contact_hit_lists_are_bit_exact(w, h):
    sc = scene(CI)
    o, d = view_rays(CI, w, h)
    r = _renderer("fp32")
    g = _gpu(r, sc, o, d)
    ref = _oracle(sc, o, d, _oracle_opts(r))
    print(f"{w}x{h}: {len(g['prim'])} hits, fallbacks {g['stats']['num_fallbacks']}")
    assert len(g["prim"]) > len(o) // 4
    np.testing.assert_array_equal(g["ray_off"], ref["ray_off"])
    np.testing.assert_array_equal(g["prim"], ref["prim"])


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("t_stop", [1e-4, 0.0])
def test_contact_forward_matches_oracle(precision, t_stop):
    sc = scene(CI)
    o, d = view_rays(CI, 96, 70)
    r = _renderer(precision, t_stop)
    g = _gpu(r, sc, o, d)
    ref = _oracle(sc, o, d, _oracle_opts(r))
    same = g["n_used"] == ref["n_used"]
    err = np.abs(g["rgb"] - ref["rgb"]).max(1)
    terr = np.abs(g["trans"] - ref["trans"])
    print(f"{precision} t_stop={t_stop}: max err {err[same].max():.3g}, T err {terr[same].max():.3g}, "
          f"cut mismatches {(~same).sum()}")
    assert err[same].max() <= TOL[precision]
    assert terr[same].max() <= 4 * TOL[precision]
    assert (~same).sum() <= max(1, len(o) // 1000)
    if (~same).any():
        assert err[~same].max() <= t_stop + TOL[precision]


def _grad_case(precision, w, h, t_stop=1e-4, order=0, centre=None):
    sc = scene(CI)
    o, d = view_rays(CI, w, h)
    r = _renderer(precision, t_stop, order)
    g = _gpu(r, sc, o, d)
    oo = _oracle_opts(r, precision)
    p = oracle.to_tensors(sc)
    _, margin = contact_margins(p["center"], p["scale"], p["quat"], p["mlp"], torch.from_numpy(o.astype(np.float64)),
                                torch.from_numpy(d.astype(np.float64)), MODEL, oo)
    ref = _oracle(sc, o, d, oo, centre=centre)
    keep = (g["n_used"] == ref["n_used"]) & (margin >= RELU_AMBIGUOUS[precision])
    R = len(o)
    print(f"{precision}: rays masked {R - int(keep.sum())} of {R} "
          f"(cut {int((g['n_used'] != ref['n_used']).sum())})")
    assert R - keep.sum() <= MASK_MAX * R
    g_rgb = (np.random.default_rng(6004).standard_normal((R, 3)) / R).astype(np.float32)
    g_rgb[~keep] = 0.0
    _, _, want = contact_loss_and_grads(sc, o, d, MODEL, oo, g_rgb, centre=centre)
    t, to, td = g["dev"]
    got = r.backward(g["ws"], t["center"], t["scale"], t["quat"], t["mlp"], to, td, torch.from_numpy(g_rgb).cuda())
    return {k: v.cpu().numpy() for k, v in zip(KEYS, got)}, want


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_contact_gradients_match_oracle(precision):
    got, want = _grad_case(precision, 96, 70)
    for k in KEYS:
        err = float(np.abs(got[k] - want[k]).max() / max(np.abs(want[k]).max(), 1e-30))
        print(f"  {k}: {err:.2e}")
        assert err <= TOL[precision], k


def test_contact_gradients_without_termination():
    got, want = _grad_case("fp32", 64, 48, t_stop=0.0)
    for k in KEYS:
        err = float(np.abs(got[k] - want[k]).max() / max(np.abs(want[k]).max(), 1e-30))
        assert err <= TOL["fp32"], (k, err)


def test_contact_tile_order():
    """Tile order: hit sets and counts as in exact order, every packet's
    hits in the order of the depths along its virtual ray; RGB and
    gradients against the oracle in the same order."""
    sc = scene(CI)
    o, d = view_rays(CI, 64, 48)
    r = _renderer("fp32", order=1)
    g = _gpu(r, sc, o, d)
    ref = _oracle(sc, o, d, _oracle_opts(r))
    np.testing.assert_array_equal(g["ray_off"], ref["ray_off"])
    # (float32 keys: near-ties may order either way; count them)
    differ = [i for i in range(len(o))
              if not np.array_equal(g["prim"][g["ray_off"][i]:g["ray_off"][i + 1]],
                                    ref["prim"][ref["ray_off"][i]:ref["ray_off"][i + 1]])]
    assert len(differ) <= max(1, len(o) // 1000)
    same = np.ones(len(o), bool)
    same[differ] = False
    same &= g["n_used"] == ref["n_used"]
    assert np.abs(g["rgb"] - ref["rgb"])[same].max() <= TOL["fp32"]
    got, want = _grad_case("fp32", 64, 48, order=1)
    for k in KEYS:
        err = float(np.abs(got[k] - want[k]).max() / max(np.abs(want[k]).max(), 1e-30))
        assert err <= 1e-4, (k, err)


def test_contact_full_frame_sampled_rays():
    """The 800x800 frame of 2048 primitives in one call, as the benchmark
    launches it, checked on 512 seeded rays (hit lists and RGB)."""
    sc = scene(CI)
    o, dd, _ = synth.make_rays(CFG)
    r = _renderer("bf16x3")
    g = _gpu(r, sc, o, dd)
    idx = np.sort(np.random.default_rng(79).choice(len(o), 512, replace=False))
    ref = _oracle(sc, o[idx], dd[idx], _oracle_opts(r))
    for n, i in enumerate(idx):
        np.testing.assert_array_equal(g["prim"][g["ray_off"][i]:g["ray_off"][i + 1]],
                                      ref["prim"][ref["ray_off"][n]:ref["ray_off"][n + 1]])
    same = g["n_used"][idx] == ref["n_used"]
    err = np.abs(g["rgb"][idx] - ref["rgb"])[same].max()
    print(f"full frame: {len(g['prim'])} hits, rgb err {err:.3g}, stats {g['stats']}")
    assert err <= TOL["bf16x3"]


def test_contact_plain_bf16_is_not_compiled():
    """Plain bfloat16 misses the 2e-3 RGB bar on the 72-input network
    (3.0e-3 measured): the contact primitive runs in FP32 and split BF16."""
    from paper_2606_03877_amd import MsplatError, _lib
    sc = scene(CI)
    o, d = view_rays(CI, 16, 8)
    r = _renderer("bf16")
    with pytest.raises(MsplatError) as e:
        _gpu(r, sc, o, d)
    assert e.value.status == _lib.MSPLAT_E_UNSUPPORTED


def test_contact_rejects_slot_features():
    from paper_2606_03877_amd import MsplatError
    sc = scene(CI)
    o, d = view_rays(CI, 16, 8)
    r = _renderer("fp32")
    g = _gpu(r, sc, o, d)
    with pytest.raises(MsplatError):
        r.slot_forward(g["ws"], torch.zeros((CFG.num_prims, 4, 8), device="cuda"), len(o))
