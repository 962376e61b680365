"""Shared seeded cases for the GPU parity tests (inputs from synth, expected
values from the oracle, GPU results through the C ABI binding)."""
import functools

import numpy as np
import torch

import oracle
import synth

GPU = None


def gpu_available() -> bool:
    global GPU
    if GPU is None:
        GPU = torch.cuda.is_available()
    return GPU


def spec_of(cfg, precision):
    from paper_2606_03877_amd import NetSpec
    return NetSpec(cfg.num_prims, cfg.pe_freqs, cfg.hidden_width, cfg.hidden_layers, cfg.out_dim,
                   precision)


def opts_of(cfg, t_stop=None, jitter_seed=1234, order=0):
    from paper_2606_03877_amd import RenderOpts
    return RenderOpts(samples_fixed=cfg.samples_fixed, samples_min=cfg.samples_min,
                      samples_max=cfg.samples_max, samples_per_unit=cfg.samples_per_unit,
                      t_stop=cfg.t_stop if t_stop is None else t_stop, jitter=cfg.jitter,
                      jitter_seed=jitter_seed, order=order)


# ReLU gates are decisions of a floating-point sum: the oracle takes them in
# the arithmetic of the form under test (oracle.gate_preacts), and its
# gradient follows the branch those gates select
GATE_FORM = {"fp32": "fp64", "bf16": "bf16", "bf16x3": "bf16x3"}


def oracle_opts(o, precision=None):
    """Oracle options of library options ``o``; with ``precision`` the ReLU
    gates are taken in that form's arithmetic."""
    return oracle.Opts(samples_fixed=o.samples_fixed, samples_min=o.samples_min,
                       samples_max=o.samples_max, samples_per_unit=o.samples_per_unit,
                       t_stop=o.t_stop, jitter=o.jitter, jitter_seed=o.jitter_seed,
                       background=tuple(o.background), order=o.order,
                       gate_form=GATE_FORM[precision] if precision else "fp64")


def oracle_model(cfg):
    return oracle.Model(cfg.pe_freqs, cfg.hidden_width, cfg.hidden_layers, cfg.out_dim)


@functools.lru_cache(maxsize=None)
def scene(ci):
    return synth.make_scene(synth.CONFIGS[ci])


def view_camera(ci, width, height, seed=None):
    """The camera of view_rays."""
    cfg = synth.CONFIGS[ci]
    rng = np.random.default_rng(1000 * ci + 1 if seed is None else seed)
    return synth.make_camera(rng, width, height, cfg.camera_radius, cfg.fov_deg)


def view_rays(ci, width, height, seed=None):
    """Rays of one (ragged if asked) view drawn like the configuration's cameras."""
    o, d, _ = synth.camera_rays(view_camera(ci, width, height, seed))
    return o, d


def to_dev(sc, o, d):
    dev = torch.device("cuda", 0)
    t = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in sc.items()}
    return t, torch.from_numpy(np.ascontiguousarray(o)).to(dev), torch.from_numpy(np.ascontiguousarray(d)).to(dev)


# ReLU margin (oracle.relu_margin: distance of the closest gate from
# switching, in units of its rounding noise, measured on the pre-activations
# of the form's own arithmetic, GATE_FORM) below which the kernel may still
# take a gate the other way: for float32 about 16 unit roundoffs (2^-24); for
# the bfloat16 forms the oracle's pre-activations differ from the kernel's
# only by float32 sums and the float32 encoding the operands are cut from
RELU_AMBIGUOUS = {"fp32": 1e-6, "bf16x3": 1e-6, "bf16": 1e-6}
# largest share of a case's rays that may be left without upstream gradient
# (a termination cut or a ReLU gate decided within rounding)
MASK_MAX = 0.05


def oracle_render(ci, sc, o, d, opts, ray_ids=None, chunk=4096, margins=False, centre=None, precision=None):
    """Oracle forward in chunks (of whole 64-ray packets); with ``margins``
    also the smallest ReLU margin over each ray's samples (``relu_margin``, inf
    for rays without samples), gates taken in ``precision``'s arithmetic.
    ``centre`` gives tile order's per-ray virtual rays when the rays are a
    scattered subset of a batch."""
    cfg = synth.CONFIGS[ci]
    p = oracle.to_tensors(sc)
    oo = oracle_opts(opts, precision)
    rgbs, trs, fts, nus, offs, prims, mrg = [], [], [], [], [0], [], []
    for s in range(0, len(o), chunk):
        e = min(len(o), s + chunk)
        ids = None if ray_ids is None else ray_ids[s:e]
        out = oracle.render(p["center"], p["scale"], p["quat"], p["mlp"],
                            torch.from_numpy(o[s:e].astype(np.float64)),
                            torch.from_numpy(d[s:e].astype(np.float64)), oracle_model(cfg), oo,
                            ray_index_base=s, ray_ids=ids, keep_samples=margins,
                            centre=None if centre is None else (centre[0][s:e], centre[1][s:e]))
        if margins:
            m = np.full(e - s, np.inf)
            smp = out["samples"]
            if smp is not None:
                np.minimum.at(m, smp["ray"], smp["relu_margin"])
            mrg.append(m)
        rgbs.append(out["rgb"].numpy())
        trs.append(out["trans"].numpy())
        fts.append(out["feat"].numpy())
        nus.append(out["n_used"])
        offs.extend((out["ray_off"][1:] + offs[-1]).tolist())
        prims.append(out["prim"])
    res = {"rgb": np.concatenate(rgbs), "trans": np.concatenate(trs), "feat": np.concatenate(fts),
           "n_used": np.concatenate(nus), "ray_off": np.array(offs, np.int64),
           "prim": np.concatenate(prims)}
    if margins:
        res["relu_margin"] = np.concatenate(mrg)
    return res


def gpu_render(ci, precision, sc, o, d, opts):
    from paper_2606_03877_amd import Renderer
    cfg = synth.CONFIGS[ci]
    r = Renderer(spec_of(cfg, precision), opts)
    t, to, td = to_dev(sc, o, d)
    rgb, trans, feat, ws = r.forward(t["center"], t["scale"], t["quat"], t["mlp"], to, td)
    torch.cuda.synchronize()
    st = r.stats(ws)
    off, prim, tc, nused = r.hits(ws, len(o))
    return {"rgb": rgb.cpu().numpy(), "trans": trans.cpu().numpy(),
            "feat": None if feat is None else feat.cpu().numpy(), "stats": st,
            "ray_off": off, "prim": prim, "t_c": tc, "hit_nused": nused,
            "renderer": r, "ws": ws, "dev": (t, to, td)}


def ray_nused(res):
    off = res["ray_off"]
    cs = np.concatenate([[0], np.cumsum(res["hit_nused"].astype(np.int64))])
    return cs[off[1:]] - cs[off[:-1]]


def compare_rgb(g, ref, tol, t_stop, idx=None):
    """Max-abs RGB error over rays whose composited sample count agrees, and
    the count/error of rays where the termination cut fell on another sample."""
    nu_g = ray_nused(g)
    if idx is not None:
        nu_g = nu_g[idx]
        grgb = g["rgb"][idx]
        gtr = g["trans"][idx]
    else:
        grgb, gtr = g["rgb"], g["trans"]
    same = nu_g == ref["n_used"]
    err = np.abs(grgb - ref["rgb"]).max(1)
    terr = np.abs(gtr - ref["trans"])
    out = {"max_err": float(err[same].max()) if same.any() else 0.0,
           "max_terr": float(terr[same].max()) if same.any() else 0.0,
           "mean_err": float(err.mean()), "n_cut_mismatch": int((~same).sum()),
           "cut_mismatch_err": float(err[~same].max()) if (~same).any() else 0.0,
           "E1": float(np.linalg.norm(grgb - ref["rgb"], axis=1).mean()),
           "E2": float(np.sqrt((np.linalg.norm(grgb - ref["rgb"], axis=1) ** 2).mean()))}
    return out


def gradient_mask(g_nused, ref_fwd, precision, R):
    """Rays that carry an upstream gradient: the termination cut on the same
    sample as the oracle's, and no ReLU gate within rounding of switching in
    the form's arithmetic.  At most MASK_MAX of the rays are left out."""
    same = g_nused == ref_fwd["n_used"]
    clear = ref_fwd["relu_margin"] >= RELU_AMBIGUOUS[precision]
    keep = same & clear
    print(f"rays left out: {R - int(keep.sum())} of {R} (cut {int((~same).sum())}, "
          f"gate {int((~clear).sum())})")
    assert R - keep.sum() <= MASK_MAX * R
    return keep
