"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a library
routine (scipy rotations, numpy polynomial roots, a numpy MLP chain), a closed
form, an invariant, brute-force marching, or complex-step derivatives.
"""
import math

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

import oracle
import synth

F64 = torch.float64


def t64(x):
    return torch.from_numpy(np.array(x, np.float64))


def render_np(scene, o, d, model, opts, **kw):
    p = oracle.to_tensors(scene)
    return oracle.render(p["center"], p["scale"], p["quat"], p["mlp"], t64(o), t64(d), model, opts, **kw)


def scipy_rot(q_wxyz):
    q = np.asarray(q_wxyz, np.float64)
    return Rotation.from_quat(np.stack([q[..., 1], q[..., 2], q[..., 3], q[..., 0]], -1)).as_matrix()


def lam(scale, q):
    r = scipy_rot(q)
    return r @ np.diag(1.0 / np.asarray(scale, np.float64) ** 2) @ r.T


def const_params(model, rgb, sigma):
    """MLP parameters whose output is constant: every output weight is zero,
    output bias = (logit(rgb), softplus^-1(sigma), 0...)."""
    th = np.zeros(model.num_params)
    dims = model.layer_dims()
    off = sum(i * o + o for i, o in dims[:-1])
    fi, fo = dims[-1]
    off += fi * fo
    rgb = np.asarray(rgb, np.float64)
    th[off:off + 3] = np.log(rgb / (1 - rgb))
    th[off + 3] = math.log(math.expm1(sigma))
    return th


SMALL = oracle.Model(pe_freqs=2, hidden_width=8, hidden_layers=2, out_dim=4)


def chord(o, d, mu, scale, q):
    """Entry/exit of the ray in the ellipsoid from the quadratic
    (o + t d - mu)^T Lambda (o + t d - mu) = 1, by numpy.roots."""
    L = lam(scale, q)
    r = np.asarray(o, np.float64) - np.asarray(mu, np.float64)
    d = np.asarray(d, np.float64)
    roots = np.roots([d @ L @ d, 2 * d @ L @ r, r @ L @ r - 1])
    roots = np.sort(roots.real) if np.all(np.isreal(roots)) else None
    return roots


# ---------------------------------------------------------------- geometry --

def test_rotation_matches_scipy_hamilton():
    rng = np.random.default_rng(0)
    q = rng.standard_normal((50, 4)) * rng.uniform(0.2, 3.0, (50, 1))
    r = oracle.quat_to_rotmat(t64(q)).numpy()
    np.testing.assert_allclose(r, scipy_rot(q), atol=1e-14)
    np.testing.assert_allclose(np.linalg.det(r), 1.0, atol=1e-13)
    np.testing.assert_allclose(r @ np.swapaxes(r, 1, 2), np.broadcast_to(np.eye(3), r.shape), atol=1e-13)
    np.testing.assert_allclose(oracle.quat_to_rotmat(t64(-q)).numpy(), r, atol=1e-14)


def test_local_frame_metric():
    rng = np.random.default_rng(1)
    s = rng.uniform(0.05, 0.5, (10, 3))
    q = rng.standard_normal((10, 4))
    m = oracle.local_frame(t64(s), t64(q)).numpy()
    for i in range(10):
        np.testing.assert_allclose(m[i].T @ m[i], lam(s[i], q[i]), rtol=1e-12, atol=1e-9)


def test_contact_depth_is_argmin_of_eq1():
    """t_c (clamped at 0) minimises |o + t d - mu|^2_Lambda over t >= 0."""
    from scipy.optimize import minimize_scalar
    rng = np.random.default_rng(2)
    for _ in range(40):
        mu = rng.uniform(-1, 1, 3)
        s = rng.uniform(0.05, 0.5, 3)
        q = rng.standard_normal(4)
        o = rng.standard_normal(3)
        o = 3 * o / np.linalg.norm(o)
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        L = lam(s, q)
        f = lambda t: (o + t * d - mu) @ L @ (o + t * d - mu)
        res = minimize_scalar(f, bounds=(0.0, 20.0), method="bounded", options={"xatol": 1e-12})
        isx = oracle.intersect(t64(o[None]), t64(d[None]), t64(mu[None]), t64(s[None]), t64(q[None]))
        tc = float(isx["tc"][0, 0])
        assert abs(max(tc, 0.0) - res.x) < 1e-6


def test_chord_matches_quadratic_roots_and_midpoint():
    rng = np.random.default_rng(3)
    n_hit = 0
    for _ in range(300):
        mu = rng.uniform(-1, 1, 3)
        s = rng.uniform(0.05, 0.5, 3)
        q = rng.standard_normal(4)
        o = rng.standard_normal(3)
        o = 3 * o / np.linalg.norm(o)
        d = (mu + rng.uniform(-0.3, 0.3, 3)) - o
        d /= np.linalg.norm(d)
        isx = oracle.intersect(t64(o[None]), t64(d[None]), t64(mu[None]), t64(s[None]), t64(q[None]))
        roots = chord(o, d, mu, s, q)
        hit = bool(isx["hit"][0, 0])
        if roots is None or roots[1] <= 0:
            assert not hit
            continue
        assert hit
        n_hit += 1
        np.testing.assert_allclose(float(isx["ta"][0, 0]), max(roots[0], 0.0), atol=1e-10)
        np.testing.assert_allclose(float(isx["tb"][0, 0]), roots[1], atol=1e-10)
        np.testing.assert_allclose(float(isx["tc"][0, 0]), 0.5 * (roots[0] + roots[1]), atol=1e-10)
    assert n_hit > 50


def test_sphere_through_center_has_chord_2r():
    r = 0.37
    o = np.array([[0.0, -3.0, 0.5]])
    d = np.array([[0.0, 1.0, 0.0]])
    isx = oracle.intersect(t64(o), t64(d), t64([[0.2 * 0, 0.4, 0.5]]), t64([[r, r, r]]),
                           t64([[0.3, -0.2, 0.9, 0.1]]))
    assert abs(float(isx["tb"][0, 0] - isx["ta"][0, 0]) - 2 * r) < 1e-13
    assert abs(float(isx["tc"][0, 0]) - 3.4) < 1e-13


def test_hit_set_matches_bruteforce_marching():
    """Point-in-ellipsoid marching along each ray brackets [t_a, t_b]."""
    rng = np.random.default_rng(4)
    npr, nr = 6, 160
    mu = rng.uniform(-1, 1, (npr, 3))
    s = np.exp(rng.uniform(np.log(0.1), np.log(0.5), (npr, 3)))
    q = rng.standard_normal((npr, 4))
    eye = np.array([0.3, -3.0, 0.4])
    tgt = rng.uniform(-1, 1, (nr, 3))
    d = tgt - eye
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = np.broadcast_to(eye, d.shape)
    isx = oracle.intersect(t64(o), t64(d), t64(mu), t64(s), t64(q))
    h = 2e-4
    ts = np.arange(0.0, 6.0, h)
    checked = 0
    for p in range(npr):
        L = lam(s[p], q[p])
        for r in range(nr):
            x = o[r][None, :] + ts[:, None] * d[r][None, :] - mu[p][None, :]
            inside = np.einsum("ti,ij,tj->t", x, L, x) <= 1.0
            hit = bool(isx["hit"][r, p])
            if inside.sum() >= 3:
                assert hit
                t_in, t_out = ts[inside][0], ts[inside][-1]
                assert abs(t_in - float(isx["ta"][r, p])) <= h
                assert abs(t_out - float(isx["tb"][r, p])) <= h
                checked += 1
            elif inside.sum() == 0 and float(isx["g"][r, p]) < -1e-3:
                assert not hit
    assert checked > 30


# ------------------------------------------------------------------ network --

def test_mlp_matches_numpy_chain():
    rng = np.random.default_rng(5)
    m = oracle.Model(pe_freqs=6, hidden_width=64, hidden_layers=3, out_dim=20)
    th = rng.standard_normal(m.num_params)
    x = rng.standard_normal((37, m.in_dim))
    h = x
    off = 0
    dims = m.layer_dims()
    for li, (fi, fo) in enumerate(dims):
        w = th[off:off + fi * fo].reshape(fo, fi)
        b = th[off + fi * fo:off + fi * fo + fo]
        off += fi * fo + fo
        h = np.einsum("oi,ni->no", w, h) + b
        if li < len(dims) - 1:
            h = np.maximum(h, 0)
    got = oracle.mlp_apply(t64(th), t64(x), m).numpy()
    np.testing.assert_allclose(got, h, rtol=1e-12, atol=1e-12)


def test_encoding_closed_forms():
    p = t64([[0.5, 0.25, -1.0]])
    g = oracle.encode(p, 3).numpy()[0]
    assert g.shape == (3 + 18,)
    np.testing.assert_allclose(g[:3], [0.5, 0.25, -1.0])
    # level 0: sin(pi p), cos(pi p)
    np.testing.assert_allclose(g[3:6], [1.0, math.sqrt(0.5), 0.0], atol=1e-15)
    np.testing.assert_allclose(g[6:9], [0.0, math.sqrt(0.5), -1.0], atol=1e-15)
    # level 1: sin(2 pi p), cos(2 pi p)
    np.testing.assert_allclose(g[9:12], [0.0, 1.0, 0.0], atol=1e-15)
    np.testing.assert_allclose(g[12:15], [-1.0, 0.0, 1.0], atol=1e-15)
    # doubling identities between consecutive levels on random points
    rng = np.random.default_rng(6)
    pr = rng.uniform(-1, 1, (100, 3))
    ge = oracle.encode(t64(pr), 5).numpy()
    for lv in range(4):
        s0, c0 = ge[:, 3 + 6 * lv:6 + 6 * lv], ge[:, 6 + 6 * lv:9 + 6 * lv]
        s1, c1 = ge[:, 9 + 6 * lv:12 + 6 * lv], ge[:, 12 + 6 * lv:15 + 6 * lv]
        np.testing.assert_allclose(s1, 2 * s0 * c0, atol=1e-13)
        np.testing.assert_allclose(c1, c0 ** 2 - s0 ** 2, atol=1e-13)


# -------------------------------------------------------------- compositing --

def _one_prim_scene(model, mu, s, q, rgb, sigma):
    return {"center": np.asarray([mu], np.float64), "scale": np.asarray([s], np.float64),
            "quat": np.asarray([q], np.float64), "mlp": const_params(model, rgb, sigma)[None]}


@pytest.mark.parametrize("K", [1, 7, 32])
@pytest.mark.parametrize("jitter", [0, 1])
def test_constant_density_opacity_closed_form(K, jitter):
    """A constant-density primitive gives opacity 1 - exp(-sigma L) for any K."""
    rng = np.random.default_rng(7)
    mu, s, q = [0.1, -0.2, 0.3], [0.3, 0.15, 0.4], rng.standard_normal(4)
    sc = _one_prim_scene(SMALL, mu, s, q, [0.2, 0.5, 0.9], 3.7)
    eye = np.array([2.0, -2.5, 0.7])
    tg = np.asarray(mu) + rng.uniform(-0.2, 0.2, (40, 3))
    d = tg - eye
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = np.broadcast_to(eye, d.shape)
    out = render_np(sc, o, d, SMALL, oracle.Opts(samples_fixed=K, jitter=jitter, jitter_seed=3))
    for r in range(len(d)):
        roots = chord(o[r], d[r], mu, s, q)
        if roots is None or roots[1] <= 0:
            np.testing.assert_allclose(out["rgb"][r].numpy(), 0.0)
            continue
        L = roots[1] - max(roots[0], 0.0)
        a = 1 - math.exp(-3.7 * L)
        np.testing.assert_allclose(out["rgb"][r].numpy(), a * np.array([0.2, 0.5, 0.9]), rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(float(out["trans"][r]), 1 - a, rtol=1e-12)


def test_two_disjoint_constant_primitives_compose_in_depth_order():
    m = SMALL
    c1, c2 = np.array([0.9, 0.1, 0.2]), np.array([0.1, 0.8, 0.3])
    th = np.stack([const_params(m, c1, 2.0), const_params(m, c2, 5.0)])
    # primitive 1 is listed second but lies in front of primitive 0
    sc = {"center": np.array([[0.0, 1.0, 0.0], [0.0, -1.0, 0.0]]),
          "scale": np.array([[0.3, 0.3, 0.3], [0.2, 0.2, 0.2]]),
          "quat": np.array([[1.0, 0, 0, 0], [0.7, 0.1, 0.2, 0.3]]), "mlp": th[::-1].copy()}
    o = np.array([[0.0, -4.0, 0.0]])
    d = np.array([[0.0, 1.0, 0.0]])
    out = render_np(sc, o, d, m, oracle.Opts(samples_fixed=5, jitter=1))
    # front: primitive 1 (radius 0.2) carries th[0] = (c1, sigma 2);
    # back: primitive 0 (radius 0.3) carries th[1] = (c2, sigma 5)
    a_front = 1 - math.exp(-2.0 * 0.4)
    a_back = 1 - math.exp(-5.0 * 0.6)
    want = a_front * c1 + (1 - a_front) * a_back * c2
    np.testing.assert_allclose(out["rgb"][0].numpy(), want, rtol=1e-12)
    assert list(out["prim"]) == [1, 0]


def test_misses_give_background_and_unit_transmittance():
    sc = synth.make_scene(synth.CONFIGS[0])
    m = oracle.Model(4, 32, 2, 4)
    o = np.array([[0.0, 0.0, 3.0], [3.0, 0.0, 0.0]])
    d = np.array([[0.0, 0.0, 1.0], [1.0, 0.0, 0.0]])     # pointing away from the scene
    out = render_np(sc, o, d, m, oracle.Opts(samples_fixed=8, background=(0.25, 0.5, 0.75)))
    np.testing.assert_allclose(out["rgb"].numpy(), [[0.25, 0.5, 0.75]] * 2)
    np.testing.assert_allclose(out["trans"].numpy(), 1.0)


def _frame(ci, res=32):
    cfg = synth.CONFIGS[ci]
    sc = synth.make_scene(cfg)
    rng = np.random.default_rng(1000 * ci + 1)
    cam = synth.make_camera(rng, res, res, cfg.camera_radius)
    o, d, _ = synth.camera_rays(cam)
    m = oracle.Model(cfg.pe_freqs, cfg.hidden_width, cfg.hidden_layers, cfg.out_dim)
    return cfg, sc, o.astype(np.float64), d.astype(np.float64), m


def test_white_primitives_give_rgb_equal_one_minus_T():
    """With every colour 1 the pixel equals sum of weights = 1 - T (Sec. 3.3)."""
    cfg, sc, o, d, m = _frame(0)
    rng = np.random.default_rng(9)
    th = np.stack([const_params(m, [1 - 1e-15] * 3, s) for s in rng.uniform(0.5, 8, cfg.num_prims)])
    sc = dict(sc, mlp=th)
    out = render_np(sc, o, d, m, oracle.Opts(samples_fixed=16))
    rgb, tr = out["rgb"].numpy(), out["trans"].numpy()
    assert np.all((tr >= 0) & (tr <= 1))
    np.testing.assert_allclose(rgb, np.repeat(1 - tr[:, None], 3, 1), atol=1e-12)


def test_transmittance_monotone_and_weights_bounded():
    cfg, sc, o, d, m = _frame(1, 48)
    out = render_np(sc, o, d, m, oracle.Opts(samples_fixed=16, jitter=1), keep_samples=True)
    smp = out["samples"]
    tau = smp["tau"].numpy()
    assert np.all(tau >= 0)
    ray = smp["ray"]
    for r in np.unique(ray)[:200]:
        t = np.exp(-np.cumsum(tau[ray == r]))
        assert np.all(np.diff(t) <= 1e-15) and np.all((t >= 0) & (t <= 1))
    assert np.all(out["rgb"].numpy() <= 1 + 1e-12) and np.all(out["rgb"].numpy() >= 0)


def test_relabeling_primitives_leaves_image_unchanged():
    cfg, sc, o, d, m = _frame(1, 40)
    opts = oracle.Opts(samples_fixed=16, jitter=1, jitter_seed=11, t_stop=1e-4)
    a = render_np(sc, o, d, m, opts)
    perm = np.random.default_rng(10).permutation(cfg.num_prims)
    sc2 = {k: np.asarray(v)[perm] for k, v in sc.items()}
    b = render_np(sc2, o, d, m, opts)
    np.testing.assert_allclose(a["rgb"].numpy(), b["rgb"].numpy(), atol=1e-13)
    np.testing.assert_array_equal(perm[b["prim"]], a["prim"])


def test_rigid_motion_of_scene_and_camera_leaves_image_unchanged():
    cfg, sc, o, d, m = _frame(0, 32)
    rot = Rotation.from_euler("xyz", [0.3, -1.1, 2.0])
    tr = np.array([0.4, -0.7, 1.3])
    qs = sc["quat"].astype(np.float64)
    qr = (rot * Rotation.from_quat(np.c_[qs[:, 1:], qs[:, :1]])).as_quat()
    sc2 = dict(sc, center=rot.apply(sc["center"].astype(np.float64)) + tr, quat=np.c_[qr[:, 3:], qr[:, :3]])
    opts = oracle.Opts(samples_fixed=32, jitter=1, jitter_seed=2)
    a = render_np(sc, o, d, m, opts)
    b = render_np(sc2, rot.apply(o) + tr, rot.apply(d), m, opts)
    np.testing.assert_allclose(a["rgb"].numpy(), b["rgb"].numpy(), atol=1e-11)


def test_samples_are_stratified_in_their_bins():
    cfg, sc, o, d, m = _frame(0, 32)
    out = render_np(sc, o, d, m, oracle.Opts(samples_fixed=32, jitter=1, jitter_seed=5), keep_samples=True)
    smp = out["samples"]
    h, k = smp["hit"], smp["k"]
    ta, tb = out["t_a"].numpy()[h], out["t_b"].numpy()[h]
    dl = (tb - ta) / 32
    t = smp["t"].numpy()
    assert np.all(t >= ta + k * dl - 1e-12) and np.all(t < ta + (k + 1) * dl + 1e-12)
    u = smp["u"]
    assert np.all((u >= 0) & (u < 1)) and np.all(u * 2 ** 24 == np.floor(u * 2 ** 24))
    hist = np.histogram(u, bins=16, range=(0, 1))[0]
    e = len(u) / 16
    assert ((hist - e) ** 2 / e).sum() < 60          # chi2(15) far tail


def _pcg_inverse(h):
    """Inverse of the PCG output permutation (Jarzynski and Olano, JCGT 2020),
    undone step by step from its published constants: the final xorshift by
    22 (its own inverse, as 2 x 22 >= 32), the odd multiplier 277803737 (its
    inverse modulo 2^32), the data-dependent xorshift (the top four bits are
    unchanged and give the shift back), the LCG step 747796405 v + 2891336453."""
    m = (1 << 32) - 1
    out = []
    for x in (int(v) for v in np.asarray(h, np.uint32)):
        word = x ^ (x >> 22)
        y = (word * pow(277803737, -1, 1 << 32)) & m
        sh = (y >> 28) + 4
        state, t = y, y >> sh
        while t:
            state ^= t
            t >>= sh
        out.append(((state - 2891336453) * pow(747796405, -1, 1 << 32)) & m)
    return np.array(out, np.uint64)


def test_pcg_hash_is_the_published_permutation():
    """The sample-offset hash is a bijection of the 32-bit integers: it is
    undone by the inverse of each published step, it maps 2^20 distinct
    inputs to distinct outputs (a random function would collide about 128
    times), and one flipped input bit changes about half the output bits."""
    from oracle.pcg import pcg_hash
    rng = np.random.default_rng(11)
    v = rng.integers(0, 1 << 32, 4096, dtype=np.uint64).astype(np.uint32)
    v[:4] = [0, 1, 0xFFFFFFFF, 0x80000000]
    np.testing.assert_array_equal(_pcg_inverse(pcg_hash(v)), v.astype(np.uint64))
    h = pcg_hash(np.arange(1 << 20, dtype=np.uint32))
    assert len(np.unique(h)) == 1 << 20
    flips = [np.unpackbits((pcg_hash(v) ^ pcg_hash(v ^ np.uint32(1 << b))).view(np.uint8)).sum() / len(v)
             for b in range(32)]
    assert 15.0 < min(flips) and max(flips) < 17.0


def test_early_termination_stops_after_first_sample_below_threshold():
    m = SMALL
    nprim = 12
    th = np.stack([const_params(m, [0.5, 0.5, 0.5], 40.0) for _ in range(nprim)])
    sc = {"center": np.c_[np.zeros(nprim), np.linspace(-1.5, 1.5, nprim), np.zeros(nprim)],
          "scale": np.full((nprim, 3), 0.1), "quat": np.tile([1.0, 0, 0, 0], (nprim, 1)), "mlp": th}
    o = np.array([[0.0, -4.0, 0.0]])
    d = np.array([[0.0, 1.0, 0.0]])
    full = render_np(sc, o, d, m, oracle.Opts(samples_fixed=10, jitter=0))
    cut = render_np(sc, o, d, m, oracle.Opts(samples_fixed=10, jitter=0, t_stop=1e-4))
    tau = 40.0 * 0.2 / 10
    n_exp = int(math.floor(-math.log(1e-4) / tau)) + 1    # first sample with T_after < 1e-4
    assert int(cut["n_used"][0]) == n_exp
    assert math.exp(-(n_exp - 1) * tau) >= 1e-4 > math.exp(-n_exp * tau)
    assert abs(float(cut["trans"][0]) - math.exp(-n_exp * tau)) < 1e-15
    assert np.all(np.abs(cut["rgb"].numpy() - full["rgb"].numpy()) < 1e-4)


def _numpy_field(sc, model, x, p):
    """Independent density/colour of primitive p at world points x (numpy)."""
    r = scipy_rot(np.asarray(sc["quat"][p], np.float64))
    loc = (x - np.asarray(sc["center"][p], np.float64)) @ r / np.asarray(sc["scale"][p], np.float64)
    feats = [loc]
    for lv in range(model.pe_freqs):
        feats += [np.sin(2 ** lv * np.pi * loc), np.cos(2 ** lv * np.pi * loc)]
    h = np.concatenate(feats, 1)
    th = np.asarray(sc["mlp"][p], np.float64)
    off = 0
    dims = model.layer_dims()
    for li, (fi, fo) in enumerate(dims):
        w = th[off:off + fi * fo].reshape(fo, fi)
        b = th[off + fi * fo:off + fi * fo + fo]
        off += fi * fo + fo
        h = h @ w.T + b
        if li < len(dims) - 1:
            h = np.maximum(h, 0)
    return 1 / (1 + np.exp(-h[:, :3])), np.logaddexp(0, h[:, 3])


def test_converges_to_dense_marching_on_disjoint_supports():
    """At large K the oracle agrees with fine uniform marching of the summed
    field sum_i 1[x in E_i] sigma_i(x) (the continuous operator of the
    rendering definition; the discrete form converges as the step shrinks)."""
    m = oracle.Model(pe_freqs=2, hidden_width=16, hidden_layers=2, out_dim=4)
    rng = np.random.default_rng(12)
    th = rng.uniform(-0.6, 0.6, (2, m.num_params))
    sc = {"center": np.array([[0.0, -0.6, 0.0], [0.1, 0.6, 0.05]]),
          "scale": np.array([[0.35, 0.25, 0.3], [0.3, 0.4, 0.2]]),
          "quat": rng.standard_normal((2, 4)), "mlp": th}
    eye = np.array([0.05, -4.0, 0.02])
    tg = np.c_[rng.uniform(-0.15, 0.15, 12), np.zeros(12), rng.uniform(-0.1, 0.1, 12)]
    d = tg - eye
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = np.broadcast_to(eye, d.shape)
    out = render_np(sc, o, d, m, oracle.Opts(samples_fixed=2048, jitter=0))
    h = 2.5e-5
    ts = np.arange(0.0, 6.0, h) + 0.5 * h
    for r in range(len(d)):
        x = o[r][None] + ts[:, None] * d[r][None]
        sig = np.zeros(len(ts))
        col = np.zeros((len(ts), 3))
        for p in range(2):
            rel = x - sc["center"][p]
            L = lam(sc["scale"][p], sc["quat"][p])
            inside = np.einsum("ti,ij,tj->t", rel, L, rel) <= 1
            if inside.any():
                c, s = _numpy_field(sc, m, x[inside], p)
                sig[inside] += s
                col[inside] = c
        tau = sig * h
        t_before = np.exp(-np.concatenate([[0.0], np.cumsum(tau)[:-1]]))
        ref = ((t_before * (1 - np.exp(-tau)))[:, None] * col).sum(0)
        np.testing.assert_allclose(out["rgb"][r].numpy(), ref, atol=2e-3)


def test_discrete_stability_bound_for_perturbed_samples():
    """|dC| <= max|dc| + 2 max|c| sum|dtau| (discrete form of the rendering
    operator's stability lemma), checked on a perturbed network."""
    cfg, sc, o, d, m = _frame(1, 32)
    opts = oracle.Opts(samples_fixed=16, jitter=1)
    a = render_np(sc, o, d, m, opts, keep_samples=True)
    rng = np.random.default_rng(13)
    sc2 = dict(sc, mlp=sc["mlp"] + 1e-3 * rng.standard_normal(sc["mlp"].shape).astype(np.float32))
    b = render_np(sc2, o, d, m, opts, keep_samples=True)
    sa, sb = a["samples"], b["samples"]
    dc = np.abs(sa["c"].numpy() - sb["c"].numpy()).max(1)
    dt = np.abs(sa["tau"].numpy() - sb["tau"].numpy())
    for r in np.unique(sa["ray"]):
        sel = sa["ray"] == r
        bound = dc[sel].max() + 2 * dt[sel].sum()
        assert np.abs(a["rgb"][r].numpy() - b["rgb"][r].numpy()).max() <= bound + 1e-15


# ---------------------------------------------------------------- gradients --

def _grad_case():
    cfg = synth.CONFIGS[0]
    sc = synth.make_scene(cfg)
    keep = [0, 3, 5]
    sc = {k: np.asarray(v, np.float64)[keep] for k, v in sc.items()}
    sc["mlp"] *= 1.3
    rng = np.random.default_rng(1)
    cam = synth.make_camera(rng, 24, 24, 3.0)
    o, d, _ = synth.camera_rays(cam)
    m = oracle.Model(cfg.pe_freqs, cfg.hidden_width, cfg.hidden_layers, cfg.out_dim)
    opts = oracle.Opts(samples_fixed=8, jitter=1, jitter_seed=4, t_stop=1e-3)
    w = np.random.default_rng(2).standard_normal((len(o), 3))
    return sc, o.astype(np.float64), d.astype(np.float64), m, opts, w


def test_autograd_matches_complex_step():
    sc, o, d, m, opts, w = _grad_case()
    _, _, _, g, _ = oracle.loss_and_grads(sc, o, d, m, opts, grad_rgb=w)
    rng = np.random.default_rng(3)
    picks = [("center", (i, j)) for i in range(3) for j in range(3)]
    picks += [("scale", (i, j)) for i in range(3) for j in range(3)]
    picks += [("quat", (i, j)) for i in range(3) for j in range(4)]
    picks += [("mlp", (i, int(j))) for i in range(3) for j in rng.choice(m.num_params, 8, replace=False)]
    nz = 0
    for key, idx in picks:
        cs = oracle.complex_step(sc, o, d, m, opts, key, idx, w)
        ad = float(g[key][idx])
        assert abs(cs - ad) <= 1e-9 * max(1.0, abs(cs)), (key, idx, cs, ad)
        nz += abs(cs) > 1e-8
    assert nz > 30


def test_central_differences_agree_with_autograd():
    # without the termination cut, so that the step does not move a discrete
    # decision (complex step above covers the cut)
    sc, o, d, m, opts, w = _grad_case()
    opts = oracle.Opts(samples_fixed=opts.samples_fixed, jitter=1, jitter_seed=4)
    _, _, _, g, _ = oracle.loss_and_grads(sc, o, d, m, opts, grad_rgb=w)
    def L(s2):
        out = render_np(s2, o, d, m, opts)
        return float((out["rgb"].numpy() * w).sum())
    for key, idx in [("center", (0, 1)), ("scale", (1, 2)), ("quat", (2, 0)), ("mlp", (0, 5)),
                     ("mlp", (1, 1500)), ("mlp", (2, m.num_params - 1))]:
        h = 1e-7      # a near-grazing ray makes the truncation term large at 1e-6
        sp = {k: v.copy() for k, v in sc.items()}
        sm = {k: v.copy() for k, v in sc.items()}
        sp[key][idx] += h
        sm[key][idx] -= h
        fd = (L(sp) - L(sm)) / (2 * h)
        assert abs(fd - g[key][idx]) <= 1e-5 * max(1.0, abs(fd)), (key, idx, fd, g[key][idx])


def test_quaternion_gradient_is_orthogonal_to_q_and_missed_primitive_gets_zero():
    sc, o, d, m, opts, w = _grad_case()
    sc["center"][2] = [40.0, 40.0, 40.0]          # out of every ray's reach
    _, _, _, g, _ = oracle.loss_and_grads(sc, o, d, m, opts, grad_rgb=w)
    for i in range(3):
        assert abs(g["quat"][i] @ sc["quat"][i]) < 1e-12 * max(1, np.abs(g["quat"][i]).max())
    for k in ("center", "scale", "quat", "mlp"):
        assert np.all(g[k][2] == 0)
    assert np.abs(g["mlp"][0]).max() > 0


def test_relu_noise_matches_monte_carlo_rounding_model():
    """Perturb every product and bias of the forward pass by an independent
    relative N(0, u^2) error and compare the spread of the hidden
    pre-activations with u e of relu_noise (two hidden layers, where the
    model is exact to first order)."""
    rng = np.random.default_rng(11)
    model = oracle.Model(pe_freqs=2, hidden_width=32, hidden_layers=2, out_dim=4)
    theta = rng.standard_normal(model.num_params) * 0.4
    x = rng.standard_normal((3, model.in_dim))
    ref = oracle.relu_noise(theta, x, model)
    u, trials = 1e-7, 4000
    dims = model.layer_dims()
    ws, off = [], 0
    for fi, fo in dims[:-1]:
        w = theta[off:off + fi * fo].reshape(fo, fi)
        off += fi * fo
        ws.append((w, theta[off:off + fo]))
        off += fo
    for row in range(x.shape[0]):
        zs = [[] for _ in ws]
        for _ in range(trials):
            h = x[row]
            for li, (w, b) in enumerate(ws):
                prod = w * h[None, :] * (1 + u * rng.standard_normal(w.shape))
                z = prod.sum(1) + b * (1 + u * rng.standard_normal(b.shape))
                zs[li].append(z)
                h = np.maximum(z, 0)
        for li in range(len(ws)):
            z_ref, e_ref = ref[li][0][row], ref[li][1][row]
            std = np.std(np.array(zs[li]), axis=0)
            # units far from their switching point (noise model linear there)
            far = np.abs(z_ref) > 1e3 * u * e_ref
            ratio = std[far] / (u * e_ref[far])
            assert np.all(np.abs(ratio - 1) < 0.08), (row, li, ratio.min(), ratio.max())


def test_relu_margin_is_the_smallest_noise_scaled_distance():
    rng = np.random.default_rng(12)
    model = oracle.Model(pe_freqs=2, hidden_width=32, hidden_layers=3, out_dim=4)
    theta = rng.standard_normal(model.num_params) * 0.3
    x = rng.standard_normal((50, model.in_dim))
    m = oracle.relu_margin(theta, x, model)
    per = np.stack([(np.abs(z) / e).min(1) for z, e in oracle.relu_noise(theta, x, model)], 1)
    np.testing.assert_array_equal(m, per.min(1))
    # the noise scale is invariant to relabelling the hidden units of a layer
    fi, fo = model.layer_dims()[0]
    perm = rng.permutation(fo)
    th = theta.copy()
    w0 = th[:fi * fo].reshape(fo, fi)[perm]
    b0 = th[fi * fo:fi * fo + fo][perm]
    th[:fi * fo] = w0.ravel()
    th[fi * fo:fi * fo + fo] = b0
    f1, o1 = model.layer_dims()[1]
    s1 = fi * fo + fo
    th[s1:s1 + f1 * o1] = theta[s1:s1 + f1 * o1].reshape(o1, f1)[:, perm].ravel()
    np.testing.assert_allclose(oracle.relu_margin(th, x, model), m, rtol=1e-12)


def test_relu_margin_zero_for_a_unit_exactly_at_its_switching_point():
    rng = np.random.default_rng(13)
    model = oracle.Model(pe_freqs=2, hidden_width=32, hidden_layers=1, out_dim=4)
    fi, fo = model.layer_dims()[0]
    theta = rng.standard_normal(model.num_params)
    x = rng.standard_normal((64, model.in_dim))
    x[9] = rng.integers(-3, 4, model.in_dim)
    theta[:fi * fo] = rng.integers(-3, 4, fi * fo)
    w = theta[:fi * fo].reshape(fo, fi)
    theta[fi * fo + 5] = -(w[5] @ x[9])        # unit 5 of row 9 sits exactly at zero
    m = oracle.relu_margin(theta, x, model)
    assert m[9] == 0.0
    assert (np.delete(m, 9) > 0).all()


# -------------------------------------------------------------- tile order --

def _tilted(tan_t):
    c = 1.0 / math.sqrt(1.0 + tan_t * tan_t)
    return np.array([-tan_t * c, 0.0, c])


def _two_sphere_tile_case():
    """Spheres A at (0,0,5) and B at (0.1,0,5.02), radius 2, constant colours.
    Along +z A's contact depth is smaller (5 < 5.02); along the ray e tilted
    by atan 0.3 towards -x it is B's (t_B - t_A = -0.1 sin + 0.02 cos < 0).
    Packet 0: 64 copies of e; packet 1: 63 rays along +z and e at lane 5;
    packet 2 (ragged, 11 rays): e first, then +z rays."""
    m = SMALL
    ca, cb = np.array([0.9, 0.2, 0.1]), np.array([0.1, 0.3, 0.8])
    sa, sb = 0.7, 1.3
    sc = {"center": np.array([[0.0, 0.0, 5.0], [0.1, 0.0, 5.02]]),
          "scale": np.full((2, 3), 2.0), "quat": np.array([[1.0, 0, 0, 0], [1.0, 0, 0, 0]]),
          "mlp": np.stack([const_params(m, ca, sa), const_params(m, cb, sb)])}
    e, z = _tilted(0.3), np.array([0.0, 0.0, 1.0])
    d = np.concatenate([np.tile(e, (64, 1)), np.tile(z, (64, 1)), np.tile(z, (11, 1))])
    d[64 + 5] = e
    d[128] = e
    o = np.zeros_like(d)
    return sc, o, d, (ca, sa), (cb, sb)


def test_packet_centres_are_mean_origin_and_normalised_direction_sum():
    sc, o, d, _, _ = _two_sphere_tile_case()
    o = o + np.arange(len(o))[:, None] * np.array([0.01, -0.02, 0.03])
    oc, dc = oracle.packet_centres(o, d)
    for s, e in [(0, 64), (64, 128), (128, len(o))]:
        v = d[s:e].sum(0)
        np.testing.assert_allclose(dc[s:e], np.broadcast_to(v / np.linalg.norm(v), (e - s, 3)), rtol=1e-15)
        np.testing.assert_allclose(oc[s:e], np.broadcast_to(o[s:e].mean(0), (e - s, 3)), rtol=1e-15)
    np.testing.assert_allclose(dc[0], _tilted(0.3), rtol=1e-15)


def test_tile_order_composites_in_the_virtual_rays_depth_order():
    """Closed form: a ray meeting constant primitives X then Y gives
    alpha_X c_X + (1 - alpha_X) alpha_Y c_Y with alpha = 1 - exp(-sigma L)."""
    sc, o, d, (ca, sa), (cb, sb) = _two_sphere_tile_case()
    exact = render_np(sc, o, d, SMALL, oracle.Opts(samples_fixed=6, jitter=1, order=0))
    tile = render_np(sc, o, d, SMALL, oracle.Opts(samples_fixed=6, jitter=1, order=1))

    def alpha(i, r, sigma):
        roots = chord(o[r], d[r], sc["center"][i], sc["scale"][i], sc["quat"][i])
        return 1 - math.exp(-sigma * (roots[1] - max(roots[0], 0.0)))

    def prims(out, r):
        return list(out["prim"][out["ray_off"][r]:out["ray_off"][r + 1]])

    for r in range(len(d)):
        tilted = np.allclose(d[r], _tilted(0.3))
        aa, ab = alpha(0, r, sa), alpha(1, r, sb)
        a_first = aa * ca + (1 - aa) * ab * cb
        b_first = ab * cb + (1 - ab) * aa * ca
        # exact order follows the ray itself
        assert prims(exact, r) == ([1, 0] if tilted else [0, 1])
        np.testing.assert_allclose(exact["rgb"][r].numpy(), b_first if tilted else a_first, rtol=1e-12)
        # tile order: packet 0's virtual ray is the tilted one, the others' are near +z
        b_in_front = r < 64
        assert prims(tile, r) == ([1, 0] if b_in_front else [0, 1])
        np.testing.assert_allclose(tile["rgb"][r].numpy(), b_first if b_in_front else a_first, rtol=1e-12)
        # hit sets, chords and transmittance do not depend on the order
        np.testing.assert_allclose(float(tile["trans"][r]), float(exact["trans"][r]), rtol=1e-12)


def test_tile_order_equals_exact_order_when_a_packets_rays_coincide():
    cfg = synth.CONFIGS[0]
    sc = synth.make_scene(cfg)
    rng = np.random.default_rng(3)
    cam = synth.make_camera(rng, 64, 64, cfg.camera_radius, cfg.fov_deg)
    o, d, _ = synth.camera_rays(cam)
    m = oracle.Model(cfg.pe_freqs, cfg.hidden_width, cfg.hidden_layers, cfg.out_dim)
    opts = dict(samples_fixed=cfg.samples_fixed, jitter=1, jitter_seed=9)
    full = render_np(sc, o, d, m, oracle.Opts(order=0, **opts))
    multi = np.nonzero(np.diff(full["ray_off"]) >= 2)[0]
    assert len(multi) >= 8
    n = 64 * 7 + 13                       # ragged last packet
    pick = np.repeat(multi[:: max(1, len(multi) // 8)][:8], 64)[:n]
    o, d = o[pick], d[pick]
    a = render_np(sc, o, d, m, oracle.Opts(order=0, **opts))
    b = render_np(sc, o, d, m, oracle.Opts(order=1, **opts))
    assert int(a["ray_off"][-1]) > n // 4
    assert np.array_equal(a["prim"], b["prim"]) and np.array_equal(a["ray_off"], b["ray_off"])
    np.testing.assert_array_equal(a["rgb"].numpy(), b["rgb"].numpy())


def test_tile_order_keeps_every_rays_hit_set_and_sample_positions():
    cfg = synth.CONFIGS[0]
    sc = synth.make_scene(cfg)
    cam = synth.make_camera(np.random.default_rng(4), 64, 64, cfg.camera_radius, cfg.fov_deg)
    o, d, _ = synth.camera_rays(cam)
    m = oracle.Model(cfg.pe_freqs, cfg.hidden_width, cfg.hidden_layers, cfg.out_dim)
    opts = dict(samples_fixed=cfg.samples_fixed, jitter=0)
    a = render_np(sc, o, d, m, oracle.Opts(order=0, **opts))
    b = render_np(sc, o, d, m, oracle.Opts(order=1, **opts))
    assert np.array_equal(a["ray_off"], b["ray_off"])
    moved = 0
    for r in range(len(o)):
        s, e = a["ray_off"][r], a["ray_off"][r + 1]
        pa, pb = a["prim"][s:e], b["prim"][s:e]
        assert sorted(pa) == sorted(pb)
        # same chord per (ray, primitive) whatever its rank
        ta = dict(zip(pa, a["t_a"][s:e].numpy()))
        tb = dict(zip(pb, b["t_a"][s:e].numpy()))
        assert all(ta[p] == tb[p] for p in pa)
        if e - s <= 1:
            np.testing.assert_array_equal(a["rgb"][r].numpy(), b["rgb"][r].numpy())
        moved += int(not np.array_equal(pa, pb))
    # the packets are camera tiles: the orders differ on few rays only
    assert moved <= 0.05 * len(o)


# ----------------------------------------------------------- slot features --

def _ray_to_local_foot(mu, s, q, foot_local, d_local, back=6.0):
    """World ray whose closest approach to the primitive, measured in its
    scale-normalised frame, is the local point ``foot_local`` (d_local must be
    orthogonal to it): the local line foot + t d_local mapped to the world."""
    r = scipy_rot(q)
    to_world = r @ np.diag(s)
    x = np.asarray(mu) + to_world @ np.asarray(foot_local)
    d = to_world @ np.asarray(d_local)
    d /= np.linalg.norm(d)
    return x - back * d, d


def test_equal_slots_give_opacity_times_embedding():
    rng = np.random.default_rng(21)
    mu, s, q = [0.1, -0.2, 0.3], [0.3, 0.15, 0.4], rng.standard_normal(4)
    sc = _one_prim_scene(SMALL, mu, s, q, [0.2, 0.5, 0.9], 3.7)
    e = rng.standard_normal(5)
    sc["slots"] = np.tile(e, (1, 4, 1))
    eye = np.array([2.0, -2.5, 0.7])
    d = np.asarray(mu) + rng.uniform(-0.2, 0.2, (30, 3)) - eye
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = np.broadcast_to(eye, d.shape)
    p = oracle.to_tensors(sc)
    out = oracle.render(p["center"], p["scale"], p["quat"], p["mlp"], t64(o), t64(d), SMALL,
                        oracle.Opts(samples_fixed=7, jitter=1, jitter_seed=2), slots=p["slots"])
    for r in range(len(d)):
        roots = chord(o[r], d[r], mu, s, q)
        a = 0.0 if roots is None or roots[1] <= 0 else 1 - math.exp(-3.7 * (roots[1] - max(roots[0], 0.0)))
        np.testing.assert_allclose(out["slot_feat"][r].numpy(), a * e, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("k", [0, 2])
def test_slot_gates_closed_form_at_a_tetrahedral_offset(k):
    """A contact offset u = r a_k gives g_k = e^r / (e^r + 3 e^(-r/3)) (the
    frame's directions meet at a . a' = -1/3), the rest equal; one-hot slot
    embeddings make the feature the gate vector times the hit's opacity."""
    rng = np.random.default_rng(22)
    mu, s, q = [0.3, 0.1, -0.2], [0.5, 0.2, 0.35], rng.standard_normal(4)
    sigma, rr = 2.5, 0.6
    sc = _one_prim_scene(SMALL, mu, s, q, [0.5, 0.5, 0.5], sigma)
    sc["slots"] = np.eye(4)[None].copy()
    a = oracle.TETRA[k]
    d_loc = np.cross(a, [0.3, -0.5, 0.8])
    d_loc /= np.linalg.norm(d_loc)
    o, d = _ray_to_local_foot(mu, s, q, -rr * a, d_loc)
    out = render_np(sc, o[None], d[None], SMALL, oracle.Opts(samples_fixed=9, jitter=0), slots=t64(sc["slots"]))
    out_f = out["slot_feat"][0].numpy()
    roots = chord(o, d, mu, s, q)
    alpha = 1 - math.exp(-sigma * (roots[1] - roots[0]))
    gk = math.exp(rr) / (math.exp(rr) + 3 * math.exp(-rr / 3))
    want = np.full(4, (1 - gk) / 3)
    want[k] = gk
    np.testing.assert_allclose(out_f, alpha * want, rtol=1e-10)


def _slot_scene(m):
    c1, c2 = np.array([0.9, 0.1, 0.2]), np.array([0.1, 0.8, 0.3])
    return {"center": np.array([[0.0, 1.0, 0.0], [0.0, -1.0, 0.0]]),
            "scale": np.array([[0.3, 0.3, 0.3], [0.2, 0.2, 0.2]]),
            "quat": np.array([[1.0, 0, 0, 0], [0.7, 0.1, 0.2, 0.3]]),
            "mlp": np.stack([const_params(m, c2, 5.0), const_params(m, c1, 2.0)])}


def test_slot_features_of_two_disjoint_primitives_compose_in_depth_order():
    m = SMALL
    sc = _slot_scene(m)
    rng = np.random.default_rng(23)
    e0, e1 = rng.standard_normal(6), rng.standard_normal(6)
    sc["slots"] = np.stack([np.tile(e0, (4, 1)), np.tile(e1, (4, 1))])
    o = np.array([[0.0, -4.0, 0.0]])
    d = np.array([[0.0, 1.0, 0.0]])
    out = render_np(sc, o, d, m, oracle.Opts(samples_fixed=5, jitter=1), slots=t64(sc["slots"]))
    a_front = 1 - math.exp(-2.0 * 0.4)      # primitive 1 (radius 0.2, sigma 2) is in front
    a_back = 1 - math.exp(-5.0 * 0.6)
    np.testing.assert_allclose(out["slot_feat"][0].numpy(), a_front * e1 + (1 - a_front) * a_back * e0,
                               rtol=1e-12)


def test_slot_feature_gradients_match_central_differences():
    cfg = synth.CONFIGS[0]
    m = oracle.Model(cfg.pe_freqs, cfg.hidden_width, cfg.hidden_layers, cfg.out_dim)
    sc = {k: v.astype(np.float64) for k, v in synth.make_scene(cfg).items()}
    rng = np.random.default_rng(24)
    sc["slots"] = rng.standard_normal((cfg.num_prims, 4, 5))
    cam = synth.make_camera(np.random.default_rng(5), 24, 24, cfg.camera_radius, cfg.fov_deg)
    o, d, _ = synth.camera_rays(cam)
    o, d = o.astype(np.float64), d.astype(np.float64)
    gs = rng.standard_normal((len(o), 5))
    # no termination cut, so that a step does not move a discrete decision
    opts = oracle.Opts(samples_fixed=8, jitter=1, jitter_seed=4)
    _, _, _, grads, _ = oracle.loss_and_grads(sc, o, d, m, opts, grad_rgb=np.zeros((len(o), 3)), grad_slot=gs)

    def loss(scn):
        p = oracle.to_tensors(scn)
        out = oracle.render(p["center"], p["scale"], p["quat"], p["mlp"], t64(o), t64(d), m, opts,
                            slots=p["slots"])
        return float((out["slot_feat"].numpy() * gs).sum())

    checked = 0
    for key in ("center", "scale", "quat", "slots", "mlp"):
        flat = np.abs(grads[key]).reshape(-1)
        for idx in np.argsort(flat)[-2:]:
            # fourth-order central difference at a small step: near-grazing
            # hits and the encoding's high frequencies give the loss large
            # higher derivatives (the difference converges to the gradient as
            # the step shrinks: 1e-5 is off by 6e-4, 1e-7 by 1e-7)
            def at(step):
                sp = {k: v.copy() for k, v in sc.items()}
                sp[key].reshape(-1)[idx] += step
                return loss(sp)
            h = 1e-7
            fd = (8 * (at(h) - at(-h)) - (at(2 * h) - at(-2 * h))) / (12 * h)
            np.testing.assert_allclose(grads[key].reshape(-1)[idx], fd, rtol=1e-5, atol=1e-9)
            checked += 1
    assert checked == 10


# ---------------------------------------------------------------------------
# ReLU gates taken in the kernel's bfloat16 forms (oracle.gate_preacts)
# ---------------------------------------------------------------------------

class _Dims:
    """A network shape for the gate tests: layer_dims only."""

    def __init__(self, *dims):
        self.dims = dims

    def layer_dims(self):
        return [(self.dims[i], self.dims[i + 1]) for i in range(len(self.dims) - 1)]


def test_bf16_rounding_by_hand():
    # bfloat16 has 8 significant bits: the spacing above 1 is 2^-7
    vals = [1 + 2 ** -8,            # halfway between 1 and 1 + 2^-7: ties to the even 1
            1 + 3 * 2 ** -8,        # halfway between 1 + 2^-7 and 1 + 2^-6: ties to the even 1 + 2^-6
            1 + 2 ** -8 + 2 ** -20,  # just above halfway: up
            -(2 + 2 ** -6),         # exact (spacing 2^-6 above 2)
            3.0 * 2 ** -130,        # a subnormal with bits only above the low 16: kept
            2.0 ** -140]            # a subnormal whose bits all lie in the low 16: rounded to 0
    want = [1.0, 1 + 2 ** -6, 1 + 2 ** -7, -(2 + 2 ** -6), 3.0 * 2 ** -130, 0.0]
    got = oracle.bf16_round(np.array(vals))
    np.testing.assert_array_equal(got, want)
    # and the library's own conversion agrees on random float32 values
    x = np.random.default_rng(4).standard_normal(5000).astype(np.float32) * 10.0 ** np.random.default_rng(5).integers(-6, 6, 5000)
    np.testing.assert_array_equal(oracle.bf16_round(x), torch.from_numpy(x).bfloat16().double().numpy())


def test_split_pairs_carry_sixteen_bits():
    x = np.random.default_rng(6).standard_normal(5000).astype(np.float32).astype(np.float64)
    hi, lo = oracle.split_bf16(x)
    assert np.all(np.abs(hi + lo - x) <= 2.0 ** -16 * np.abs(x))
    # a value with at most 16 significant bits is carried exactly
    y = np.array([1 + 2 ** -9 + 2 ** -15, -3.0 * (1 + 2 ** -12)])
    hi, lo = oracle.split_bf16(y)
    np.testing.assert_array_equal(hi + lo, y)


def test_gate_taken_in_the_kernel_form_by_hand():
    """w = 1 + 2^-9 + 2^-20 splits to (1, 2^-9) and rounds to 1; with x = 1 and
    first-layer bias -(1 + 2^-9) (split (-1, -2^-9), rounded -1) the FP64
    pre-activation is 2^-20 > 0 but both bfloat16 forms see exactly 0: the gate
    is closed there, open in FP64."""
    m = _Dims(1, 1, 1)
    w0, b0, w1, b1 = 1 + 2 ** -9 + 2 ** -20, -(1 + 2 ** -9), 1.0, 0.0
    theta = torch.tensor([w0, b0, w1, b1], dtype=torch.float64)
    x = torch.ones((1, 1), dtype=torch.float64)
    for form in ("bf16", "bf16x3"):
        z, = oracle.gate_preacts(theta, x, m, form)
        assert z[0, 0] == 0.0
    # the FP64 branch passes the 2^-20, the kernel-form branch nothing, and the
    # gradient follows the branch: d out / d w0 = w1 x on the open branch, 0 closed
    for form, val, gw in (("fp64", 2.0 ** -20, 1.0), ("bf16x3", 0.0, 0.0)):
        th = theta.clone().requires_grad_(True)
        out = oracle.mlp_apply(th, x, m, gate_form=form)
        assert float(out) == val
        out.sum().backward()
        assert float(th.grad[0]) == gw
    # a hidden layer's bias is a float32 value added as it is: z = 1 * 1 + b1
    m2 = _Dims(1, 1, 1, 1)
    b1 = -(1 + 2 ** -12)                       # not a bfloat16 value
    th2 = torch.tensor([1.0, 0.0, 1.0, b1, 1.0, 0.0], dtype=torch.float64)
    z0, z1 = oracle.gate_preacts(th2, x, m2, "bf16")
    assert z0[0, 0] == 1.0 and z1[0, 0] == -(2.0 ** -12)


def test_gates_match_fp64_away_from_zero_and_exactly_on_bf16_operands():
    rng = np.random.default_rng(8)
    m = _Dims(5, 16, 16, 4)
    n = sum(i * o + o for i, o in m.layer_dims())
    # operands that bfloat16 holds exactly (multiples of 2^-6 in [-2, 2]) and
    # sums exact in float64: the emulated pre-activations equal FP64's
    theta = rng.integers(-128, 129, n) / 64.0
    x = rng.integers(-128, 129, (50, 5)) / 64.0
    zs_fp = []
    h = x
    off = 0
    for li, (fi, fo) in enumerate(m.layer_dims()[:-1]):
        w = theta[off:off + fi * fo].reshape(fo, fi)
        off += fi * fo
        b = theta[off:off + fo]
        off += fo
        z = h @ w.T + b
        zs_fp.append(z)
        h = np.maximum(z, 0)
    # (layer 2 inputs are sums of products of such values: exact in bf16x3 pairs
    # only while they keep 16 significant bits, so compare the first layer exactly)
    for form in ("bf16", "bf16x3"):
        zs = oracle.gate_preacts(torch.from_numpy(theta), torch.from_numpy(x), m, form)
        np.testing.assert_array_equal(zs[0], zs_fp[0])
    # random operands: the split form's pre-activations stay within 2^-15 of the
    # scale sum |w||x| of FP64, so every gate farther than that agrees
    theta = rng.standard_normal(n) * 0.5
    x = rng.standard_normal((400, 5))
    zs = oracle.gate_preacts(torch.from_numpy(theta), torch.from_numpy(x), m, "bf16x3")
    w0 = theta[:80].reshape(16, 5)
    b0 = theta[80:96]
    z0 = x @ w0.T + b0
    scale = np.abs(x) @ np.abs(w0).T + np.abs(b0)
    assert np.all(np.abs(zs[0] - z0) <= 2.0 ** -15 * scale)
