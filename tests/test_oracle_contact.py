"""Pins of the contact-point primitive's oracle (oracle/contact.py) against
what the paper and the mathematics fix, independently of its own code:
line integrals by quadrature, hand-computed residuals and encodings,
closed-form compositing, the 3-sigma support boundary, Eq. 2's clamp, and
complex-step derivatives."""
import math

import numpy as np
import pytest
import torch
from scipy import integrate
from scipy.spatial.transform import Rotation

import oracle
from oracle.contact import KAPPA, ContactModel, contact_loss_and_grads, encode_vec, render_contact

MODEL = ContactModel()


def _lambda(scale, quat):
    """Lambda = R diag(s^-2) R^T with R from scipy (scalar-last quaternion)."""
    w, x, y, z = quat
    r = Rotation.from_quat([x, y, z, w]).as_matrix()
    return r @ np.diag(1.0 / np.asarray(scale) ** 2) @ r.T


def _const_mlp(rgb_raw, sigma_raw, model=MODEL):
    """A network whose output is constant: every weight zero, output biases set."""
    th = np.zeros(model.num_params)
    th[-4:-1] = rgb_raw
    th[-1] = sigma_raw
    return th


def _softplus(x):
    return math.log1p(math.exp(x))


def _render(scene, o, d, opts=None, model=MODEL):
    p = {k: torch.from_numpy(np.asarray(v, np.float64)) for k, v in scene.items()}
    return render_contact(p["center"], p["scale"], p["quat"], p["mlp"],
                          torch.from_numpy(np.asarray(o, np.float64)), torch.from_numpy(np.asarray(d, np.float64)),
                          model, opts or oracle.Opts())


def _unit(v):
    v = np.asarray(v, np.float64)
    return v / np.linalg.norm(v)


def test_optical_depth_is_the_line_integral_of_the_gaussian_density():
    """sigma G delta_i equals the integral over t of sigma exp(-1/2 (x-mu)^T Lambda (x-mu))
    along the ray (reading of the falloff and the scalar thickness), for a
    rotated anisotropic primitive and rays whose contact depth is positive."""
    mu = np.array([0.2, -0.1, 0.3])
    s = np.array([0.15, 0.05, 0.09])
    q = _unit([0.8, 0.3, -0.4, 0.2])
    lam = _lambda(s, q)
    sig_raw = 0.7
    scene = {"center": mu[None], "scale": s[None], "quat": q[None], "mlp": _const_mlp([0, 0, 0], sig_raw)[None]}
    rng = np.random.default_rng(3)
    o = np.array([0.0, -3.0, 0.5])
    ds = []
    for _ in range(6):
        # aim at a point near the centre
        tgt = mu + rng.normal(0, 0.08, 3)
        ds.append(_unit(tgt - o))
    ds = np.array(ds)
    out = _render(scene, np.repeat(o[None], len(ds), 0), ds)
    nhit = np.diff(out["ray_off"])
    sigma = _softplus(sig_raw)
    for i, d in enumerate(ds):
        f = lambda t: sigma * math.exp(-0.5 * (o + t * d - mu) @ lam @ (o + t * d - mu))
        ref, _ = integrate.quad(f, -50, 50, points=[float((mu - o) @ d)], epsabs=1e-13, epsrel=1e-12, limit=200)
        m2 = min((o + t * d - mu) @ lam @ (o + t * d - mu) for t in np.linspace(0, 6, 60001))
        if m2 >= KAPPA ** 2:
            assert nhit[i] == 0
            continue
        assert nhit[i] == 1
        tau = float(out["tau"][out["ray_off"][i]])
        assert abs(tau - ref) <= 1e-9 * max(ref, 1e-3), (tau, ref)


def test_constant_primitive_composites_alpha_times_colour():
    """C = (1 - exp(-tau)) sigmoid(c~) + exp(-tau) bg for one constant primitive."""
    mu = np.array([0.0, 0.0, 0.0])
    s = np.array([0.2, 0.2, 0.2])
    scene = {"center": mu[None], "scale": s[None], "quat": np.array([[1.0, 0, 0, 0]]),
             "mlp": _const_mlp([0.3, -1.0, 2.0], 0.1)[None]}
    b = 0.25                                                     # impact parameter
    o = np.array([[b, -3.0, 0.0]])
    d = np.array([[0.0, 1.0, 0.0]])
    bg = (0.1, 0.2, 0.3)
    out = _render(scene, o, d, oracle.Opts(background=bg))
    tau = _softplus(0.1) * math.exp(-0.5 * b * b / 0.04) * math.sqrt(2 * math.pi) * 0.2
    a = 1 - math.exp(-tau)
    col = 1 / (1 + np.exp(-np.array([0.3, -1.0, 2.0])))
    np.testing.assert_allclose(out["rgb"].numpy()[0], a * col + (1 - a) * np.array(bg), rtol=0, atol=1e-14)
    assert abs(float(out["trans"][0]) - (1 - a)) < 1e-14


def test_support_ends_at_three_standard_deviations():
    s = 0.1
    scene = {"center": np.zeros((1, 3)), "scale": np.full((1, 3), s), "quat": np.array([[1.0, 0, 0, 0]]),
             "mlp": _const_mlp([0, 0, 0], 1.0)[None]}
    o = np.array([[KAPPA * s * 0.999, -3.0, 0.0], [KAPPA * s * 1.001, -3.0, 0.0]])
    d = np.array([[0.0, 1.0, 0.0]] * 2)
    out = _render(scene, o, d)
    assert list(np.diff(out["ray_off"])) == [1, 0]
    assert float(out["trans"][1]) == 1.0


def test_residual_is_centre_minus_contact_point_with_the_clamp_of_eq2():
    """delta = mu - (o + t* d) with t* = max(0, t_c): a camera in front of the
    centre (t_c > 0) and one past it but inside the support (t_c < 0, so t* = 0
    and delta = mu - o)."""
    mu = np.array([0.1, 0.2, -0.1])
    s = np.array([0.3, 0.2, 0.25])
    q = _unit([1.0, 0.2, 0.1, -0.3])
    lam = _lambda(s, q)
    scene = {"center": mu[None], "scale": s[None], "quat": q[None], "mlp": _const_mlp([0, 0, 0], 0.0)[None]}
    d = _unit([0.3, 1.0, 0.2])
    o_front = mu - 2.0 * d + np.array([0.02, 0.0, 0.01])
    o_in = mu + 0.05 * d                                        # just past the centre along d
    out = _render(scene, np.array([o_front, o_in]), np.array([d, d]))
    tc_ref = [float(d @ lam @ (mu - o)) / float(d @ lam @ d) for o in (o_front, o_in)]
    assert tc_ref[0] > 0 and tc_ref[1] < 0
    np.testing.assert_allclose(out["t_c"].numpy(), tc_ref, rtol=1e-13)
    np.testing.assert_allclose(out["t_star"].numpy(), [tc_ref[0], 0.0], atol=1e-15)
    np.testing.assert_allclose(out["delta"].numpy()[0], mu - o_front - tc_ref[0] * d, atol=1e-14)
    np.testing.assert_allclose(out["delta"].numpy()[1], mu - o_in, atol=1e-15)
    # the falloff at the clamped contact point
    g_ref = math.exp(-0.5 * (mu - o_in) @ lam @ (mu - o_in))
    assert abs(float(out["falloff"][1]) - g_ref) < 1e-14


def test_encoding_layout():
    x = torch.tensor([[0.3, -0.7, 0.11, 1.9, -0.05, 0.5]], dtype=torch.float64)
    e = encode_vec(x, 6).numpy()[0]
    assert e.shape == (72,)
    for c in range(6):
        for lvl in range(6):
            a = (2 ** lvl) * math.pi * float(x[0, c])
            assert abs(e[12 * c + 2 * lvl] - math.sin(a)) < 1e-15
            assert abs(e[12 * c + 2 * lvl + 1] - math.cos(a)) < 1e-15


def test_network_input_is_direction_then_residual():
    """A network whose density reads sin(pi delta_x) and whose red channel
    reads cos(2 pi d_y), through identity-like ReLU paths with positive
    offsets: the outputs follow from hand-computed d and delta."""
    m = MODEL
    th = np.zeros(m.num_params)
    W1 = th[:72 * 32].reshape(32, 72)
    b1 = th[72 * 32:72 * 32 + 32]
    o2 = 72 * 32 + 32
    W2 = th[o2:o2 + 32 * 32].reshape(32, 32)
    b2 = th[o2 + 32 * 32:o2 + 32 * 32 + 32]
    o3 = o2 + 32 * 32 + 32
    W3 = th[o3:o3 + 32 * 4].reshape(4, 32)
    b3 = th[o3 + 32 * 4:]
    W1[0, 12 * 3 + 0] = 1.0                 # sin(2^0 pi delta_x): component 3 of [d; delta]
    b1[0] = 2.0
    W1[1, 12 * 1 + 2 * 1 + 1] = 1.0         # cos(2^1 pi d_y): component 1
    b1[1] = 2.0
    W2[0, 0] = 1.0
    W2[1, 1] = 1.0
    W3[3, 0] = 1.0                           # density raw = 2 + sin(pi delta_x)
    W3[0, 1] = 1.0                           # red raw = 2 + cos(2 pi d_y)
    b3[3] = -1.0
    b3[0] = -3.0
    mu = np.array([0.05, 0.4, 0.1])
    s = np.array([0.2, 0.2, 0.2])
    scene = {"center": mu[None], "scale": s[None], "quat": np.array([[1.0, 0, 0, 0]]), "mlp": th[None]}
    o = np.array([1.5, -2.0, 0.3])
    d = _unit(mu + np.array([0.1, 0.0, -0.05]) - o)
    out = _render(scene, o[None], d[None])
    tstar = float((mu - o) @ d)                # sphere: t_c = (mu - o) . d
    delta = mu - o - tstar * d
    dens = _softplus(2.0 + math.sin(math.pi * delta[0]) - 1.0)
    red_raw = 2.0 + math.cos(2 * math.pi * d[1]) - 3.0
    tau = dens * math.exp(-0.5 * (delta @ delta) / 0.04) * math.sqrt(2 * math.pi) * 0.2
    a = 1 - math.exp(-tau)
    assert abs(float(out["rgb"][0, 0]) - a / (1 + math.exp(-red_raw))) < 1e-14
    assert abs(float(out["rgb"][0, 1]) - a * 0.5) < 1e-14


def test_two_disjoint_primitives_composite_in_depth_order_for_any_labels():
    s = 0.1
    c1 = np.array([0.0, -0.5, 0.0])
    c2 = np.array([0.0, 0.6, 0.0])
    mlp1 = _const_mlp([1.0, -1.0, 0.0], 1.5)
    mlp2 = _const_mlp([-2.0, 0.5, 1.0], 0.2)
    o = np.array([[0.05, -3.0, 0.02]])
    d = np.array([[0.0, 1.0, 0.0]])
    tau = lambda sr, b2: _softplus(sr) * math.exp(-0.5 * b2 / s ** 2) * math.sqrt(2 * math.pi) * s
    b2 = 0.05 ** 2 + 0.02 ** 2
    a1, a2 = 1 - math.exp(-tau(1.5, b2)), 1 - math.exp(-tau(0.2, b2))
    sg = lambda v: 1 / (1 + np.exp(-np.asarray(v)))
    ref = a1 * sg([1.0, -1.0, 0.0]) + (1 - a1) * a2 * sg([-2.0, 0.5, 1.0])
    for order in ([0, 1], [1, 0]):
        cs = [c1, c2]
        ms = [mlp1, mlp2]
        scene = {"center": np.array([cs[i] for i in order]), "scale": np.full((2, 3), s),
                 "quat": np.array([[1.0, 0, 0, 0]] * 2), "mlp": np.array([ms[i] for i in order])}
        out = _render(scene, o, d)
        np.testing.assert_allclose(out["rgb"].numpy()[0], ref, atol=1e-14)


def test_early_termination_after_the_crossing_hit():
    """Three opaque primitives in a row: with T_stop between the
    transmittances after the first and after the second hit, the second is
    composited and the third is not."""
    s = 0.1
    cs = np.array([[0.0, -0.6, 0.0], [0.0, 0.0, 0.0], [0.0, 0.6, 0.0]])
    th = _const_mlp([0.0, 0.0, 0.0], 3.0)
    scene = {"center": cs, "scale": np.full((3, 3), s), "quat": np.array([[1.0, 0, 0, 0]] * 3),
             "mlp": np.array([th] * 3)}
    o = np.array([[0.0, -3.0, 0.0]])
    d = np.array([[0.0, 1.0, 0.0]])
    tau = _softplus(3.0) * math.sqrt(2 * math.pi) * s
    t1 = math.exp(-tau)
    out = _render(scene, o, d, oracle.Opts(t_stop=t1 * 0.5))
    assert int(out["n_used"][0]) == 2
    assert abs(float(out["trans"][0]) - t1 * t1) < 1e-15
    assert abs(float(out["rgb"][0, 0]) - 0.5 * (1 - t1 * t1)) < 1e-14


def test_tile_order_with_coinciding_rays_is_exact_order():
    rng = np.random.default_rng(5)
    scene = {"center": rng.uniform(-0.3, 0.3, (6, 3)), "scale": np.exp(rng.uniform(-2.5, -1.5, (6, 3))),
             "quat": rng.standard_normal((6, 4)), "mlp": rng.normal(0, 0.3, (6, MODEL.num_params))}
    o = np.repeat(np.array([[0.1, -3.0, 0.2]]), 64, 0)
    d = np.repeat(_unit([0.0, 1.0, -0.05])[None], 64, 0)
    a = _render(scene, o, d, oracle.Opts(order=0))
    b = _render(scene, o, d, oracle.Opts(order=1))
    np.testing.assert_array_equal(a["prim"], b["prim"])
    np.testing.assert_allclose(a["rgb"].numpy(), b["rgb"].numpy(), atol=0)


def test_gradients_match_complex_step():
    rng = np.random.default_rng(11)
    P = 4
    scene = {"center": rng.uniform(-0.2, 0.2, (P, 3)), "scale": np.exp(rng.uniform(-2.3, -1.6, (P, 3))),
             "quat": rng.standard_normal((P, 4)), "mlp": rng.normal(0, 0.4, (P, MODEL.num_params))}
    # a camera outside and rays towards the cluster (one origin inside a support)
    o = np.array([[0.0, -2.5, 0.1]] * 12 + [list(scene["center"][0] + 0.01)])
    d = np.array([_unit(scene["center"][i % P] + rng.normal(0, 0.05, 3) - o[i]) for i in range(13)])
    g_rgb = rng.standard_normal((13, 3))
    _, _, grads = contact_loss_and_grads(scene, o, d, MODEL, oracle.Opts(), g_rgb)
    h = 1e-30
    for key, idx in [("center", (0, 1)), ("center", (2, 0)), ("scale", (1, 2)), ("scale", (3, 0)),
                     ("quat", (0, 0)), ("quat", (2, 3)), ("mlp", (1, 5)), ("mlp", (3, MODEL.num_params - 1)),
                     ("mlp", (0, 72 * 32 + 10))]:
        p = {k: torch.from_numpy(np.asarray(v, np.float64)).to(torch.complex128) for k, v in scene.items()}
        p[key] = p[key].clone()
        p[key][idx] += 1j * h
        out = render_contact(p["center"], p["scale"], p["quat"], p["mlp"], torch.from_numpy(o), torch.from_numpy(d),
                             MODEL, oracle.Opts())
        cs = float((out["rgb"] * torch.from_numpy(g_rgb).to(torch.complex128)).sum().imag) / h
        assert abs(cs - grads[key][idx]) <= 1e-10 * max(1.0, abs(cs)), (key, idx, cs, grads[key][idx])
    # gradient with respect to the raw quaternion is orthogonal to it
    dots = (grads["quat"] * scene["quat"]).sum(1)
    assert np.abs(dots).max() < 1e-10 * np.abs(grads["quat"]).max()
