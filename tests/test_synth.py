"""The seeded input generators: the per-packet tile-centre rays that tile
order can take as its virtual rays."""
import numpy as np

import oracle
import synth


def _cam(w, h, seed=3):
    return synth.make_camera(np.random.default_rng(seed), w, h, 3.0, 50.0)


def test_tile_ray_passes_through_the_tile_centre():
    # the image-plane direction is affine in the pixel position, so the ray
    # through the centre of an 8x8 tile points along the mean of the
    # (unnormalised) directions through the centres of its four middle pixels
    cam = _cam(32, 24)
    rays = synth.packet_tile_rays(cam)
    assert rays.shape == (12, 6)
    o, d, pix = synth.camera_rays(cam)
    f = cam["focal"]
    for k in (0, 5, 11):
        p = pix[64 * k:64 * k + 64]
        x0, y0 = (p % 32).min(), (p // 32).min()
        acc = np.zeros(3)
        for dy in (3, 4):
            for dx in (3, 4):
                u = (x0 + dx + 0.5 - 16) / f
                v = (y0 + dy + 0.5 - 12) / f
                acc += cam["fwd"] + u * cam["right"] - v * cam["up"]
        want = acc / np.linalg.norm(acc)
        np.testing.assert_allclose(rays[k, 3:], want, atol=1e-6)
        np.testing.assert_allclose(rays[k, :3], cam["eye"], atol=1e-6)
        # every pixel of the packet lies in that tile
        assert set(zip(p % 32 - x0, p // 32 - y0)) == {(i, j) for i in range(8) for j in range(8)}


def test_tile_ray_differs_from_the_mean_ray_at_second_order():
    # the default virtual ray (mean origin, normalised direction sum) and the
    # tile-centre ray agree to first order in the tile's angular size and
    # differ beyond it off the optical axis
    cam = _cam(64, 64)
    rays = synth.packet_tile_rays(cam)
    o, d, _ = synth.camera_rays(cam)
    oc, dc = oracle.packet_centres(o, d)
    ang = [np.arccos(np.clip(rays[k, 3:] @ dc[64 * k], -1, 1)) for k in range(len(rays))]
    tile = 8 / cam["focal"]          # angular size of a tile
    assert max(ang) < tile ** 2
    assert max(ang) > 0.0


def test_ragged_packets_take_their_bounding_box_centre():
    cam = _cam(20, 12)
    rays = synth.packet_tile_rays(cam)
    n = 20 * 12
    assert rays.shape == ((n + 63) // 64, 6)
    np.testing.assert_allclose(np.linalg.norm(rays[:, 3:], axis=1), 1.0, atol=1e-6)
