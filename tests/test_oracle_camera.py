"""Pins of the oracle's camera side (the bidirectional combination of the
paper's closing discussion: path replay on camera paths, light tracing for
the rest).

Camera samples are a path tracer with next-event estimation at Lambertian
and rough-conductor vertices and emission counted after specular bounces.
Checked against facts that do not come from the camera code itself:
  * the closed-form transmission of a flat glass slab (textbook Fresnel and
    a geometric series of internal reflections, Eq. 1 with a delta BSDF);
  * the closed-form image of a point light over a Lambertian plane;
  * the light tracer, an independent estimator of the same measurement
    (Eq. 1), on a diffuse box and on the rough-conductor mirror;
  * the partition of path space: light paths plus camera paths whose first
    vertex is specular give the full camera estimate on the glass slab;
  * central finite differences and the emitter-radiance scaling identity of
    the camera gradient.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_32920_amd import scenes
from test_oracle_pins import _expected_point_light_image, _gauss_legendre


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build(force=False)


def _fresnel(cos_i, ior):
    """Unpolarized Fresnel reflectance entering a medium of index ior."""
    sin_t2 = (1.0 - cos_i * cos_i) / (ior * ior)
    cos_t = np.sqrt(1.0 - sin_t2)
    rs = (cos_i - ior * cos_t) / (cos_i + ior * cos_t)
    rp = (ior * cos_i - cos_t) / (ior * cos_i + cos_t)
    return 0.5 * (rs * rs + rp * rp)


def _slab_expected(sc, depth):
    """Pixel values of slab_view_scene: Le times the tent-filtered slab
    transmission sum_{k <= K} (1-F)^2 F^(2k), with 2 + 2k dielectric
    vertices allowed below the depth cap (K = (depth - 3) // 2)."""
    cam = sc["camera"]
    W, H = cam["width"], cam["height"]
    t = np.tan(np.radians(cam["fov_deg"]) / 2)
    a = W / H
    ior = sc["mat_ior"][0]
    K = (depth - 3) // 2

    def value(ux, uy):
        qx = (2 * ux / W - 1) * a * t
        qy = (1 - 2 * uy / H) * t
        c = 1.0 / np.sqrt(1.0 + qx * qx + qy * qy)   # camera looks straight down
        F = _fresnel(c, ior)
        return sc["Le"][0] * sum((1 - F) ** 2 * F ** (2 * k) for k in range(K + 1))

    def axis(p, n):
        xs, ws = [], []
        for lo, hi in ((p - 0.5, p + 0.5), (p + 0.5, p + 1.5)):
            lo, hi = max(lo, 0.0), min(hi, float(n))
            if hi <= lo:
                continue
            x, w = _gauss_legendre(lo, hi)
            xs.append(x)
            ws.append(w * np.maximum(0.0, 1.0 - np.abs(x - p - 0.5)))
        return np.concatenate(xs), np.concatenate(ws)

    E = np.zeros((H, W))
    for py in range(H):
        y, wy = axis(py, H)
        for px in range(W):
            x, wx = axis(px, W)
            XX, YY = np.meshgrid(x, y)
            E[py, px] = np.sum(np.outer(wy, wx) * value(XX, YY))
    return E


def _z_check(mean, se, E, max_z=6.0):
    assert np.all(se > 0)
    z = (mean - E) / se
    assert 0.4 < np.mean(z * z) < 2.0, np.mean(z * z)
    assert np.max(np.abs(z)) < max_z, np.max(np.abs(z))


@pytest.mark.parametrize("depth", [3, 8])
def test_slab_transmission_closed_form(depth):
    sc = scenes.slab_view_scene()
    E = _slab_expected(sc, depth)
    npx = E.size
    seeds, spp = 12, 2048
    imgs = np.stack([O.render_camera(sc, 40 + s, spp * npx, depth)["image"][..., 0] for s in range(seeds)])
    _z_check(imgs.mean(0), imgs.std(0, ddof=1) / np.sqrt(seeds), E)
    # the truncated series differs between the two depths by F^2 (1-F)^2 ~ 1.5e-3
    assert abs(imgs.mean() / E.mean() - 1.0) < 3e-4


def test_point_light_closed_form_camera():
    sc = scenes.plane_point_light_scene(width=16, height=16)
    E = _expected_point_light_image(sc)
    seeds, spp = 12, 64
    imgs = np.stack([O.render_camera(sc, 70 + s, spp * E.size, 1, spec_only=False)["image"][..., 0]
                     for s in range(seeds)])
    _z_check(imgs.mean(0), imgs.std(0, ddof=1) / np.sqrt(seeds), E)
    assert abs(imgs.mean(0).sum() / E.sum() - 1.0) < 2e-3


def _blocks(img, b):
    H, W = img.shape[:2]
    return img.reshape(H // b, b, W // b, b, 3).mean((1, 3))


def _agree(a_imgs, b_imgs, rel_total):
    """Seed means of two estimators agree block by block (z-test on the seed
    spread) and in total."""
    ma, mb = a_imgs.mean(0), b_imgs.mean(0)
    sa = a_imgs.std(0, ddof=1) / np.sqrt(len(a_imgs))
    sb = b_imgs.std(0, ddof=1) / np.sqrt(len(b_imgs))
    se = np.sqrt(sa * sa + sb * sb)
    keep = se > 0
    assert keep.mean() > 0.75
    assert not np.any(ma[~keep]) and not np.any(mb[~keep])   # blocks that see nothing lit
    z = (ma - mb)[keep] / se[keep]
    assert np.mean(z * z) < 2.5, np.mean(z * z)
    assert np.max(np.abs(z)) < 6.0, np.max(np.abs(z))
    assert abs(ma.sum() / mb.sum() - 1.0) < rel_total


def test_camera_matches_light_tracer_on_box():
    sc = scenes.box_scene(width=32, height=32)
    depth, seeds = 3, 6
    lt = np.stack([_blocks(O.render(sc, 100 + s, 1 << 19, depth)["image"], 8) for s in range(seeds)])
    pt = np.stack([_blocks(O.render_camera(sc, 200 + s, 128 * 1024, depth, spec_only=False)["image"], 8)
                   for s in range(seeds)])
    _agree(lt, pt, 0.01)


def test_camera_matches_light_tracer_on_rough_mirror():
    sc = scenes.mirror_scene(G=8, width=32, height=32)
    depth, seeds = 3, 6
    lt = np.stack([_blocks(O.render(sc, 300 + s, 1 << 19, depth)["image"], 8) for s in range(seeds)])
    pt = np.stack([_blocks(O.render_camera(sc, 400 + s, 256 * 1024, depth, spec_only=False)["image"], 8)
                   for s in range(seeds)])
    _agree(lt, pt, 0.03)


def test_light_paths_plus_specular_camera_paths_cover_the_slab():
    # every camera path starts at a specular or a non-specular vertex: the
    # light tracer estimates the second kind, spec_only camera paths the first
    sc = scenes.glass_slab_scene(G=8, width=32, height=32)
    depth, seeds = 6, 6
    bd = np.stack([_blocks(O.render(sc, 500 + s, 1 << 19, depth)["image"]
                           + O.render_camera(sc, 600 + s, 64 * 1024, depth)["image"], 8)
                   for s in range(seeds)])
    full = np.stack([_blocks(O.render_camera(sc, 700 + s, 256 * 1024, depth, spec_only=False)["image"], 8)
                     for s in range(seeds)])
    _agree(bd, full, 0.02)
    # the camera-side share is substantial on this framing
    cam = O.render_camera(sc, 1, 64 * 1024, depth)["image"]
    assert cam.sum() > 0.2 * full.mean(0).sum() * 64


def test_specular_camera_paths_vanish_without_glass():
    sc = scenes.box_scene(width=16, height=16)
    assert not np.any(O.render_camera(sc, 3, 16 * 256, 4)["image"])


def test_camera_path_list_is_a_partition():
    sc = scenes.glass_slab_scene(G=8, width=16, height=16)
    n = 32 * 256
    full = O.render_camera(sc, 8, n, 5)["image"]
    ids = np.arange(n, dtype=np.uint32)
    a = O.render_camera(sc, 8, n, 5, path_list=ids[ids % 3 == 0])["image"]
    b = O.render_camera(sc, 8, n, 5, path_list=ids[ids % 3 != 0])["image"]
    np.testing.assert_allclose(a + b, full, rtol=1e-12, atol=1e-15)


def _slab_grad_case(seed=5, depth=5):
    sc = scenes.glass_slab_scene(G=8, width=16, height=16, tex_res=4)
    n = 64 * 256
    img = O.render_camera(sc, seed, n, depth)["image"]
    dI = np.random.default_rng(9).normal(size=img.shape)
    g = O.gradient_camera(sc, seed, n, depth, dI)
    return sc, n, img, dI, g


def test_camera_gradient_finite_differences():
    sc, n, img, dI, g = _slab_grad_case()
    alb = sc["albedo"].reshape(-1)
    rng = np.random.default_rng(4)
    idx = rng.choice(alb.size, 8, replace=False)
    ga = g["albedo"].reshape(-1)
    assert np.count_nonzero(ga) > alb.size // 2
    for k in idx:
        h = 1e-4
        ap, am = alb.copy(), alb.copy()
        ap[k] += h
        am[k] -= h
        Jp = np.sum(dI * O.render_camera(sc, 5, n, 5, albedo=ap)["image"])
        Jm = np.sum(dI * O.render_camera(sc, 5, n, 5, albedo=am)["image"])
        fd = (Jp - Jm) / (2 * h)
        assert abs(fd - ga[k]) <= 1e-6 * max(1.0, abs(fd)), (k, fd, ga[k])


def test_camera_emitter_radiance_scaling_identity():
    # every camera term is linear in L_e per channel
    sc, n, img, dI, g = _slab_grad_case()
    lhs = sc["Le"] * g["Le"]
    rhs = (dI * img).sum((0, 1))
    np.testing.assert_allclose(lhs, rhs, rtol=1e-10)


def test_camera_matches_light_tracer_with_textured_emitter():
    # next-event texel lookup against the light tracer's emission texel
    sc = scenes.box_scene(width=16, height=16)
    sc["emitter"]["tex_res"] = 4
    sc["Le"] = np.random.default_rng(8).uniform(2.0, 20.0, size=(4, 4, 3))
    depth, seeds = 2, 6
    lt = np.stack([_blocks(O.render(sc, 800 + s, 1 << 18, depth)["image"], 4) for s in range(seeds)])
    pt = np.stack([_blocks(O.render_camera(sc, 900 + s, 256 * 256, depth, spec_only=False)["image"], 4)
                   for s in range(seeds)])
    _agree(lt, pt, 0.015)
