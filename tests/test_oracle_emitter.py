"""Pins of the oracle's directional emitter and emitter radiance texture
(the Tumbler validation of the paper differentiates the radiance texture of
a directional emitter, Sec. 6.1).

  * closed form: a textured collimated beam falling straight down on a
    Lambertian plane seen by a camera looking straight down gives, per
    pixel, the sum over texels of rho E_t / pi times the tent-filtered film
    area of the texel's footprint (Eq. 1, Eq. 20); this pins the beam
    direction, its normalisation and the texel orientation;
  * a texture whose texels are all equal renders the same paths and image
    as the untextured emitter;
  * every connection is linear in its emission texel, so per channel
    sum_t E_t dJ/dE_t = <dI, I> exactly, per seed;
  * central finite differences in single texels.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_32920_amd import scenes


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build(force=False)


def _tent_integral(p, a, b):
    """Integral over u in [a, b] of max(0, 1 - |u - p - 1/2|)."""
    def Phi(v):  # antiderivative of the unit tent from -1, v clipped to [-1, 1]
        v = min(max(v, -1.0), 1.0)
        return v - math.copysign(v * v / 2.0, v) + 0.5
    if b <= a:
        return 0.0
    return Phi(b - p - 0.5) - Phi(a - p - 0.5)


def _expected_directional_image(sc):
    cam = sc["camera"]
    W, H = cam["width"], cam["height"]
    h = cam["pos"][1]
    t = math.tan(math.radians(cam["fov_deg"]) / 2)
    a = W / H
    rho = sc["albedo"].reshape(-1)[0]
    em = sc["emitter"]
    R = em["tex_res"]
    E = sc["Le"].reshape(R, R, 3)
    o, e1, e2 = em["o"], em["e1"], em["e2"]
    # camera looking down, up +z: film u_x = W/2 (1 - X/(h a t)), u_y = H/2 (1 - Z/(h t))
    ux = lambda X: W / 2 * (1 - X / (h * a * t))
    uy = lambda Z: H / 2 * (1 - Z / (h * t))
    img = np.zeros((H, W, 3))
    for ty in range(R):
        for tx in range(R):
            x0, x1 = o[0] + e1[0] * tx / R, o[0] + e1[0] * (tx + 1) / R
            z0, z1 = o[2] + e2[2] * ty / R, o[2] + e2[2] * (ty + 1) / R
            ua, ub = sorted((ux(x0), ux(x1)))
            va, vb = sorted((uy(z0), uy(z1)))
            ua, ub, va, vb = max(ua, 0.0), min(ub, W), max(va, 0.0), min(vb, H)
            for py in range(H):
                fy = _tent_integral(py, va, vb)
                if fy == 0.0:
                    continue
                for px in range(W):
                    fx = _tent_integral(px, ua, ub)
                    img[py, px] += rho / math.pi * E[ty, tx] * fx * fy
    return img


def test_directional_textured_closed_form():
    sc = scenes.directional_plane_scene(width=16, height=16)
    E = _expected_directional_image(sc)
    assert E.max() > 0
    seeds, n = 16, 1 << 18
    imgs = np.stack([O.render(sc, 4000 + s, n, 1)["image"] for s in range(seeds)])
    mean = imgs.mean(0)
    se = imgs.std(0, ddof=1) / np.sqrt(seeds)
    lit = se > 0
    assert np.all(E[~lit] == 0) and np.all(mean[~lit] == 0)
    z = (mean[lit] - E[lit]) / se[lit]
    assert 0.6 < np.mean(z * z) < 1.6, np.mean(z * z)
    assert np.max(np.abs(z)) < 5.5
    tot = imgs.sum((1, 2, 3))
    assert abs(tot.mean() / E.sum() - 1.0) < 4 * tot.std(ddof=1) / np.sqrt(seeds) / E.sum() + 1e-12
    # the transposed texture (u0 along e2) is far from the samples
    sc_t = dict(sc, Le=sc["Le"].reshape(4, 4, 3).transpose(1, 0, 2).reshape(-1).copy())
    Et = _expected_directional_image(sc_t)
    zt = (mean[lit] - Et[lit]) / se[lit]
    assert np.mean(zt * zt) > 10.0


def test_uniform_texture_equals_untextured():
    sc = scenes.tumbler_scene(G=8, width=32, height=32, tex_res=4)
    flat = dict(sc, emitter=dict(sc["emitter"], tex_res=0), Le=np.array([20.0, 15.0, 10.0]))
    tex = dict(sc, Le=np.tile([20.0, 15.0, 10.0], 16))
    r0 = O.render(flat, 5, 8192, 5, per_path=True, threads=1)
    r1 = O.render(tex, 5, 8192, 5, per_path=True, threads=1)
    assert np.array_equal(r0["sig"], r1["sig"]) and np.array_equal(r0["image"], r1["image"])


def test_emitter_texture_scaling_identity():
    sc = scenes.tumbler_scene(G=8, width=32, height=32, tex_res=4)
    r = O.render(sc, 6, 16384, 5)
    dI = np.random.default_rng(8).normal(size=r["image"].shape)
    g = O.gradient(sc, 6, 16384, 5, dI)
    lhs = (sc["Le"] * g["Le"]).reshape(-1, 3).sum(0)
    rhs = np.einsum("hwc,hwc->c", dI, r["image"])
    np.testing.assert_allclose(lhs, rhs, rtol=1e-10)
    assert np.count_nonzero(g["Le"]) == g["Le"].size


def test_finite_differences_emitter_texture():
    sc = scenes.tumbler_scene(G=8, width=32, height=32, tex_res=4)
    seed, n, D = 9, 4096, 5
    T = O.render(sc, 99, n, D, Le=sc["Le_target"])["image"]
    I = O.render(sc, seed, n, D)["image"]
    _, dI = O.loss_and_adjoint(I, T)
    g = O.gradient(sc, seed, n, D, dI)["Le"]
    le0 = sc["Le"].copy()
    h = 1e-4
    for k in list(np.argsort(-np.abs(g))[:6]) + [0, 7, 25]:
        lp, lm = le0.copy(), le0.copy()
        lp[k] += h
        lm[k] -= h
        fd = (O.loss_and_adjoint(O.render(sc, seed, n, D, Le=lp)["image"], T)[0]
              - O.loss_and_adjoint(O.render(sc, seed, n, D, Le=lm)["image"], T)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * np.abs(g).max(), (k, fd, g[k])
