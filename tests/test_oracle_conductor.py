"""Pins of the oracle's rough conductor (the roughened mirror of the
paper's attached validation, Sec. 6.1) against facts other than its own
formulas:

  * the GGX distribution is normalised, int D(m) (m.n) dm = 1 (Gauss-Legendre);
  * Smith's G1 equals its tangent form 2 / (1 + sqrt(1 + a^2 tan^2)), is at
    most one and tends to one at normal incidence;
  * the BRDF is reciprocal, f(wi, wo) = f(wo, wi);
  * the sampler and the evaluation agree: for uniform uniforms, the mean of
    the sampled weight times test functions of wo equals the hemisphere
    integral of f (wo.n) / F0 times the same functions (the sampling density,
    its Jacobian and the weight together against the evaluated BRDF);
  * at vanishing roughness the reflection is the mirror law with weight one;
  * the light tracer's image of a conductor plane under a point light equals
    its closed form (the pixel-filtered radiance F0 f I0 cos / r^2);
  * with Lambertian and conductor vertices only, every connection at depth i
    is a degree-i monomial in the albedo / reflectance texels (Euler);
  * central finite differences of the loss in the mirror's heights
    (attached, equal signatures) and in its reflectance (detached).
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_32920_amd import scenes


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build(force=False)


def _gl(a, b, n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (b - a) * x + 0.5 * (a + b), 0.5 * (b - a) * w


@pytest.mark.parametrize("a", [0.05, 0.15, 0.4, 0.9])
def test_ggx_normalised(a):
    # int over the hemisphere of D(m) (m.n) = 2 pi int_0^1 D(c) c dc; the
    # peak near c = 1 has width ~a^2: split the interval geometrically
    edges = np.concatenate([[0.0], 1.0 - np.geomspace(1.0, 1e-9, 40)[1:], [1.0]])
    tot = 0.0
    for lo, hi in zip(edges[:-1], edges[1:]):
        c, w = _gl(lo, hi, 24)
        tot += sum(wi * O.ggx_terms(a, ci, 0.5)[0] * ci for ci, wi in zip(c, w))
    assert abs(2 * math.pi * tot - 1.0) < 1e-9, tot


@pytest.mark.parametrize("a", [0.05, 0.3, 0.8])
def test_smith_g1_tangent_form(a):
    for cv in (0.02, 0.2, 0.5, 0.8, 0.999999):
        g1 = O.ggx_terms(a, 0.5, cv)[1]
        t2 = (1 - cv * cv) / (cv * cv)
        assert abs(g1 - 2.0 / (1.0 + math.sqrt(1.0 + a * a * t2))) < 1e-13
        assert 0.0 < g1 <= 1.0
    assert abs(O.ggx_terms(a, 0.5, 1.0)[1] - 1.0) < 1e-15


def _dir(theta, phi):
    return np.array([math.sin(theta) * math.cos(phi), math.sin(theta) * math.sin(phi), math.cos(theta)])


def test_reciprocity():
    rng = np.random.default_rng(3)
    n = np.array([0.0, 0.0, 1.0])
    for _ in range(50):
        wi, wo = _dir(rng.uniform(0, 1.5), rng.uniform(0, 6.3)), _dir(rng.uniform(0, 1.5), rng.uniform(0, 6.3))
        a = rng.uniform(0.05, 0.8)
        f_io = O.conductor_conn(wi, wo, n, a) / (wo @ n)
        f_oi = O.conductor_conn(wo, wi, n, a) / (wi @ n)
        assert abs(f_io - f_oi) <= 1e-12 * abs(f_io)


@pytest.mark.parametrize("a,theta_i", [(0.15, 0.3), (0.4, 1.0), (0.8, 0.6)])
def test_sampler_matches_evaluation(a, theta_i):
    """E_u[w(u) phi(wo(u))] = int f (wo.n)/F0 phi(wo) dwo for several phi."""
    n = np.array([0.0, 0.0, 1.0])
    wi = _dir(theta_i, 0.4)
    # the sampler over a stratified grid of uniforms (midpoints)
    k = 300
    us = (np.arange(k) + 0.5) / k
    phis = [lambda w: 1.0, lambda w: w[0], lambda w: w[2] ** 2, lambda w: w[1] * w[2]]
    mc = np.zeros(len(phis))
    for u0 in us:
        for u1 in us:
            code, wo, wgt = O.conductor(wi, n, a, u0, u1)
            if code == 0:
                mc += wgt * np.array([p(wo) for p in phis])
    mc /= k * k
    # the evaluated BRDF integrated over the hemisphere of wo
    ct, wt = _gl(0.0, 1.0, 96)
    pp, wp = _gl(0.0, 2 * math.pi, 128)
    quad = np.zeros(len(phis))
    for c, w1 in zip(ct, wt):
        s = math.sqrt(1 - c * c)
        for p, w2 in zip(pp, wp):
            wo = np.array([s * math.cos(p), s * math.sin(p), c])
            val = O.conductor_conn(wi, wo, n, a)
            quad += w1 * w2 * val * np.array([q(wo) for q in phis])
    np.testing.assert_allclose(mc, quad, rtol=2e-2, atol=2e-3 * abs(quad[0]))
    assert 0.3 < quad[0] <= 1.0   # directional albedo over F0: masking loses energy, never gains


def test_vanishing_roughness_is_a_mirror():
    n = np.array([0.0, 0.0, 1.0])
    rng = np.random.default_rng(5)
    for _ in range(20):
        wi = _dir(rng.uniform(0.05, 1.3), rng.uniform(0, 6.28))
        code, wo, wgt = O.conductor(wi, n, 1e-6, rng.uniform(0, 0.99), rng.uniform(0, 1))
        assert code == 0
        np.testing.assert_allclose(wo, 2 * (wi @ n) * n - wi, atol=1e-5)
        assert abs(wgt - 1.0) < 1e-5


def _expected_conductor_plane_image(sc):
    cam = sc["camera"]
    W, H = cam["width"], cam["height"]
    h = cam["pos"][1]
    t = np.tan(np.radians(cam["fov_deg"]) / 2)
    asp = W / H
    F0 = sc["albedo"].reshape(-1)[0]
    I0 = sc["Le"][0]
    rough = sc["mat_ior"][0]
    lp = np.asarray(sc["emitter"]["o"], float)
    cp = np.asarray(cam["pos"], float)
    n = np.array([0.0, 1.0, 0.0])

    def radiance(ux, uy):
        qx = (2 * ux / W - 1) * asp * t
        qy = (1 - 2 * uy / H) * t
        X = np.array([-h * qx, 0.0, h * qy])
        dl, dc = lp - X, cp - X
        r2 = dl @ dl
        wi, wc = dl / math.sqrt(r2), dc / np.linalg.norm(dc)
        # radiance toward the camera: F0 f(wi, wc) I0 (wi.n) / r^2
        return F0 * O.conductor_conn(wi, wc, n, rough) / (wc @ n) * I0 * (wi @ n) / r2

    def axis_nodes(p, nn):
        xs, ws = [], []
        for lo, hi in ((p - 0.5, p + 0.5), (p + 0.5, p + 1.5)):
            lo, hi = max(lo, 0.0), min(hi, float(nn))
            if hi <= lo:
                continue
            x, w = _gl(lo, hi, 8)
            xs.append(x)
            ws.append(w * np.maximum(0.0, 1.0 - np.abs(x - p - 0.5)))
        return np.concatenate(xs), np.concatenate(ws)

    E = np.zeros((H, W))
    for py in range(H):
        y, wy = axis_nodes(py, H)
        for px in range(W):
            x, wx = axis_nodes(px, W)
            E[py, px] = sum(wy[i] * wx[k] * radiance(x[k], y[i]) for i in range(len(y)) for k in range(len(x)))
    return E


def test_point_light_conductor_plane_closed_form():
    sc = scenes.plane_point_light_scene(width=12, height=12, roughness=0.35, light_h=0.8)
    E = _expected_conductor_plane_image(sc)
    seeds, n = 16, 1 << 18
    imgs = np.stack([O.render(sc, 3000 + s, n, 1)["image"][..., 0] for s in range(seeds)])
    mean = imgs.mean(0)
    se = imgs.std(0, ddof=1) / np.sqrt(seeds)
    z = (mean - E) / se
    assert np.all(se > 0)
    assert 0.6 < np.mean(z * z) < 1.8, np.mean(z * z)
    assert np.max(np.abs(z)) < 6.0
    assert abs(mean.sum() / E.sum() - 1.0) < 5e-3


def test_mirror_euler_homogeneity():
    sc = scenes.mirror_scene(G=8, width=32, height=32)
    seed, n, D = 4, 20000, 4
    r = O.render(sc, seed, n, D, slices=True)
    dI = np.random.default_rng(2).normal(size=r["image"].shape)
    g = O.gradient(sc, seed, n, D, dI)
    lhs = np.sum(sc["albedo"] * g["albedo"])
    rhs = sum((i + 1) * np.sum(dI * r["slices"][i]) for i in range(D))
    assert abs(lhs - rhs) <= 1e-9 * max(1.0, abs(rhs)), (lhs, rhs)
    # both texels carry gradient: the wall's albedo and the mirror's F0
    assert np.all(np.abs(g["albedo"].reshape(2, 3)) > 0)


def test_mirror_reflectance_finite_differences():
    sc = scenes.mirror_scene(G=8, width=32, height=32)
    seed, n, D = 6, 6000, 4
    T = O.render(sc, 99, n, D, heights=sc["heights_target"])["image"]
    I = O.render(sc, seed, n, D)["image"]
    _, dI = O.loss_and_adjoint(I, T)
    g = O.gradient(sc, seed, n, D, dI)["albedo"].reshape(-1)
    alb = sc["albedo"].reshape(-1)
    for i in (3, 4, 5):   # the mirror's F0 channels
        h = 1e-6
        ap, am = alb.copy(), alb.copy()
        ap[i] += h; am[i] -= h
        fd = (O.loss_and_adjoint(O.render(sc, seed, n, D, albedo=ap.reshape(sc["albedo"].shape))["image"], T)[0]
              - O.loss_and_adjoint(O.render(sc, seed, n, D, albedo=am.reshape(sc["albedo"].shape))["image"], T)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-5 * abs(g[i]) + 1e-12, (i, fd, g[i])


def test_mirror_heights_finite_differences_attached():
    sc = scenes.mirror_scene(G=8, width=32, height=32)
    seed, n, D = 5, 4096, 4
    T = O.render(sc, 99, n, D, heights=sc["heights_target"])["image"]
    r0 = O.render(sc, seed, n, D, per_path=True)
    _, dI = O.loss_and_adjoint(r0["image"], T)
    gh = O.gradient(sc, seed, n, D, dI, flags=O.ATTACHED)["heights"]
    assert np.count_nonzero(gh) > 20
    h0 = sc["heights"].copy()
    eps, checked = 1e-7, 0
    for k in np.argsort(-np.abs(gh))[:12]:
        hp, hm = h0.copy(), h0.copy()
        hp[k] += eps
        hm[k] -= eps
        rp = O.render(sc, seed, n, D, heights=hp, per_path=True)
        rm = O.render(sc, seed, n, D, heights=hm, per_path=True)
        if not (np.array_equal(rp["sig"], r0["sig"]) and np.array_equal(rm["sig"], r0["sig"])):
            continue
        fd = (O.loss_and_adjoint(rp["image"], T)[0] - O.loss_and_adjoint(rm["image"], T)[0]) / (2 * eps)
        assert abs(fd - gh[k]) <= 1e-5 * np.abs(gh).max(), (k, fd, gh[k])
        checked += 1
    assert checked >= 6
