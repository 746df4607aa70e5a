"""Pins of the oracle's scattering steps against optics and closed forms.

The smooth dielectric (the slab material of the caustic workload, Sec. 6)
is driven one event at a time through the oracle's own step and checked
against facts that do not depend on how the oracle writes them:
  * Snell's law (refracted direction coplanar, n1 sin t1 = n2 sin t2),
    including the exit side (relative index inverted);
  * the Fresnel reflectance in its angle form (s and p amplitudes as
    sin/tan of the angle sum and difference), its normal-incidence value
    ((n - 1)/(n + 1))^2, the vanishing p amplitude at Brewster's angle, where
    the reflected and refracted rays are perpendicular;
  * total internal reflection beyond the critical angle;
  * the mirror law;
  * the lobe rule (reflect iff the lobe uniform is below F) and the two
    path-ending cases of a shading normal that differs from the geometric
    one.
Multi-bounce diffuse transport (the cosine direction law and the albedo
weight of a scattering vertex, Eq. 2) is pinned by the closed-form depth-2
image of a point light, a Lambertian floor and a Lambertian wall: the
expected once-reflected radiance on the wall is an integral over the floor,
evaluated by Gauss-Legendre quadrature.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_32920_amd import scenes

N1, N2 = 1.0, 1.5
UP = np.array([0.0, 1.0, 0.0])
ALMOST_ONE = 1.0 - 2.0 ** -24


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build(force=False)


def _down(theta, phi=0.4):
    """Unit direction travelling downwards at angle theta from -y."""
    return np.array([math.sin(theta) * math.cos(phi), -math.cos(theta), math.sin(theta) * math.sin(phi)])


def _up(theta, phi=0.4):
    """Unit direction travelling upwards at angle theta from +y."""
    return np.array([math.sin(theta) * math.cos(phi), math.cos(theta), math.sin(theta) * math.sin(phi)])


def _fresnel_angles(ti, n_i, n_t):
    """Unpolarized reflectance from the angle form of the Fresnel equations."""
    tt = math.asin(n_i / n_t * math.sin(ti))
    rs = -math.sin(ti - tt) / math.sin(ti + tt)
    rp = math.tan(ti - tt) / math.tan(ti + tt)
    return 0.5 * (rs * rs + rp * rp), rs, rp, tt


def test_normal_incidence_reflectance():
    R0 = ((N2 - N1) / (N2 + N1)) ** 2  # 0.04
    for w, expect_t in ((np.array([0.0, -1.0, 0.0]), -1.0), (np.array([0.0, 1.0, 0.0]), 1.0)):
        code, wo, refl, F = O.dielectric(w, UP, UP, N2, ALMOST_ONE)
        assert code == 0 and not refl
        assert abs(F - R0) < 1e-15
        np.testing.assert_allclose(wo, [0.0, expect_t, 0.0], atol=1e-15)  # straight through
        code, wo, refl, F = O.dielectric(w, UP, UP, N2, 0.0)
        assert code == 0 and refl
        np.testing.assert_allclose(wo, -w, atol=1e-15)                      # straight back


@pytest.mark.parametrize("entering", [True, False])
def test_snell_law_of_the_refracted_direction(entering):
    n_i, n_t = (N1, N2) if entering else (N2, N1)
    tmax = math.radians(85) if entering else math.asin(N1 / N2) - 1e-3
    for ti in np.linspace(0.05, tmax, 12):
        w = _down(ti) if entering else _up(ti)
        code, wo, refl, F = O.dielectric(w, UP, UP, N2, ALMOST_ONE)
        assert code == 0 and not refl, ti
        assert abs(np.linalg.norm(wo) - 1.0) < 1e-14
        # the refracted ray continues through the interface ...
        assert np.sign(wo[1]) == np.sign(w[1])
        # ... in the plane of incidence, on the same side of the normal ...
        plane = np.cross(w, UP)
        assert abs(np.dot(plane / np.linalg.norm(plane), wo)) < 1e-14
        assert np.dot(wo[[0, 2]], w[[0, 2]]) > 0
        # ... bent by Snell's law
        sin_t = np.linalg.norm(np.cross(wo, UP))
        assert abs(n_i * math.sin(ti) - n_t * sin_t) < 1e-14, (ti, sin_t)


@pytest.mark.parametrize("entering", [True, False])
def test_fresnel_reflectance_angle_form(entering):
    n_i, n_t = (N1, N2) if entering else (N2, N1)
    tmax = math.radians(88) if entering else math.asin(N1 / N2) - 1e-4
    for ti in np.linspace(0.02, tmax, 25):
        w = _down(ti) if entering else _up(ti)
        F_ref = _fresnel_angles(ti, n_i, n_t)[0]
        F = O.dielectric(w, UP, UP, N2, 0.5)[3]
        assert abs(F - F_ref) < 1e-13, (ti, F, F_ref)
    # Stokes reciprocity: the reflectance of a refracted pair of angles is
    # the same from either side
    for ti in np.linspace(0.1, 1.4, 7):
        tt = math.asin(N1 / N2 * math.sin(ti))
        Fo = O.dielectric(_down(ti), UP, UP, N2, 0.5)[3]
        Fi = O.dielectric(_up(tt), UP, UP, N2, 0.5)[3]
        assert abs(Fo - Fi) < 1e-13


@pytest.mark.parametrize("entering", [True, False])
def test_brewster_angle(entering):
    n_i, n_t = (N1, N2) if entering else (N2, N1)
    tb = math.atan(n_t / n_i)
    w = _down(tb) if entering else _up(tb)
    F, rs, rp, tt = _fresnel_angles(tb, n_i, n_t)
    assert abs(rp) < 1e-15
    code, wr, refl, Fo = O.dielectric(w, UP, UP, N2, 0.0)
    assert code == 0 and refl
    code, wt, refl, _ = O.dielectric(w, UP, UP, N2, ALMOST_ONE)
    assert code == 0 and not refl
    assert abs(Fo - 0.5 * rs * rs) < 1e-14      # only the s polarization reflects
    assert abs(np.dot(wr, wt)) < 1e-14          # reflected and refracted rays are perpendicular


def test_total_internal_reflection():
    tc = math.asin(N1 / N2)
    for ti in (tc + 1e-6, tc + 0.1, math.radians(70), math.radians(89)):
        w = _up(ti)
        code, wo, refl, F = O.dielectric(w, UP, UP, N2, ALMOST_ONE)
        assert F == 1.0 and refl and code == 0, ti
        np.testing.assert_allclose(wo, [w[0], -w[1], w[2]], atol=1e-15)
    # just inside the critical angle some light still leaves, grazing
    code, wo, refl, F = O.dielectric(_up(tc - 1e-6), UP, UP, N2, ALMOST_ONE)
    assert F < 1.0 and not refl and code == 0
    assert 0.0 < wo[1] < 2e-3
    # from outside there is no critical angle
    assert O.dielectric(_down(math.radians(89.9)), UP, UP, N2, 0.5)[3] < 1.0


def test_mirror_law_with_a_tilted_normal():
    n = np.array([0.3, 0.9, -0.2])
    n /= np.linalg.norm(n)
    for ti in (0.2, 0.7, 1.2):
        w = _down(ti, 1.1)
        code, wo, refl, F = O.dielectric(w, n, n, N2, 0.0)
        assert code == 0 and refl
        assert abs(np.dot(wo, n) + np.dot(w, n)) < 1e-14      # angle out = angle in
        assert abs(np.dot(np.cross(w, n), wo)) < 1e-14         # in the plane of incidence
        assert abs(np.linalg.norm(wo) - 1.0) < 1e-14


def test_lobe_choice_threshold():
    w = _down(0.9)
    F = O.dielectric(w, UP, UP, N2, 0.5)[3]
    assert 0.0 < F < 1.0
    assert O.dielectric(w, UP, UP, N2, np.nextafter(F, 0.0))[2]
    assert not O.dielectric(w, UP, UP, N2, F)[2]


def test_shading_normal_cases_that_end_the_path():
    # arriving from behind the shading normal although in front of the
    # geometric one: no lobe can be evaluated
    ns = np.array([-math.sin(math.radians(30)), math.cos(math.radians(30)), 0.0])
    w_back = np.array([-math.cos(math.radians(10)), -math.sin(math.radians(10)), 0.0])  # travelling -x, down
    assert np.dot(w_back, UP) < 0 and np.dot(w_back, ns) > 0
    assert O.dielectric(w_back, UP, ns, N2, 0.5)[0] == 7
    # a slightly tilted shading normal mirrors a grazing ray below the
    # geometric surface: the reflection leaves on the wrong side
    ns = np.array([math.sin(math.radians(3)), math.cos(math.radians(3)), 0.0])
    w = np.array([math.cos(math.radians(5)), -math.sin(math.radians(5)), 0.0])
    mirrored = w - 2.0 * np.dot(w, ns) * ns
    assert np.dot(w, ns) < 0 and mirrored[1] < 0
    code, wo, refl, F = O.dielectric(w, UP, ns, N2, 0.0)
    assert refl and code == 8
    np.testing.assert_allclose(wo, mirrored, atol=1e-15)
    # the same ray refracted stays below the surface: valid
    code, wo, refl, F = O.dielectric(w, UP, ns, N2, ALMOST_ONE)
    assert not refl and code == 0 and wo[1] < 0


# ---------------------------------------------------------------- two bounces
def _gl(a, b, n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (b - a) * x + 0.5 * (a + b), 0.5 * (b - a) * w


def _expected_two_bounce_image(sc, nf=8, na=24):
    """E[I^(2)_p] = integral over the film of F(u, p) L2(x(u)) du, where x(u)
    is the wall point seen at film position u and
      L2(x) = rho_w / pi * integral_floor L1(y) cos_y cos_x / |x - y|^2 dA_y,
      L1(y) = rho_f / pi * I0 cos_l(y) / r_l(y)^2
    (radiance leaving the floor after one diffuse reflection of the point
    light; every surface Lambertian; nothing occludes)."""
    cam = sc["camera"]
    W, H = cam["width"], cam["height"]
    t = math.tan(math.radians(cam["fov_deg"]) / 2)
    a = W / H
    c = cam["pos"]
    dist = 1.0 - c[0]  # camera to the wall plane x = 1, along the view axis +x
    rf = sc["albedo"][0].reshape(-1)[0]
    rw = sc["albedo"][1].reshape(-1)[0]
    I0 = sc["Le"][0]
    lp = sc["emitter"]["o"]
    gx, wx = _gl(-1.0, 1.0, na)
    YX, YZ = np.meshgrid(gx, gx, indexing="ij")
    WA = np.outer(wx, wx).ravel()
    YX, YZ = YX.ravel(), YZ.ravel()
    dx, dy, dz = lp[0] - YX, lp[1], lp[2] - YZ
    r2 = dx * dx + dy * dy + dz * dz
    L1 = rf / np.pi * I0 * (dy / np.sqrt(r2)) / r2

    def L2(ux, uy):
        # camera frame: forward +x, right +z, up +y
        qx = (2 * ux / W - 1) * a * t
        qy = (1 - 2 * uy / H) * t
        xy, xz = c[1] + dist * qy, c[2] + dist * qx
        ex = 1.0 - YX[None, :]                    # wall normal (-1, 0, 0) . (y - x)
        ey = xy[:, None]                          # floor normal (0, 1, 0) . (x - y)
        ez = xz[:, None] - YZ[None, :]
        d2 = ex * ex + ey * ey + ez * ez
        return rw / np.pi * ((ex * ey / (d2 * d2)) * L1[None, :] * WA[None, :]).sum(1)

    def axis_nodes(p, n):
        xs, ws = [], []
        for lo, hi in ((p - 0.5, p + 0.5), (p + 0.5, p + 1.5)):
            lo, hi = max(lo, 0.0), min(hi, float(n))
            if hi <= lo:
                continue
            x, w = _gl(lo, hi, nf)
            xs.append(x)
            ws.append(w * np.maximum(0.0, 1.0 - np.abs(x - p - 0.5)))
        return np.concatenate(xs), np.concatenate(ws)

    E = np.zeros((H, W))
    for py in range(H):
        y, wy = axis_nodes(py, H)
        for px in range(W):
            x, wxx = axis_nodes(px, W)
            XX, YY = np.meshgrid(x, y)
            E[py, px] = np.sum(np.outer(wy, wxx).ravel() * L2(XX.ravel(), YY.ravel()))
    return E


def test_two_bounce_diffuse_closed_form():
    sc = scenes.two_plane_point_light_scene()
    E = _expected_two_bounce_image(sc)
    # the quadrature has converged
    E_fine = _expected_two_bounce_image(sc, nf=12, na=40)
    assert np.abs(E_fine - E).max() <= 1e-10 * E.max()
    seeds, n = 24, 1 << 20
    sl = np.stack([O.render(sc, 3000 + s, n, 2, slices=True)["slices"] for s in range(seeds)])
    # the floor is never on the film: the depth-1 slice is the wall's direct light only,
    # and the depth-2 slice is the light -> floor -> wall transport
    img2 = sl[:, 1, :, :, 0]
    mean = img2.mean(0)
    se = img2.std(0, ddof=1) / np.sqrt(seeds)
    assert np.all(se > 0)
    z = (mean - E) / se
    assert 0.5 < np.mean(z * z) < 1.8, np.mean(z * z)
    assert np.max(np.abs(z)) < 5.0
    tot = img2.sum((1, 2))
    z_tot = (tot.mean() - E.sum()) / (tot.std(ddof=1) / np.sqrt(seeds))
    assert abs(z_tot) < 4.0, z_tot
    assert abs(tot.mean() / E.sum() - 1.0) < 0.02
    # grey albedo and intensity: the channels agree
    assert np.array_equal(sl[0, 1, ..., 0], sl[0, 1, ..., 2])
