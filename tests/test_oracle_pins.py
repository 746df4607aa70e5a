"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself:
  * published Philox known-answer vectors;
  * the closed-form expected image of a point light over a Lambertian plane
    (importance, normalization, projection and tent filter; Eq. 1, Eq. 20);
  * exact per-seed identities of the gradient: emitter-radiance scaling
    (f_i is linear in L_e, Eq. 2) and Euler homogeneity in the albedo
    (the i-th connection is a degree-i monomial in the albedos, Eq. 2);
  * central finite differences of the loss;
  * the reservoir's selection law and unbiasedness (Eq. 8-10).
"""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_32920_amd import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build(force=False)


def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox_kat.txt")) if not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        ctr, key, want = v[0:4], v[4:6], v[6:10]
        seed = key[0] | (key[1] << 32)
        got = O.philox(seed, ctr)
        assert [int(x) for x in got] == want


def _gauss_legendre(a, b, n=12):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (b - a) * x + 0.5 * (a + b), 0.5 * (b - a) * w


def _expected_point_light_image(sc):
    """E[I_p] = integral over film of F(u, p) * L(x(u)) du, with
    L(x) = rho/pi * I0 cos(theta_l) / r^2 (Lambertian plane y=0, point light).

    The camera looks straight down from (0, h, 0) with up = +z.  Its image
    x axis runs along world -x (right = forward x up) and the image y axis
    (rows, top to bottom) along world -z; film coordinate u maps to the
    plane point x(u) = h * (-qx, 0, qy), qx = (2 u_x / W - 1) a t,
    qy = (1 - 2 u_y / H) t, t = tan(fov/2), a = W/H.
    """
    cam = sc["camera"]
    W, H = cam["width"], cam["height"]
    h = cam["pos"][1]
    t = np.tan(np.radians(cam["fov_deg"]) / 2)
    a = W / H
    rho = sc["albedo"].reshape(-1)[0]
    I0 = sc["Le"][0]
    lp = sc["emitter"]["o"]

    def radiance(ux, uy):
        qx = (2 * ux / W - 1) * a * t
        qy = (1 - 2 * uy / H) * t
        X, Z = -h * qx, h * qy
        dx, dy, dz = lp[0] - X, lp[1], lp[2] - Z
        r2 = dx * dx + dy * dy + dz * dz
        cos_l = dy / np.sqrt(r2)
        return rho / np.pi * I0 * cos_l / r2

    def axis_nodes(p, n):
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
        y, wy = axis_nodes(py, H)
        for px in range(W):
            x, wx = axis_nodes(px, W)
            XX, YY = np.meshgrid(x, y)
            E[py, px] = np.sum(np.outer(wy, wx) * radiance(XX, YY))
    return E


def test_point_light_closed_form():
    sc = scenes.plane_point_light_scene(width=16, height=16)
    E = _expected_point_light_image(sc)
    seeds, n = 16, 1 << 18
    imgs = np.stack([O.render(sc, 1000 + s, n, 1)["image"][..., 0] for s in range(seeds)])
    mean = imgs.mean(0)
    se = imgs.std(0, ddof=1) / np.sqrt(seeds)
    z = (mean - E) / se
    assert np.all(se > 0)
    assert 0.6 < np.mean(z * z) < 1.8, np.mean(z * z)
    assert np.max(np.abs(z)) < 6.0
    # aggregate bias well below one percent
    assert abs(mean.sum() / E.sum() - 1.0) < 3e-3
    # channels are identical for grey albedo and intensity
    img = O.render(sc, 5, 4096, 1)["image"]
    assert np.array_equal(img[..., 0], img[..., 1]) and np.array_equal(img[..., 0], img[..., 2])


def _box_case(width=64, depth=4, n=16384, seed=3):
    sc = scenes.box_scene(width=width, height=width)
    r = O.render(sc, seed, n, depth, slices=True)
    rng = np.random.default_rng(11)
    dI = rng.normal(size=r["image"].shape)
    g = O.gradient(sc, seed, n, depth, dI)
    return sc, r, dI, g


def test_emitter_radiance_scaling_identity():
    # every connection is linear in L_e per channel, so
    # L_e[c] * dJ/dL_e[c] = sum_p dI[p,c] * I[p,c] with J = <dI, I>
    sc, r, dI, g = _box_case()
    lhs = sc["Le"] * g["Le"]
    rhs = np.einsum("hwc,hwc->c", dI, r["image"])
    np.testing.assert_allclose(lhs, rhs, rtol=1e-10, atol=0)


def test_albedo_euler_homogeneity():
    # connection at vertex i carries i albedo factors (i-1 scatter + 1
    # connection BSDF), so sum_k rho_k dJ/drho_k = sum_i i <dI, I^(i)>
    sc, r, dI, g = _box_case()
    lhs = np.einsum("thwc,thwc->c", sc["albedo"], g["albedo"])
    depth = r["slices"].shape[0]
    rhs = sum((i + 1) * np.einsum("hwc,hwc->c", dI, r["slices"][i]) for i in range(depth))
    np.testing.assert_allclose(lhs, rhs, rtol=1e-10, atol=0)
    # the slices partition the image
    np.testing.assert_allclose(r["slices"].sum(0), r["image"], rtol=1e-12, atol=1e-15)


def test_finite_differences_box():
    sc = scenes.box_scene(width=16, height=16)
    seed, n, depth = 21, 2048, 4
    T = O.render(sc, 99, n, depth, albedo=sc["albedo_target"])["image"]

    def loss(alb, le):
        return O.loss_and_adjoint(O.render(sc, seed, n, depth, albedo=alb, Le=le)["image"], T)[0]

    I = O.render(sc, seed, n, depth)["image"]
    _, dI = O.loss_and_adjoint(I, T)
    g = O.gradient(sc, seed, n, depth, dI)
    alb0, le0 = sc["albedo"].copy(), sc["Le"].copy()
    flat = g["albedo"].reshape(-1)
    rng = np.random.default_rng(5)
    idx = np.concatenate([np.argsort(-np.abs(flat))[:10],
                          rng.choice(np.nonzero(flat)[0], 10, replace=False)])
    gmax = np.abs(flat).max()
    h = 1e-5
    for k in idx:
        ap, am = alb0.copy().reshape(-1), alb0.copy().reshape(-1)
        ap[k] += h
        am[k] -= h
        fd = (loss(ap.reshape(alb0.shape), le0) - loss(am.reshape(alb0.shape), le0)) / (2 * h)
        assert abs(fd - flat[k]) <= 1e-6 * gmax, (k, fd, flat[k])
    for c in range(3):
        lp, lm = le0.copy(), le0.copy()
        lp[c] += h * le0[c]
        lm[c] -= h * le0[c]
        fd = (loss(alb0, lp) - loss(alb0, lm)) / (2 * h * le0[c])
        assert abs(fd - g["Le"][c]) <= 1e-7 * abs(g["Le"][c]) + 1e-12


def test_reservoir_threshold_and_law():
    # replacement iff u < w_i / Omega_i: first valid candidate always kept
    below = np.nextafter(0.7, 0) - 2.0 ** -24
    R, W = O.reservoir([0.3, 0.7], [0.99, 0.7 - 2.0 ** -24])
    assert R == 2 and abs(W - 1.0 / 0.7) < 1e-12
    R, W = O.reservoir([0.3, 0.7], [0.0, 0.7])
    assert R == 1 and abs(W - 1.0 / 0.3) < 1e-12
    assert below < 0.7
    # zero weights are never candidates
    assert O.reservoir([0.0, 0.0], [0.1, 0.1])[0] == 0
    # chi-square of the selection law Pr(R = i) = w_i / Omega_k
    w = np.array([0.5, 2.0, 0.0, 1.0, 3.5, 0.25])
    rng = np.random.default_rng(7)
    n = 120000
    u = np.floor(rng.uniform(size=(n, len(w))) * 2 ** 24) / 2 ** 24
    counts = np.zeros(len(w) + 1)
    Lrgb = rng.uniform(0.1, 1.0, size=(len(w), 3))
    est = np.zeros((n, 3))
    for k in range(n):
        R, Wr = O.reservoir(w, u[k])
        counts[R] += 1
        est[k] = Wr * Lrgb[R - 1]
    p = w / w.sum()
    expected = n * p
    nz = p > 0
    chi2 = np.sum((counts[1:][nz] - expected[nz]) ** 2 / expected[nz])
    assert counts[0] == 0 and counts[3] == 0
    assert chi2 < 25.0  # 4 dof, p ~ 5e-5
    # Eq. 10: the reweighted selection (Omega/w_R) L_R is unbiased for the
    # sum of the candidates' L_i (zero-weight candidates never enter)
    want = (Lrgb * (w > 0)[:, None]).sum(0)
    se = est.std(0, ddof=1) / np.sqrt(n)
    assert np.all(np.abs(est.mean(0) - want) < 4.5 * se), (est.mean(0), want, se)


def test_reservoir_estimator_unbiased_in_scene():
    # Eq. 10 at scene level: the image that splats only (Omega/w_R) L_R has
    # the same expectation as the full light-tracing image
    sc = scenes.box_scene(width=32, height=32)
    d = []
    for s in range(12):
        full = O.render(sc, 500 + s, 8192, 4)["flux"]
        sel = O.render(sc, 500 + s, 8192, 4, flags=O.SPLAT_SELECTED)["flux"]
        d.append(sel - full)
    d = np.array(d)
    z = d.mean(0) / (d.std(0, ddof=1) / np.sqrt(len(d)))
    assert np.all(np.abs(z) < 4.5), z


def test_reservoir_estimator_mean_of_selection():
    # E_R[(Omega_k / w_R) L_R] = sum_i L_i (Eq. 10), by exact enumeration
    w = np.array([0.2, 1.3, 0.7])
    L = np.array([[0.1, 0.2, 0.3], [1.0, 0.5, 0.2], [0.4, 0.4, 0.9]])
    Om = w.sum()
    exp = sum((w[i] / Om) * (Om / w[i]) * L[i] for i in range(3))
    np.testing.assert_allclose(exp, L.sum(0), rtol=1e-14)


def test_single_connection_paths_make_reslrb_exact():
    # with at most one connection per path (D = 1), R is that connection and
    # Omega/w_R = 1, so the ResLRB gradient equals the naive gradient per seed
    sc = scenes.plane_point_light_scene(width=16, height=16)
    r = O.render(sc, 9, 8192, 1, per_path=True)
    assert np.all(r["W"][r["R"] > 0] == 1.0)
    dI = np.random.default_rng(2).normal(size=r["image"].shape)
    gn = O.gradient(sc, 9, 8192, 1, dI, mode=O.MODE_NAIVE)
    gr = O.gradient(sc, 9, 8192, 1, dI, mode=O.MODE_RESLRB)
    np.testing.assert_allclose(gr["albedo"], gn["albedo"], rtol=1e-13)
    np.testing.assert_allclose(gr["Le"], gn["Le"], rtol=1e-13)


def test_flux_conservation_of_tent_splat():
    # tent taps form a partition of unity: with every splat >= 1.5 px inside
    # the film, the image sums to the total connection flux
    sc = scenes.plane_point_light_scene(width=16, height=16)
    v = sc["tri_v"].copy()
    v[..., 0] = np.clip(v[..., 0], -0.3, 0.3)
    v[..., 2] = np.clip(v[..., 2], -0.3, 0.3)
    sc["tri_v"] = v
    r = O.render(sc, 4, 20000, 1)
    assert r["flux"][0] > 0
    np.testing.assert_allclose(r["image"].sum((0, 1)), r["flux"], rtol=1e-12)


def test_path_list_is_a_partition():
    sc = scenes.box_scene(width=32, height=32)
    n = 4096
    full = O.render(sc, 8, n, 4)["image"]
    ids = np.arange(n, dtype=np.uint32)
    a = O.render(sc, 8, n, 4, path_list=ids[::2])["image"]
    b = O.render(sc, 8, n, 4, path_list=ids[1::2])["image"]
    np.testing.assert_allclose(a + b, full, rtol=1e-12, atol=1e-15)


def test_reslrb_gradient_unbiased_vs_naive():
    # E[ResLRB gradient] = naive gradient (Eq. 10-11), same fixed dI
    sc = scenes.box_scene(width=16, height=16)
    dI = np.random.default_rng(3).normal(size=(16, 16, 3))
    gn, gr = [], []
    for s in range(24):
        gn.append(O.gradient(sc, 700 + s, 4096, 4, dI)["Le"])
        gr.append(O.gradient(sc, 700 + s, 4096, 4, dI, mode=O.MODE_RESLRB)["Le"])
    d = np.array(gr) - np.array(gn)
    z = d.mean(0) / (d.std(0, ddof=1) / np.sqrt(len(d)))
    assert np.all(np.abs(z) < 4.5), z
    # the two estimators are different per seed (several candidates per path)
    assert np.max(np.abs(d)) > 0
    r = O.render(sc, 700, 4096, 4, per_path=True)
    assert np.mean(r["W"][r["R"] > 0] > 1.0) > 0.3


def test_finite_differences_heights_attached():
    # attached gradients w.r.t. heightfield heights (Sec. 3.3): every vertex
    # position, normal, refraction, projection and tent weight is an AD
    # expression of the heights; checked against central differences with
    # the decision signatures equal at +h and -h
    sc = scenes.caustic_scene(G=8, width=32, height=32)
    seed, n, D = 5, 4096, 4
    T = O.render(sc, 99, n, D, heights=sc["heights_target"])["image"]
    r0 = O.render(sc, seed, n, D, per_path=True)
    _, dI = O.loss_and_adjoint(r0["image"], T)
    gh = O.gradient(sc, seed, n, D, dI, flags=O.ATTACHED)["heights"]
    assert np.count_nonzero(gh) > 20
    h0 = sc["heights"].copy()
    eps = 1e-7
    checked = 0
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
    assert checked >= 8
    # detached mode leaves the heights alone
    assert O.gradient(sc, seed, n, D, dI)["heights"] is None or not np.any(
        O.gradient(sc, seed, n, D, dI)["heights"])


def test_caustic_reslrb_equals_naive_with_single_connections():
    # at depth 3 a caustic path connects at most once (receiver), so the
    # reservoir always keeps that connection with weight 1 and the attached
    # ResLRB gradient equals the attached naive gradient per seed
    sc = scenes.caustic_scene(G=8, width=32, height=32)
    r = O.render(sc, 6, 4096, 3, per_path=True)
    assert np.all(r["W"][r["R"] > 0] == 1.0)
    dI = np.random.default_rng(4).normal(size=r["image"].shape)
    gn = O.gradient(sc, 6, 4096, 3, dI, flags=O.ATTACHED)
    gr = O.gradient(sc, 6, 4096, 3, dI, mode=O.MODE_RESLRB, flags=O.ATTACHED)
    np.testing.assert_allclose(gr["heights"], gn["heights"], rtol=1e-12, atol=1e-15)
