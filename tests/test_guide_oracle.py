"""Pins of the oracle's learned emission guide against facts other than itself.

  * the network equals a plain PyTorch CPU network with the same weights,
    exactly in float64 and, with bfloat16 operands, up to the rare double
    rounding of torch's float64 -> float32 -> bfloat16 conversion;
  * the folded mixture density integrates to one over the emitting
    hemisphere (product Gauss-Legendre quadrature);
  * the sampler draws from that density (binned chi-square, and the share of
    the cosine component is 1 - alpha);
  * the training-loss gradient equals central finite differences;
  * Adam equals torch.optim.Adam;
  * the guided light tracer is unbiased: its mean image over seeds matches
    the cosine-emission tracer's within sampling error, and its albedo
    gradient equals finite differences of the guided image;
  * the diffuse guide table: texel centres lie where an independent affine
    fit of each quad's chart puts them, entries are the network at both
    sides, alpha = 0 reduces it to cosine sampling, the guided tracer
    (emission and diffuse vertices) stays unbiased, its albedo and attached
    heights gradients equal finite differences, and the training samples'
    S add up to the flux of the later connections.
"""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2609_32920_amd import scenes


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build(force=False)


def _split(w):
    shapes = ((64, 6), (64, 64), (64, 64), (41, 64))
    out, k = [], 0
    for n_out, n_in in shapes:
        W = w[k:k + n_out * n_in].reshape(n_out, n_in); k += n_out * n_in
        b = w[k:k + n_out]; k += n_out
        out.append((torch.tensor(W), torch.tensor(b)))
    assert k == w.size
    return out


def _torch_net(w, feats, bf16):
    def r(t):
        return t.to(torch.float32).to(torch.bfloat16).to(torch.float64) if bf16 else t
    h = torch.tensor(feats)
    layers = _split(w)
    for i, (W, b) in enumerate(layers):
        h = torch.nn.functional.linear(r(h), r(W), b)
        if i < 3:
            h = torch.relu(h)
    return h.numpy()


def _features(sc, x, n):
    tv = sc["tri_v"].reshape(-1, 3)
    em = sc["emitter"]
    o, e1, e2 = (np.asarray(em[k]) for k in ("o", "e1", "e2"))
    pts = np.vstack([tv, o, o + e1, o + e2, o + e1 + e2])
    lo, hi = pts.min(0), pts.max(0)
    c, h = 0.5 * (lo + hi), 0.5 * (hi - lo)
    return np.hstack([(x - c) / h, n])


def _rand_inputs(sc, count, seed):
    rng = np.random.default_rng(seed)
    tv = sc["tri_v"].reshape(-1, 3)
    x = rng.uniform(tv.min(0), tv.max(0), size=(count, 3))
    n = rng.normal(size=(count, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    return x, n


def test_network_matches_torch():
    sc = scenes.box_scene()
    w = scenes.guide_random_weights(3)
    x, n = _rand_inputs(sc, 500, 1)
    feats = _features(sc, x, n)
    got = O.guide_eval(sc, w, x, n, bf16=False)
    want = _torch_net(w, feats, False)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)
    got = O.guide_eval(sc, w, x, n, bf16=True)
    want = _torch_net(w, feats, True)
    err = np.abs(got - want).max(axis=1)
    scale = np.abs(want).max()
    # exact unless a float64 value sat within 2^-24 of a bfloat16 tie
    assert np.mean(err <= 1e-12 * scale) >= 0.97, np.mean(err <= 1e-12 * scale)
    assert err.max() <= 2e-2 * scale


def _raw_outputs(count, seed, logk=(-3.0, 6.0)):
    rng = np.random.default_rng(seed)
    o = rng.normal(size=(count, 41))
    o[:, 3:40:5] = rng.uniform(*logk, size=(count, 8))
    o[:, 4:40:5] *= 2.0
    return o


def _hemisphere_grid(n, nt=1200, npf=2400):
    """Product Gauss-Legendre (cos theta) x midpoint (phi) rule about n."""
    ct, wt = np.polynomial.legendre.leggauss(nt)
    ct, wt = 0.5 * (ct + 1.0), 0.5 * wt
    phi = (np.arange(npf) + 0.5) * (2 * math.pi / npf)
    C, P = np.meshgrid(ct, phi, indexing="ij")
    S = np.sqrt(1 - C * C)
    a = np.array([1.0, 0.0, 0.0]) if abs(n[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    t1 = np.cross(n, a); t1 /= np.linalg.norm(t1)
    t2 = np.cross(n, t1)
    d = (S * np.cos(P))[..., None] * t1 + (S * np.sin(P))[..., None] * t2 + C[..., None] * n
    wq = (wt[:, None] * np.full(npf, 2 * math.pi / npf)[None, :])
    return d.reshape(-1, 3), wq.reshape(-1)


def test_mixture_density_normalised():
    o = _raw_outputs(4, 11)
    rng = np.random.default_rng(5)
    for i in range(o.shape[0]):
        n = rng.normal(size=3); n /= np.linalg.norm(n)
        d, wq = _hemisphere_grid(n)
        pdf = O.guide_pdf(np.repeat(o[i:i + 1], d.shape[0], 0), np.repeat(n[None], d.shape[0], 0), d)
        assert abs(np.sum(pdf * wq) - 1.0) < 2e-4, np.sum(pdf * wq)
    # below the emitting hemisphere the density is zero
    pdf = O.guide_pdf(o[:1], np.array([[0.0, 0.0, 1.0]]), np.array([[0.0, 0.6, -0.8]]))
    assert pdf[0] == 0.0


def test_sampler_matches_density():
    from scipy import stats
    o = _raw_outputs(3, 21, logk=(-1.0, 3.0))
    rng = np.random.default_rng(9)
    nb_t, nb_p, N = 16, 32, 400_000
    for i in range(o.shape[0]):
        n = rng.normal(size=3); n /= np.linalg.norm(n)
        g = rng.uniform(size=(N, 3))
        d, comp = O.guide_sample(np.repeat(o[i:i + 1], N, 0), np.repeat(n[None], N, 0), g)
        assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-12)
        assert np.all(d @ n >= -1e-15)
        alpha = 0.9 / (1 + math.exp(-o[i, 40]))
        share = np.mean(comp == 0)
        assert abs(share - (1 - alpha)) < 5 * math.sqrt(alpha * (1 - alpha) / N)
        # equal-solid-angle bins in (cos theta, phi) about n
        a = np.array([1.0, 0.0, 0.0]) if abs(n[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
        t1 = np.cross(n, a); t1 /= np.linalg.norm(t1)
        t2 = np.cross(n, t1)
        ct = np.clip(d @ n, 0, 1 - 1e-15)
        ph = np.mod(np.arctan2(d @ t2, d @ t1), 2 * math.pi)
        bi = np.minimum((ct * nb_t).astype(int), nb_t - 1) * nb_p + np.minimum((ph / (2 * math.pi) * nb_p).astype(int), nb_p - 1)
        counts = np.bincount(bi, minlength=nb_t * nb_p)
        # expected mass per bin by a 6 x 6 Gauss-Legendre rule inside each bin
        x6, w6 = np.polynomial.legendre.leggauss(6)
        cts = ((np.arange(nb_t)[:, None] + 0.5 * (x6[None] + 1)) / nb_t).reshape(-1)
        phs = ((np.arange(nb_p)[:, None] + 0.5 * (x6[None] + 1)) * (2 * math.pi / nb_p)).reshape(-1)
        C, P = np.meshgrid(cts, phs, indexing="ij")
        S = np.sqrt(1 - C * C)
        dirs = (S * np.cos(P))[..., None] * t1 + (S * np.sin(P))[..., None] * t2 + C[..., None] * n
        pdf = O.guide_pdf(np.repeat(o[i:i + 1], dirs.size // 3, 0), np.repeat(n[None], dirs.size // 3, 0),
                          dirs.reshape(-1, 3)).reshape(nb_t, 6, nb_p, 6)
        wt = np.einsum("i,j->ij", w6, w6) * (0.5 / nb_t) * (0.5 * 2 * math.pi / nb_p)
        mass = np.einsum("aibj,ij->ab", pdf, wt).reshape(-1)
        assert abs(mass.sum() - 1) < 1e-3
        exp = mass * N
        keep = exp > 5
        chi2 = np.sum((counts[keep] - exp[keep]) ** 2 / exp[keep])
        p = stats.chi2.sf(chi2, keep.sum() - 1)
        assert p > 1e-4, (i, chi2, keep.sum(), p)


def test_loss_gradient_matches_finite_differences():
    sc = scenes.box_scene()
    w = scenes.guide_random_weights(4, scale=0.7)
    smp = scenes.guide_sample_batch(sc, 48, 12)
    L0, g = O.guide_loss_grad(sc, w, smp, bf16=False)
    assert np.isfinite(L0) and np.any(g != 0)
    rng = np.random.default_rng(2)
    # every bias and weight block, random entries of each
    idx = np.concatenate([rng.choice(np.arange(a, b), 25, replace=False) for a, b in
                          ((0, 384), (384, 448), (448, 4544), (4544, 4608), (4608, 8704),
                           (8704, 8768), (8768, 11392), (11392, 11433))])
    ok = 0
    for i in idx:
        h = 1e-6 * max(1.0, abs(w[i]))
        wp, wm = w.copy(), w.copy()
        wp[i] += h; wm[i] -= h
        fd = (O.guide_loss_grad(sc, wp, smp, bf16=False)[0] - O.guide_loss_grad(sc, wm, smp, bf16=False)[0]) / (2 * h)
        if abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-7:
            ok += 1
    # a handful may straddle a ReLU kink or a clamp edge
    assert ok >= 0.97 * len(idx), (ok, len(idx))


def test_adam_matches_torch():
    rng = np.random.default_rng(0)
    w0 = rng.normal(size=50)
    grads = [rng.normal(size=50) for _ in range(4)]
    p = torch.nn.Parameter(torch.tensor(w0))
    opt = torch.optim.Adam([p], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    w, m, v = w0.copy(), np.zeros(50), np.zeros(50)
    for t, g in enumerate(grads, start=1):
        p.grad = torch.tensor(g)
        opt.step()
        w, m, v = O.adam(w, g, m, v, t, 3e-3)
    np.testing.assert_allclose(w, p.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_emission_uses_counter_uniforms():
    sc = scenes.box_scene()
    w = scenes.guide_random_weights(6)
    seed, n = 77, 64
    e = O.guide_emit(sc, seed, n, w)
    em = sc["emitter"]
    o, e1, e2 = (np.asarray(em[k]) for k in ("o", "e1", "e2"))
    nrm = np.cross(e1, e2); area = np.linalg.norm(nrm); nrm /= area
    u = np.array([O.philox(seed, (p, 0, 0, 0)) for p in range(n)]) >> 8
    g = np.array([O.philox(seed, (p, 0, 1, 0)) for p in range(n)]) >> 8
    u, g = u * 2.0 ** -24, g[:, :3] * 2.0 ** -24
    x = o + u[:, :1] * e1 + u[:, 1:2] * e2
    np.testing.assert_allclose(e["x"], x, rtol=0, atol=1e-15)
    raw = O.guide_eval(sc, w, x, np.repeat(nrm[None], n, 0))
    d, comp = O.guide_sample(raw, np.repeat(nrm[None], n, 0), g)
    np.testing.assert_array_equal(e["comp"], comp)
    np.testing.assert_allclose(e["w"], d, rtol=0, atol=1e-15)
    pdf = O.guide_pdf(raw, np.repeat(nrm[None], n, 0), d)
    np.testing.assert_allclose(e["factor"], area * (d @ nrm) / pdf, rtol=1e-14)
    assert len(set(comp.tolist())) > 3


def _blocks(img, k=4):
    H, W, _ = img.shape
    return img.reshape(k, H // k, k, W // k, 3).sum(axis=(1, 3)).reshape(-1)


def test_guided_tracer_unbiased():
    sc = scenes.box_scene(width=32, height=32)
    w = scenes.guide_random_weights(8)
    seeds, n = 24, 6000
    gs = np.array([_blocks(O.render(sc, 1000 + s, n, 4, guide_w=w)["image"]) for s in range(seeds)])
    us = np.array([_blocks(O.render(sc, 5000 + s, n, 4)["image"]) for s in range(seeds)])
    diff = gs.mean(0) - us.mean(0)
    se = np.sqrt(gs.var(0, ddof=1) / seeds + us.var(0, ddof=1) / seeds)
    z = diff / se
    assert np.max(np.abs(z)) < 4.5, np.max(np.abs(z))
    # the guide really changes the estimator: guided emission is not cosine
    e = O.guide_emit(sc, 3, 2000, w)
    assert np.std(e["factor"]) > 0.05 * np.mean(e["factor"])


def test_guided_gradient_matches_finite_differences():
    sc = scenes.box_scene(width=16, height=16, tex_res=4)
    w = scenes.guide_random_weights(8)
    seed, n, D = 3, 3000, 3
    T = O.render(sc, 99, 20000, D, albedo=sc["albedo_target"])["image"]
    I = O.render(sc, seed, n, D, guide_w=w)["image"]
    _, dI = O.loss_and_adjoint(I, T)
    g = O.gradient(sc, seed, n, D, dI, guide_w=w)
    rng = np.random.default_rng(1)
    alb = sc["albedo"]
    flat = alb.reshape(-1)
    for i in rng.choice(flat.size, 6, replace=False):
        h = 1e-5
        ap, am = flat.copy(), flat.copy()
        ap[i] += h; am[i] -= h
        Ip = O.render(sc, seed, n, D, albedo=ap.reshape(alb.shape), guide_w=w)["image"]
        Im = O.render(sc, seed, n, D, albedo=am.reshape(alb.shape), guide_w=w)["image"]
        fd = np.sum(dI * (Ip - Im)) / (2 * h)
        assert abs(fd - g["albedo"].reshape(-1)[i]) <= 1e-6 * max(1e-3, abs(fd)), (i, fd, g["albedo"].reshape(-1)[i])
    fdl = []
    for c in range(3):
        lp, lm = sc["Le"].copy(), sc["Le"].copy()
        lp[c] += 1e-5; lm[c] -= 1e-5
        Ip = O.render(sc, seed, n, D, Le=lp, guide_w=w)["image"]
        Im = O.render(sc, seed, n, D, Le=lm, guide_w=w)["image"]
        fdl.append(np.sum(dI * (Ip - Im)) / 2e-5)
    np.testing.assert_allclose(g["Le"], fdl, rtol=1e-6)


def test_guided_attached_heights_match_finite_differences():
    # guided emission leaves the attached derivative structure alone: the
    # emitted direction is fixed in world space and its density is held
    # fixed, so the heights gradient of the guided estimator is the
    # derivative of the guided image (central differences, equal signatures)
    sc = scenes.caustic_scene(G=8, width=32, height=32)
    w = scenes.guide_aimed_weights()
    seed, n, D = 5, 4096, 4
    T = O.render(sc, 99, n, D, heights=sc["heights_target"])["image"]
    r0 = O.render(sc, seed, n, D, per_path=True, guide_w=w)
    _, dI = O.loss_and_adjoint(r0["image"], T)
    gh = O.gradient(sc, seed, n, D, dI, flags=O.ATTACHED, guide_w=w)["heights"]
    assert np.count_nonzero(gh) > 20
    h0 = sc["heights"].copy()
    eps, checked = 1e-7, 0
    for k in np.argsort(-np.abs(gh))[:12]:
        hp, hm = h0.copy(), h0.copy()
        hp[k] += eps
        hm[k] -= eps
        rp = O.render(sc, seed, n, D, heights=hp, per_path=True, guide_w=w)
        rm = O.render(sc, seed, n, D, heights=hm, per_path=True, guide_w=w)
        if not (np.array_equal(rp["sig"], r0["sig"]) and np.array_equal(rm["sig"], r0["sig"])):
            continue
        fd = (O.loss_and_adjoint(rp["image"], T)[0] - O.loss_and_adjoint(rm["image"], T)[0]) / (2 * eps)
        assert abs(fd - gh[k]) <= 1e-5 * np.abs(gh).max(), (k, fd, gh[k])
        checked += 1
    assert checked >= 8


# ----------------------------------------------------------------- diffuse guide
def _quad_affine(sc, tex):
    """Least-squares affine map chart (u, v, 1) -> position over the
    triangles of texture `tex` (a planar quad), and their unit normal."""
    rows, pos = [], []
    for t in range(sc["tri_v"].shape[0]):
        m = sc["tri_mat"][t]
        if sc["mat_type"][m] != scenes.MAT_LAMBERT or sc["mat_tex"][m] != tex:
            continue
        for k in range(3):
            rows.append([*sc["tri_uv"][t, k], 1.0])
            pos.append(sc["tri_v"][t, k])
        e1 = sc["tri_v"][t, 1] - sc["tri_v"][t, 0]
        e2 = sc["tri_v"][t, 2] - sc["tri_v"][t, 0]
        nrm = np.cross(e1, e2)
    M, *_ = np.linalg.lstsq(np.array(rows), np.array(pos), rcond=None)
    return M, nrm / np.linalg.norm(nrm)


def test_texel_centres_on_the_quads():
    sc = scenes.box_scene(width=16, height=16, tex_res=4)
    t = O.guide_table(sc, scenes.guide_random_weights(2))
    R = sc["tex_res"]
    assert t["ok"].all()
    for tex in range(sc["n_tex"]):
        M, nrm = _quad_affine(sc, tex)
        for ty in range(R):
            for tx in range(R):
                k = (tex * R + ty) * R + tx
                want = np.array([(tx + 0.5) / R, (ty + 0.5) / R, 1.0]) @ M
                np.testing.assert_allclose(t["x"][k], want, atol=1e-12)
                np.testing.assert_allclose(t["n"][k], nrm, atol=1e-12)


def test_guide_table_entries_are_the_network_at_both_sides():
    sc = scenes.box_scene(width=16, height=16, tex_res=4)
    w = scenes.guide_random_weights(3)
    t = O.guide_table(sc, w)
    raw0 = O.guide_eval(sc, w, t["x"], t["n"])
    raw1 = O.guide_eval(sc, w, t["x"], -t["n"])
    np.testing.assert_array_equal(t["raw"][0::2], raw0)
    np.testing.assert_array_equal(t["raw"][1::2], raw1)
    assert np.abs(raw0 - raw1).max() > 1e-3   # the normal input matters


def _cosine_only(w):
    w = np.array(w, np.float64)
    w[-1] = -1e3          # mixing logit: alpha = 0.9 sigmoid(-1000) = 0
    return w


def test_diffuse_guide_with_zero_alpha_is_cosine_sampling():
    # alpha = 0 leaves only the cosine component: the same directions (from
    # the same two uniforms) and weight cos / (pi cos / pi) = 1
    sc = scenes.box_scene(width=16, height=16, tex_res=4)
    w = _cosine_only(scenes.guide_random_weights(4))
    a = O.render(sc, 5, 4000, 5, per_path=True)
    b = O.render(sc, 5, 4000, 5, per_path=True, guide_w=w, guide_diffuse=True)
    c = O.render(sc, 5, 4000, 5, per_path=True, guide_w=w)
    np.testing.assert_array_equal(b["sig"], c["sig"])
    np.testing.assert_allclose(b["image"], c["image"], rtol=1e-12, atol=1e-12 * c["image"].max())
    assert np.abs(a["image"] - c["image"]).max() > 0   # the emission guide itself is on


def _aimed_up(logk=2.5):
    return scenes.guide_aimed_weights(direction=(0.0, 1.0, 0.3), logk=logk, spread=0.2)


def test_diffuse_guided_tracer_unbiased():
    sc = scenes.box_scene(width=32, height=32)
    w = _aimed_up()
    seeds, n = 24, 6000
    gs = np.array([_blocks(O.render(sc, 1000 + s, n, 4, guide_w=w, guide_diffuse=True)["image"])
                   for s in range(seeds)])
    us = np.array([_blocks(O.render(sc, 5000 + s, n, 4)["image"]) for s in range(seeds)])
    diff = gs.mean(0) - us.mean(0)
    se = np.sqrt(gs.var(0, ddof=1) / seeds + us.var(0, ddof=1) / seeds)
    z = diff / se
    assert np.max(np.abs(z)) < 4.5, np.max(np.abs(z))
    # the diffuse guide really changes the estimator: its samples are not
    # cosine distributed (q differs from cos / pi)
    smp = O.guide_vertex_samples(sc, 3, 2000, 4, w)
    on = smp[:, 9] > 0
    assert on.mean() > 0.3
    cosq = np.einsum("ij,ij->i", smp[on, 3:6], smp[on, 6:9]) / math.pi
    assert np.std(cosq / smp[on, 9]) > 0.1 * np.mean(cosq / smp[on, 9])


def test_diffuse_guided_gradient_matches_finite_differences():
    sc = scenes.box_scene(width=16, height=16, tex_res=4)
    w = _aimed_up()
    seed, n, D = 3, 3000, 4
    T = O.render(sc, 99, 20000, D, albedo=sc["albedo_target"])["image"]
    I = O.render(sc, seed, n, D, guide_w=w, guide_diffuse=True)["image"]
    _, dI = O.loss_and_adjoint(I, T)
    g = O.gradient(sc, seed, n, D, dI, guide_w=w, guide_diffuse=True)
    rng = np.random.default_rng(1)
    alb = sc["albedo"]
    flat = alb.reshape(-1)
    for i in rng.choice(flat.size, 6, replace=False):
        h = 1e-5
        ap, am = flat.copy(), flat.copy()
        ap[i] += h; am[i] -= h
        Ip = O.render(sc, seed, n, D, albedo=ap.reshape(alb.shape), guide_w=w, guide_diffuse=True)["image"]
        Im = O.render(sc, seed, n, D, albedo=am.reshape(alb.shape), guide_w=w, guide_diffuse=True)["image"]
        fd = np.sum(dI * (Ip - Im)) / (2 * h)
        assert abs(fd - g["albedo"].reshape(-1)[i]) <= 1e-6 * max(1e-3, abs(fd)), (i, fd, g["albedo"].reshape(-1)[i])


def test_diffuse_guided_attached_heights_match_finite_differences():
    # the caustic's diffuse vertices lie on the static receiver: the guided
    # direction there does not move with the heights, so the attached
    # gradient is the derivative of the guided image
    sc = scenes.caustic_scene(G=8, width=32, height=32)
    w = scenes.guide_aimed_weights()
    seed, n, D = 5, 4096, 4
    T = O.render(sc, 99, n, D, heights=sc["heights_target"])["image"]
    kw = dict(guide_w=w, guide_diffuse=True)
    r0 = O.render(sc, seed, n, D, per_path=True, **kw)
    _, dI = O.loss_and_adjoint(r0["image"], T)
    gh = O.gradient(sc, seed, n, D, dI, flags=O.ATTACHED, **kw)["heights"]
    assert np.count_nonzero(gh) > 20
    h0 = sc["heights"].copy()
    eps, checked = 1e-7, 0
    for k in np.argsort(-np.abs(gh))[:12]:
        hp, hm = h0.copy(), h0.copy()
        hp[k] += eps
        hm[k] -= eps
        rp = O.render(sc, seed, n, D, heights=hp, per_path=True, **kw)
        rm = O.render(sc, seed, n, D, heights=hm, per_path=True, **kw)
        if not (np.array_equal(rp["sig"], r0["sig"]) and np.array_equal(rm["sig"], r0["sig"])):
            continue
        fd = (O.loss_and_adjoint(rp["image"], T)[0] - O.loss_and_adjoint(rm["image"], T)[0]) / (2 * eps)
        assert abs(fd - gh[k]) <= 1e-5 * np.abs(gh).max(), (k, fd, gh[k])
        checked += 1
    assert checked >= 6


def test_diffuse_vertex_samples_follow_the_paths():
    # the sample's S is the luminance of the path's connections after the
    # sampled vertex: summed over paths it is the flux of the depth >= 2
    # slices of paths whose first scatter is guided (every box path is)
    sc = scenes.box_scene(width=16, height=16, tex_res=4)
    w = _aimed_up()
    seed, n, D = 8, 3000, 4
    smp = O.guide_vertex_samples(sc, seed, n, D, w)
    kw = dict(guide_w=w, guide_diffuse=True)
    lum = np.array([0.2126, 0.7152, 0.0722])
    on = smp[:, 9] > 0
    assert on.mean() > 0.5
    # every box path that scatters does so first at x_1 (a Lambertian wall),
    # so the samples' S add up to the flux of the connections at depth >= 2:
    # the flux at depth D minus the flux at depth 1 of the same paths
    f_all = O.render(sc, seed, n, D, **kw)["flux"]
    f_one = O.render(sc, seed, n, 1, **kw)["flux"]
    np.testing.assert_allclose(smp[:, 10].sum(), lum @ (f_all - f_one), rtol=1e-9)
    np.testing.assert_allclose(np.linalg.norm(smp[on, 3:6], axis=1), 1.0, atol=1e-12)
    np.testing.assert_allclose(np.linalg.norm(smp[on, 6:9], axis=1), 1.0, atol=1e-12)
    assert (np.einsum("ij,ij->i", smp[on, 3:6], smp[on, 6:9]) > 0).all()
