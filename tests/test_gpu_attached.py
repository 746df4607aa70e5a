"""GPU parity of the attached formulation (heightfield caustic scene).

The GPU's LRB-3-pass attached backward (ray Jacobians by forward-mode duals,
accumulated Jacobian transport, guarded inverse projection; Eq. 4-7,
18-19) is compared with the oracle's generic taped reverse-mode AD of the
whole path (exact).  Where the determinant guard fires, the method drops
terms by design (a singular accumulated Jacobian after a diffuse vertex);
those paths are flagged by the kernel and left out of the replay modes'
comparisons (parity unpinned there), and their share is reported and
bounded.  Paths with an ill-conditioned vertex (grazing hit, short segment,
near-critical refraction, a connection next to a tent-filter kink) are left
out by the oracle's own flag, computed in FP64, and their share is bounded.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2609_32920_amd import lt, scenes

pytestmark = pytest.mark.gpu

TOL = 1e-4


@pytest.fixture(scope="module")
def caustic16():
    from tests.gpu_common import GpuRun
    sc = scenes.caustic_scene(G=16, width=64, height=64)
    return sc, GpuRun(sc)


def _dI(shape, seed=7):
    return np.random.default_rng(seed).normal(size=shape)


def test_caustic_forward_parity(caustic16):
    from tests.gpu_common import matched_paths, maxrel
    sc, g = caustic16
    seed, n, D = 3, 65536, 6
    mask, ids, mis = matched_paths(sc, g, seed, n, D)
    print(f"caustic16 D={D} signature mismatch {mis:.2e}", flush=True)
    assert mis <= 1e-3
    e = maxrel(g.trace(seed, n, D, mask=mask)["image"], O.render(sc, seed, n, D, path_list=ids)["image"])
    print(f"caustic16 image maxrel {e:.2e}", flush=True)
    assert e <= TOL


def test_naive_attached_parity(caustic16):
    # exact chain rule over the attached tape: no inverse, no guard; paths
    # the oracle flags as ill-conditioned are left out
    from tests.gpu_common import matched_paths, maxrel
    sc, g = caustic16
    for seed, D in ((12, 3), (13, 6)):
        n = 65536
        mask, ids, mis, illc = matched_paths(sc, g, seed, n, D, want_illc=True)
        assert mis <= 1e-3
        dI = _dI((64, 64, 3), seed)
        print(f"naive attached D={D}: ill-conditioned paths {illc.mean():.2e}", flush=True)
        assert illc.mean() <= 5e-2
        keep = mask.astype(bool) & ~illc
        ids2 = np.nonzero(keep)[0].astype(np.uint32)
        gg = g.backward("naive", seed, n, D, dI, flags=lt.ATTACHED, mask=keep.astype(np.uint8))
        og = O.gradient(sc, seed, n, D, dI, flags=O.ATTACHED, path_list=ids2)
        eh, ea, el = (maxrel(gg[k], og[k]) for k in ("heights", "albedo", "Le"))
        print(f"naive attached D={D}: heights {eh:.2e} albedo {ea:.2e} Le {el:.2e}", flush=True)
        assert eh <= TOL and ea <= TOL and el <= TOL


def test_attached_parity_without_lds_copies(caustic16):
    """lds_grad = 0: the single albedo texel's gradient goes through each
    wave's write-combining cache (one texel: every scatter hits it) in all
    three attached reverse modes."""
    from tests.gpu_common import matched_paths, maxrel
    sc, g = caustic16
    seed, n, D = 14, 65536, 5
    mask, ids, mis, illc = matched_paths(sc, g, seed, n, D, want_illc=True)
    assert mis <= 1e-3
    dI = _dI((64, 64, 3), seed)
    g.ctx.set_tuning(256, 4, 0)
    try:
        for mode, omode in (("naive", O.MODE_NAIVE), ("lrb3", O.MODE_NAIVE), ("reslrb", O.MODE_RESLRB)):
            keep = mask.astype(bool) & ~illc
            if mode != "naive":
                first = g.backward(mode, seed, n, D, dI, flags=lt.ATTACHED, mask=mask, want_info=True)
                keep &= (first["info"] & 1) == 0
            ids2 = np.nonzero(keep)[0].astype(np.uint32)
            gg = g.backward(mode, seed, n, D, dI, flags=lt.ATTACHED, mask=keep.astype(np.uint8))
            og = O.gradient(sc, seed, n, D, dI, mode=omode, flags=O.ATTACHED, path_list=ids2)
            eh, ea, el = (maxrel(gg[k], og[k]) for k in ("heights", "albedo", "Le"))
            print(f"{mode} attached (no LDS copies): heights {eh:.2e} albedo {ea:.2e} Le {el:.2e}", flush=True)
            assert eh <= TOL and ea <= TOL and el <= TOL, mode
    finally:
        g.ctx.set_tuning()


def test_attached_side_state_sizes(caustic16):
    sc, g = caustic16
    n = 1 << 20
    tape = [g.ctx.side_state_bytes(g.ctx.args(1, n, d, lt.ATTACHED | lt.RECORD_TAPE)) for d in (3, 6, 12)]
    res = [g.ctx.side_state_bytes(g.ctx.args(1, n, d, lt.ATTACHED | lt.RECORD_RESERVOIR)) for d in (3, 6, 12)]
    base = [t - 128 * n * d for t, d in zip(tape, (3, 6, 12))]
    assert base[0] == base[1] == base[2]          # 128 B per vertex: linear in depth
    assert res[0] == res[1] == res[2] == 160 * n  # one record per path: flat in depth


@pytest.mark.parametrize("mode", ["lrb3", "reslrb", "lrb3_fused"])
@pytest.mark.parametrize("D", [3, 4, 6])
def test_replay_attached_parity(caustic16, D, mode):
    """lrb3: the two-kernel LRB-3 with its per-path hand-off (default);
    lrb3_fused: both passes in one kernel (lrb3_split = 0)."""
    sc, g = caustic16
    if mode == "lrb3_fused":
        g.ctx.set_tuning(lrb3_split=0)
        try:
            _replay_attached_parity(sc, g, D, "lrb3")
        finally:
            g.ctx.set_tuning()
    else:
        _replay_attached_parity(sc, g, D, mode)


def _replay_attached_parity(sc, g, D, mode):
    from tests.gpu_common import matched_paths, maxrel
    seed, n = 11, 65536
    mask, ids, mis, illc = matched_paths(sc, g, seed, n, D, want_illc=True)
    assert mis <= 1e-3
    dI = _dI((64, 64, 3), D)
    omode = O.MODE_NAIVE if mode == "lrb3" else O.MODE_RESLRB
    first = g.backward(mode, seed, n, D, dI, flags=lt.ATTACHED, mask=mask, want_info=True)
    guard = (first["info"] & 1).astype(bool)
    frac = guard.mean()
    print(f"{mode} D={D}: guard paths {guard.sum()} ({frac:.2e}), triggers {first['stats']['guard_triggers']}, "
          f"ill-conditioned (oracle) {illc.mean():.2e}", flush=True)
    assert frac <= 1e-2 and illc.mean() <= 5e-2
    keep = mask.astype(bool) & ~guard & ~illc
    ids2 = np.nonzero(keep)[0].astype(np.uint32)
    gg = g.backward(mode, seed, n, D, dI, flags=lt.ATTACHED, mask=keep.astype(np.uint8))
    og = O.gradient(sc, seed, n, D, dI, mode=omode, flags=O.ATTACHED, path_list=ids2)
    eh = maxrel(gg["heights"], og["heights"])
    ea = maxrel(gg["albedo"], og["albedo"])
    el = maxrel(gg["Le"], og["Le"])
    print(f"{mode} D={D}: heights maxrel {eh:.2e}  albedo {ea:.2e}  Le {el:.2e}", flush=True)
    assert ea <= TOL and el <= TOL
    assert eh <= TOL


def fp32_tolerance(sc):
    """Derived bound on max|gpu - ora| / max|ora| for the caustic at full size.

    An FP32 vertex carries a rounding error of a few ulps of the scene
    scale: dx ~ 4 u L with u = 2^-24, L ~ 1.  At the slab top the
    interpolated shading normal turns with the hit point at the rate kappa
    (the change of the central-difference slopes per unit length, a property
    of the heights), so the normal is off by kappa dx.  For near-normal
    incidence the refracted ray turns by (1 - 1/1.5) of that inside the
    glass (path ~0.1) and, after the flat bottom, by 1.5 times as much in air
    (path ~0.5 to the receiver): the receiver point moves by
    0.33 * 0.1 + 0.5 * 0.5 ~ 0.28 times kappa dx, on top of dx itself.  The camera maps that to
    P px per unit (P = W / (2 a tan(fov/2) z_min) for the receiver under the
    slab), and a splat's tent weights, its position derivative with them,
    change by that many pixels times its own value.  With kappa the
    largest slope change per unit over the heightfield and a factor two for
    the unmodelled terms (the emitter leg, the bottom face, wider angles):
        tol = 2 * (1 + 0.28 kappa_max) * 4 u * P.
    On the 16x16 slab kappa_max = 1.4 (the 1e-4 bar holds with room); on the
    rough 128x128 slab it is 134 and on the 224x224 slab 412, where FP32
    conditioning, not the method, sets the agreement."""
    G = int(sc["hf"]["G"])
    h = np.asarray(sc["heights"], np.float64).reshape(G, G)
    dx = 1.0 / (G - 1)
    kap = 0.0
    for hh in (h, h.T):
        S = np.empty_like(hh)
        S[:, 1:-1] = (hh[:, 2:] - hh[:, :-2]) / (2 * dx)
        S[:, 0] = (hh[:, 1] - hh[:, 0]) / dx
        S[:, -1] = (hh[:, -1] - hh[:, -2]) / dx
        kap = max(kap, np.abs(np.diff(S, axis=1)).max() / dx, np.abs(np.diff(S, axis=0)).max() / dx)
    cam = sc["camera"]
    c, t = np.asarray(cam["pos"], np.float64), np.asarray(cam["target"], np.float64)
    f = (t - c) / np.linalg.norm(t - c)
    xs = np.linspace(-0.5, 0.5, 11)
    X, Z = np.meshgrid(xs, xs)
    pts = np.stack([X.ravel(), np.zeros(X.size), Z.ravel()], 1)
    z_min = ((pts - c) @ f).min()
    W, H = cam["width"], cam["height"]
    P = W / (2 * (W / H) * np.tan(np.radians(cam["fov_deg"]) / 2) * z_min)
    return 2 * (1 + 0.28 * kap) * 4 * 2.0 ** -24 * P


# guard_max: the share of sample paths on which the determinant guard may
# fire.  The guard zeroes projections through a numerically singular
# accumulated Jacobian (Sec. 5): after a diffuse vertex (the held local
# direction makes the map rank two) and next to caustic folds, which the
# rougher 224x224 slab (slopes up to 1.3) produces on about a quarter of its
# paths (measured 139 of 511), the 128x128 one on about 4%.
@pytest.mark.parametrize("G,film,n,nsamp,guard_max", [(128, 512, 1 << 24, 2048, 0.06),
                                                       (224, 256, 1 << 20, 512, 0.35)],
                         ids=["G128_full_size", "G224_heights_beyond_lds"])
def test_full_size_caustic_sampled(G, film, n, nsamp, guard_max):
    # 128x128 heightfield, 512x512 film, depth 6, 16M paths (the attached
    # workload at full size, default launch shape; the LRB-3 backward runs
    # 768-thread workgroups with the heights copy in LDS), and a 224x224
    # heightfield whose heights (196 KB) exceed LDS, so the LRB-3 backward
    # keeps 256-thread workgroups and scatters to memory: seeded sample paths
    # kept by the path mask and compared with the oracle on those paths.
    # Left out, with bounded shares: paths whose decisions flip between FP32
    # and FP64, paths the oracle flags as ill-conditioned, and (replay modes
    # only) paths where the kernel's determinant guard fired.
    from tests.gpu_common import GpuRun, mask_of, matched_sample, maxrel
    sc = scenes.caustic_scene(G=G, width=film, height=film)
    TOL_FULL = fp32_tolerance(sc)
    print(f"caustic G={G} film {film}: derived FP32 tolerance {TOL_FULL:.2e}", flush=True)
    g = GpuRun(sc)
    D, seed = 6, 31
    ids = np.sort(np.random.default_rng(3).choice(n, nsamp, replace=False)).astype(np.uint32)
    keep, illc = matched_sample(sc, g, seed, n, D, ids)
    assert len(keep) >= len(ids) - 4
    mask = mask_of(n, keep)
    e_all = maxrel(g.trace(seed, n, D, mask=mask)["image"], O.render(sc, seed, n, D, path_list=keep)["image"])
    # the forward splat position carries the same amplified rounding as the
    # derivatives at an ill-conditioned vertex: compared on the clean paths
    gi = g.trace(seed, n, D, mask=mask_of(n, keep[~illc]))["image"]
    oi = O.render(sc, seed, n, D, path_list=keep[~illc])["image"]
    e = maxrel(gi, oi)
    print(f"caustic G={G} sampled image maxrel {e:.2e} (with ill-conditioned paths {e_all:.2e})", flush=True)
    assert e <= TOL_FULL
    dI = _dI(gi.shape, 9)
    first = g.backward("lrb3", seed, n, D, dI, flags=lt.ATTACHED, mask=mask, want_info=True)
    guard = (first["info"][keep] & 1) != 0
    print(f"caustic G={G}: of {len(keep)} sample paths, ill-conditioned (oracle) {int(illc.sum())}, "
          f"guard (kernel) {int(guard.sum())}", flush=True)
    assert illc.mean() <= 0.05 and guard.mean() <= guard_max
    clean = keep[~illc]
    replay = keep[~illc & ~guard]
    for mode in ("naive", "lrb3", "reslrb"):
        sel = clean if mode == "naive" else replay
        omode = O.MODE_RESLRB if mode == "reslrb" else O.MODE_NAIVE
        ref = O.gradient(sc, seed, n, D, dI, mode=omode, flags=O.ATTACHED, path_list=sel)
        gg = g.backward(mode, seed, n, D, dI, flags=lt.ATTACHED, mask=mask_of(n, sel))
        eh = maxrel(gg["heights"], ref["heights"])
        print(f"caustic G={G} sampled {mode}: heights maxrel {eh:.2e} over {len(sel)} paths", flush=True)
        assert eh <= TOL_FULL, mode


@pytest.mark.parametrize("mode", ["naive", "lrb3", "reslrb"])
def test_normal_mapped_panel_parity(mode):
    """A flat glass panel whose shading comes from a normal map (Sec. 6.1,
    Glass Panel): the forward and the attached gradients with respect to the
    normal-map slopes (through the Jacobians at each refraction) and the
    heights (through the geometry), against the oracle."""
    from tests.gpu_common import GpuRun, matched_paths, maxrel
    sc = scenes.glass_panel_scene(G=16, width=64, height=64)
    g = GpuRun(sc)
    seed, n, D = 23, 65536, 5
    mask, ids, mis, illc = matched_paths(sc, g, seed, n, D, want_illc=True)
    assert mis <= 1e-3 and illc.mean() <= 5e-2
    if mode == "naive":
        e = maxrel(g.trace(seed, n, D, mask=mask)["image"], O.render(sc, seed, n, D, path_list=ids)["image"])
        print(f"panel image maxrel {e:.2e}", flush=True)
        assert e <= TOL
    dI = _dI((64, 64, 3), 5)
    keep = mask.astype(bool) & ~illc
    if mode != "naive":
        first = g.backward(mode, seed, n, D, dI, flags=lt.ATTACHED, mask=mask, want_info=True)
        guard = (first["info"] & 1) != 0
        assert guard.mean() <= 1e-2
        keep &= ~guard
    sel = np.nonzero(keep)[0].astype(np.uint32)
    omode = O.MODE_RESLRB if mode == "reslrb" else O.MODE_NAIVE
    gg = g.backward(mode, seed, n, D, dI, flags=lt.ATTACHED, mask=keep.astype(np.uint8))
    og = O.gradient(sc, seed, n, D, dI, mode=omode, flags=O.ATTACHED, path_list=sel)
    en, eh, ea = (maxrel(gg[k], og[k]) for k in ("normal_map", "heights", "albedo"))
    print(f"panel {mode}: normal map maxrel {en:.2e} heights {eh:.2e} albedo {ea:.2e}", flush=True)
    assert en <= TOL and eh <= TOL and ea <= TOL
