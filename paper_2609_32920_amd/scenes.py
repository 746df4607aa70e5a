"""Seeded synthetic scene generators.

This module only *describes* inputs: triangle lists, material tables, texture
and height parameters, emitter and camera placement, and loss targets drawn
from fixed seeds.  It holds none of the light-transport arithmetic; both the
HIP library and the CPU oracle consume the arrays it returns and implement the
method on their own.

Scene dictionary layout (all arrays numpy, float64 unless noted):
  tri_v    [T,3,3]  world-space triangle vertices (static geometry)
  tri_uv   [T,3,2]  per-vertex chart/texture coordinates
  tri_mat  [T]      int32 material index
  mat_type [M]      int32: MAT_ABSORBER, MAT_LAMBERT, MAT_DIELECTRIC, MAT_CONDUCTOR
  mat_tex  [M]      int32 texture index of a Lambertian material (its albedo) or a
                    conductor (its reflectance F0); -1 otherwise
  mat_ior  [M]      refractive index of a dielectric, GGX roughness of a conductor
  n_tex, tex_res    albedo textures are [n_tex, tex_res, tex_res, 3]
  emitter  dict(type=EMIT_QUAD|EMIT_POINT|EMIT_DIRECTIONAL, o, e1, e2[, tex_res])
           (point: o = position; directional: a collimated beam leaving the
           quad along normalize(e1 x e2); tex_res > 0: the radiance Le is a
           tex_res^2 RGB texture over the quad, texel (floor(u0 R), floor(u1 R))
           of the quad coordinates u0 along e1, u1 along e2)
  camera   dict(pos, target, up, fov_deg, width, height)
  hf       dict(G, x0, z0, dx, base, mat) or None: heightfield top surface
           with vertex (i, j) at (x0 + i*dx, base + h[j*G+i], z0 + j*dx)
  albedo, Le, heights   initial parameters
  normal_map        optional [G*G*2] shading slopes (Sx, Sz) of a normal-mapped heightfield
  albedo_target, heights_target, normal_map_target   parameters that generate the loss target
"""
from __future__ import annotations

import math

import numpy as np

MAT_ABSORBER = 0
MAT_LAMBERT = 1
MAT_DIELECTRIC = 2
MAT_CONDUCTOR = 3

EMIT_QUAD = 0
EMIT_POINT = 1
EMIT_DIRECTIONAL = 2

SCENE_SEED = 2609
TARGET_SEED = 0x7A6


def _quad(o, e1, e2):
    """Two triangles of the parallelogram (o, o+e1, o+e1+e2, o+e2).

    The winding makes normalize(e1 x e2) the quad's front normal; chart
    coordinates run (0,0) at o to (1,1) at o+e1+e2.
    """
    o, e1, e2 = (np.asarray(a, np.float64) for a in (o, e1, e2))
    v = np.array([[o, o + e1, o + e1 + e2], [o, o + e1 + e2, o + e2]])
    uv = np.array([[[0, 0], [1, 0], [1, 1]], [[0, 0], [1, 1], [0, 1]]], np.float64)
    return v, uv


class _Builder:
    def __init__(self):
        self.v, self.uv, self.mat = [], [], []

    def quad(self, o, e1, e2, mat):
        v, uv = _quad(o, e1, e2)
        self.v.append(v)
        self.uv.append(uv)
        self.mat += [mat, mat]

    def arrays(self):
        return (np.concatenate(self.v).astype(np.float64),
                np.concatenate(self.uv).astype(np.float64),
                np.asarray(self.mat, np.int32))


def box_scene(width=64, height=64, tex_res=16, seed=SCENE_SEED,
              target_seed=TARGET_SEED, Le=10.0):
    """Diffuse unit box: 10 textured inward quads + one ceiling emitter.

    [0,1]^3 with the z=0 face open towards the camera.  Floor, ceiling and
    back wall are split at x=0.5, the side walls at z=0.5, giving 10 quads
    (20 triangles), each with its own tex_res^2 RGB albedo texture drawn
    U(0.2, 0.8).  A 0.25 x 0.25 one-sided emitter hangs 1e-3 below the
    ceiling, facing -y, and is a black absorber for paths that hit it.
    Pinhole camera at (0.5, 0.5, -1.4) looking +z, 40 degree vertical FOV.
    The loss target is rendered from albedo + N(0, 0.05), clipped to
    [0.01, 0.99].
    """
    b = _Builder()
    mats_type, mats_tex, mats_ior = [], [], []
    quads = [
        # floor (normal +y), split at x = 0.5
        ((0, 0, 0), (0, 0, 1), (0.5, 0, 0)),
        ((0.5, 0, 0), (0, 0, 1), (0.5, 0, 0)),
        # ceiling (normal -y)
        ((0, 1, 0), (0.5, 0, 0), (0, 0, 1)),
        ((0.5, 1, 0), (0.5, 0, 0), (0, 0, 1)),
        # back wall z = 1 (normal -z)
        ((0, 0, 1), (0, 1, 0), (0.5, 0, 0)),
        ((0.5, 0, 1), (0, 1, 0), (0.5, 0, 0)),
        # left wall x = 0 (normal +x), split at z = 0.5
        ((0, 0, 0), (0, 1, 0), (0, 0, 0.5)),
        ((0, 0, 0.5), (0, 1, 0), (0, 0, 0.5)),
        # right wall x = 1 (normal -x)
        ((1, 0, 0), (0, 0, 0.5), (0, 1, 0)),
        ((1, 0, 0.5), (0, 0, 0.5), (0, 1, 0)),
    ]
    for k, (o, e1, e2) in enumerate(quads):
        mats_type.append(MAT_LAMBERT)
        mats_tex.append(k)
        mats_ior.append(1.0)
        b.quad(o, e1, e2, k)
    em_o, em_e1, em_e2 = (0.375, 1 - 1e-3, 0.375), (0.25, 0, 0), (0, 0, 0.25)
    mats_type.append(MAT_ABSORBER)
    mats_tex.append(-1)
    mats_ior.append(1.0)
    b.quad(em_o, em_e1, em_e2, len(quads))
    tri_v, tri_uv, tri_mat = b.arrays()

    rng = np.random.default_rng(seed)
    albedo = rng.uniform(0.2, 0.8, size=(10, tex_res, tex_res, 3))
    trng = np.random.default_rng(target_seed)
    albedo_t = np.clip(albedo + trng.normal(0.0, 0.05, size=albedo.shape), 0.01, 0.99)
    return dict(
        name=f"box{width}x{height}",
        tri_v=tri_v, tri_uv=tri_uv, tri_mat=tri_mat,
        mat_type=np.asarray(mats_type, np.int32),
        mat_tex=np.asarray(mats_tex, np.int32),
        mat_ior=np.asarray(mats_ior, np.float64),
        n_tex=10, tex_res=tex_res,
        emitter=dict(type=EMIT_QUAD, o=np.array(em_o, float), e1=np.array(em_e1, float),
                     e2=np.array(em_e2, float)),
        camera=dict(pos=np.array([0.5, 0.5, -1.4]), target=np.array([0.5, 0.5, 0.5]),
                    up=np.array([0.0, 1.0, 0.0]), fov_deg=40.0, width=width, height=height),
        hf=None,
        albedo=albedo, Le=np.full(3, float(Le)), heights=None,
        albedo_target=albedo_t, heights_target=None,
    )


def box_detail_scene(width=128, height=128, tex_res=16, seed=SCENE_SEED, target_seed=TARGET_SEED, Le=10.0):
    """The diffuse box seen through a narrow window: the same camera position
    with a 12 degree vertical FOV aimed at (0.75, 0.3, 1.0), the lower right
    of the back wall.  Most light vertices connect outside the film, so the
    directions that reach the seen region carry the gradient: a scene where
    guiding diffuse vertices pays."""
    sc = box_scene(width, height, tex_res, seed, target_seed, Le)
    sc["camera"] = dict(sc["camera"], fov_deg=12.0, target=np.array([0.75, 0.3, 1.0]))
    return sc


def caustic_scene(G=128, width=512, height=512, seed=SCENE_SEED, target_seed=TARGET_SEED,
                  Le=1000.0, ior=1.5, h_sigma=0.002):
    """Glass heightfield slab over a diffuse receiver (attached workload).

    Receiver: y = 0, x,z in [-1, 1], grey albedo 0.8 (one 1x1 texture).
    Slab: dielectric (IOR 1.5) closed solid over x,z in [-0.5, 0.5]; flat
    bottom at y = 0.5 (outward normal -y), four vertical walls up to
    y = 0.6, and a G x G vertex heightfield top at y = 0.6 + h whose boundary
    ring stays at h = 0.  Heights start N(0, h_sigma) inside the ring.
    Emitter: 0.05 x 0.05 quad at y = 1 facing down.  Camera at
    (0, 0.45, -1.6) looking at (0, 0, 0.1), 50 degree FOV, kept below the slab
    so sensor connections never cross glass.  The target heights are a seeded
    product of sines that vanishes on the boundary ring.
    """
    b = _Builder()
    # materials: 0 receiver (Lambert, tex 0), 1 glass, 2 absorber (emitter)
    mat_type = np.array([MAT_LAMBERT, MAT_DIELECTRIC, MAT_ABSORBER], np.int32)
    mat_tex = np.array([0, -1, -1], np.int32)
    mat_ior = np.array([1.0, ior, 1.0])
    b.quad((-1, 0, -1), (0, 0, 2), (2, 0, 0), 0)            # receiver, normal +y
    b.quad((-0.5, 0.5, -0.5), (1, 0, 0), (0, 0, 1), 1)      # slab bottom, normal -y
    b.quad((-0.5, 0.5, -0.5), (0, 0.1, 0), (1, 0, 0), 1)    # wall z=-0.5, normal -z
    b.quad((-0.5, 0.5, 0.5), (1, 0, 0), (0, 0.1, 0), 1)     # wall z=+0.5, normal +z
    b.quad((-0.5, 0.5, -0.5), (0, 0, 1), (0, 0.1, 0), 1)    # wall x=-0.5, normal -x
    b.quad((0.5, 0.5, -0.5), (0, 0.1, 0), (0, 0, 1), 1)     # wall x=+0.5, normal +x
    em_o, em_e1, em_e2 = (-0.025, 1.0, -0.025), (0.05, 0, 0), (0, 0, 0.05)
    b.quad(em_o, em_e1, em_e2, 2)
    tri_v, tri_uv, tri_mat = b.arrays()

    rng = np.random.default_rng(seed)
    h = rng.normal(0.0, h_sigma, size=(G, G))
    h[0, :] = h[-1, :] = h[:, 0] = h[:, -1] = 0.0
    trng = np.random.default_rng(target_seed)
    amp = trng.uniform(0.005, 0.015)
    kx, kz = trng.integers(1, 4, size=2)
    xs = np.linspace(-0.5, 0.5, G)
    X, Z = np.meshgrid(xs, xs, indexing="xy")   # X[j, i] = x_i, Z[j, i] = z_j
    ht = amp * np.sin(math.pi * kx * (X + 0.5)) * np.sin(math.pi * kz * (Z + 0.5))
    ht[0, :] = ht[-1, :] = ht[:, 0] = ht[:, -1] = 0.0
    return dict(
        name=f"caustic{G}_{width}x{height}",
        tri_v=tri_v, tri_uv=tri_uv, tri_mat=tri_mat,
        mat_type=mat_type, mat_tex=mat_tex, mat_ior=mat_ior,
        n_tex=1, tex_res=1,
        emitter=dict(type=EMIT_QUAD, o=np.array(em_o, float), e1=np.array(em_e1, float),
                     e2=np.array(em_e2, float)),
        camera=dict(pos=np.array([0.0, 0.45, -1.6]), target=np.array([0.0, 0.0, 0.1]),
                    up=np.array([0.0, 1.0, 0.0]), fov_deg=50.0, width=width, height=height),
        hf=dict(G=G, x0=-0.5, z0=-0.5, dx=1.0 / (G - 1), base=0.6, mat=1),
        albedo=np.full((1, 1, 1, 3), 0.8), Le=np.full(3, float(Le)),
        heights=h.reshape(-1).copy(),
        albedo_target=None, heights_target=ht.reshape(-1).copy(),
    )


def mirror_scene(G=16, width=64, height=64, seed=SCENE_SEED, target_seed=TARGET_SEED, roughness=0.15,
                 Le=200.0, h_sigma=0.002):
    """Rough-conductor heightfield throwing a caustic onto a diffuse wall
    (the Mirror validation of the paper: attached gradients w.r.t. the
    vertex positions - here the heights - of a roughened conductor).

    Mirror: G x G heightfield over x,z in [-0.5, 0.5] at y = h (boundary
    ring at 0, inside N(0, h_sigma)), GGX roughness `roughness`, reflectance
    F0 (0.9, 0.85, 0.8) (texture 1).  Emitter: 0.1 x 0.1 quad centred at
    (-0.8, 0.8, 0) facing the mirror's centre (45 degrees).  Receiver: the
    wall x = 0.9 facing -x (y in [-0.2, 1.6], z in [-1, 1]), grey albedo 0.8
    (texture 0).  Camera at (-0.3, 0.7, -1.8) looking at (0.6, 0.55, 0), 50
    degree FOV: it sees the lit wall and the mirror.  Target heights: a
    seeded product of sines vanishing on the ring.
    """
    b = _Builder()
    # materials: 0 receiver (Lambert, tex 0), 1 mirror (conductor, tex 1), 2 absorber (emitter)
    mat_type = np.array([MAT_LAMBERT, MAT_CONDUCTOR, MAT_ABSORBER], np.int32)
    mat_tex = np.array([0, 1, -1], np.int32)
    mat_ior = np.array([1.0, float(roughness), 1.0])
    b.quad((0.9, -0.2, -1.0), (0, 0, 2), (0, 1.8, 0), 0)    # wall, normal -x
    s2 = 0.1 / math.sqrt(2.0)
    e1, e2 = np.array([s2, s2, 0.0]), np.array([0.0, 0.0, 0.1])   # e1 x e2 along (1, -1, 0)
    em_o = np.array([-0.8, 0.8, 0.0]) - 0.5 * e1 - 0.5 * e2
    b.quad(em_o, e1, e2, 2)
    tri_v, tri_uv, tri_mat = b.arrays()
    rng = np.random.default_rng(seed)
    h = rng.normal(0.0, h_sigma, size=(G, G))
    h[0, :] = h[-1, :] = h[:, 0] = h[:, -1] = 0.0
    trng = np.random.default_rng(target_seed)
    amp = trng.uniform(0.005, 0.015)
    kx, kz = trng.integers(1, 4, size=2)
    xs = np.linspace(-0.5, 0.5, G)
    X, Z = np.meshgrid(xs, xs, indexing="xy")
    ht = amp * np.sin(math.pi * kx * (X + 0.5)) * np.sin(math.pi * kz * (Z + 0.5))
    ht[0, :] = ht[-1, :] = ht[:, 0] = ht[:, -1] = 0.0
    albedo = np.zeros((2, 1, 1, 3))
    albedo[0, 0, 0] = 0.8
    albedo[1, 0, 0] = (0.9, 0.85, 0.8)
    return dict(
        name=f"mirror{G}_{width}x{height}",
        tri_v=tri_v, tri_uv=tri_uv, tri_mat=tri_mat,
        mat_type=mat_type, mat_tex=mat_tex, mat_ior=mat_ior,
        n_tex=2, tex_res=1,
        emitter=dict(type=EMIT_QUAD, o=em_o, e1=e1, e2=e2),
        camera=dict(pos=np.array([-0.3, 0.7, -1.8]), target=np.array([0.6, 0.55, 0.0]),
                    up=np.array([0.0, 1.0, 0.0]), fov_deg=50.0, width=width, height=height),
        hf=dict(G=G, x0=-0.5, z0=-0.5, dx=1.0 / (G - 1), base=0.0, mat=1),
        albedo=albedo, Le=np.full(3, float(Le)),
        heights=h.reshape(-1).copy(),
        albedo_target=None, heights_target=ht.reshape(-1).copy(),
    )


def glass_panel_scene(G=16, width=64, height=64, seed=SCENE_SEED, target_seed=TARGET_SEED, slope_sigma=0.05):
    """Normal-mapped glass panel over a diffuse receiver (attached workload
    with a normal map, the Glass Panel validation of the paper).

    The caustic scene's slab with a flat top (all heights zero) whose shading
    comes from a G x G normal map: per-vertex slopes (Sx, Sz), blended
    barycentrically, shading normal normalize(-Sx, 1, -Sz).  The map starts
    N(0, slope_sigma) per slope; the target map is a seeded smooth pattern
    (products of sines and cosines of amplitude ~0.1).
    """
    sc = caustic_scene(G=G, width=width, height=height, seed=seed, target_seed=target_seed)
    rng = np.random.default_rng(seed + 17)
    nm = rng.normal(0.0, slope_sigma, size=(G, G, 2))
    trng = np.random.default_rng(target_seed + 17)
    a, b = trng.uniform(0.05, 0.15, size=2)
    kx, kz = trng.integers(1, 4, size=2)
    xs = np.linspace(-0.5, 0.5, G)
    X, Z = np.meshgrid(xs, xs, indexing="xy")   # X[j, i] = x_i, Z[j, i] = z_j
    nt = np.stack([a * np.cos(math.pi * kx * (X + 0.5)) * np.sin(math.pi * kz * (Z + 0.5)),
                   b * np.sin(math.pi * kx * (X + 0.5)) * np.cos(math.pi * kz * (Z + 0.5))], axis=-1)
    sc.update(name=f"panel{G}_{width}x{height}", heights=np.zeros(G * G), heights_target=None,
              normal_map=nm.reshape(-1).copy(), normal_map_target=nt.reshape(-1).copy())
    return sc


def glass_slab_scene(G=16, width=64, height=64, tex_res=8, seed=SCENE_SEED, target_seed=TARGET_SEED,
                     Le=40.0, ior=1.5):
    """Glass slab over a textured diffuse receiver, seen from above (the
    Glass Slab scene of the paper, framed so that the camera looks through
    the glass: the workload of the bidirectional combination).

    Receiver: y = 0, x,z in [-1.2, 1.2], albedo texture tex_res^2 drawn
    U(0.3, 0.9) per channel (texture 0).  Slab: dielectric (IOR `ior`)
    closed solid over x,z in [-0.5, 0.5]; flat bottom at y = 0.3, walls up
    to y = 0.4, G x G vertex heightfield top at y = 0.4 (heights zero).
    Emitter: 0.4 x 0.4 quad centred at (0, 1, 0.2) facing down (an absorber
    quad in the geometry).  Camera at (0, 1.2, -1.4) looking at
    (0, 0.1, 0.15), 45 degree FOV: part of the receiver is seen directly,
    part through the slab.  Target albedo: another seeded texture.
    """
    b = _Builder()
    mat_type = np.array([MAT_LAMBERT, MAT_DIELECTRIC, MAT_ABSORBER], np.int32)
    mat_tex = np.array([0, -1, -1], np.int32)
    mat_ior = np.array([1.0, ior, 1.0])
    b.quad((-1.2, 0, -1.2), (0, 0, 2.4), (2.4, 0, 0), 0)     # receiver, normal +y
    b.quad((-0.5, 0.3, -0.5), (1, 0, 0), (0, 0, 1), 1)       # slab bottom, normal -y
    b.quad((-0.5, 0.3, -0.5), (0, 0.1, 0), (1, 0, 0), 1)     # wall z=-0.5, normal -z
    b.quad((-0.5, 0.3, 0.5), (1, 0, 0), (0, 0.1, 0), 1)      # wall z=+0.5, normal +z
    b.quad((-0.5, 0.3, -0.5), (0, 0, 1), (0, 0.1, 0), 1)     # wall x=-0.5, normal -x
    b.quad((0.5, 0.3, -0.5), (0, 0.1, 0), (0, 0, 1), 1)      # wall x=+0.5, normal +x
    em_o, em_e1, em_e2 = (-0.2, 1.0, 0.0), (0.4, 0, 0), (0, 0, 0.4)   # e1 x e2 along -y
    b.quad(em_o, em_e1, em_e2, 2)
    tri_v, tri_uv, tri_mat = b.arrays()
    rng = np.random.default_rng(seed)
    albedo = rng.uniform(0.3, 0.9, size=(1, tex_res, tex_res, 3))
    trng = np.random.default_rng(target_seed)
    albedo_t = trng.uniform(0.3, 0.9, size=(1, tex_res, tex_res, 3))
    return dict(
        name=f"slab{G}_{width}x{height}",
        tri_v=tri_v, tri_uv=tri_uv, tri_mat=tri_mat,
        mat_type=mat_type, mat_tex=mat_tex, mat_ior=mat_ior,
        n_tex=1, tex_res=tex_res,
        emitter=dict(type=EMIT_QUAD, o=np.array(em_o, float), e1=np.array(em_e1, float),
                     e2=np.array(em_e2, float)),
        camera=dict(pos=np.array([0.0, 1.2, -1.4]), target=np.array([0.0, 0.1, 0.15]),
                    up=np.array([0.0, 1.0, 0.0]), fov_deg=45.0, width=width, height=height),
        hf=dict(G=G, x0=-0.5, z0=-0.5, dx=1.0 / (G - 1), base=0.4, mat=1),
        albedo=albedo, Le=np.full(3, float(Le)),
        heights=np.zeros(G * G),
        albedo_target=albedo_t, heights_target=None,
    )


def slab_view_scene(width=8, height=8, ior=1.5, Le=2.0, fov_deg=20.0):
    """A camera looking straight down through a wide flat glass slab at a
    large emitter (closed-form pin of camera paths through specular chains).

    Emitter: quad over x,z in [-5, 5] at y = 0 facing +y, radiance Le (not
    geometry).  Slab: dielectric closed box over x,z in [-4, 4], faces at
    y = 0.4 and y = 0.6.  Camera at (0, 1.5, 0) looking down (up = +z).  A
    camera ray at angle theta to the vertical crosses the slab after 2k
    internal reflections with weight (1 - F)^2 F^(2k), F the unpolarized
    Fresnel reflectance at theta (the same at both faces).
    """
    b = _Builder()
    mat_type = np.array([MAT_DIELECTRIC], np.int32)
    mat_tex = np.array([-1], np.int32)
    mat_ior = np.array([ior])
    lo, hi, s = 0.4, 0.6, 4.0
    b.quad((-s, hi, -s), (0, 0, 2 * s), (2 * s, 0, 0), 0)     # top, normal +y
    b.quad((-s, lo, -s), (2 * s, 0, 0), (0, 0, 2 * s), 0)     # bottom, normal -y
    b.quad((-s, lo, -s), (0, hi - lo, 0), (2 * s, 0, 0), 0)   # wall z=-s, normal -z
    b.quad((-s, lo, s), (2 * s, 0, 0), (0, hi - lo, 0), 0)    # wall z=+s, normal +z
    b.quad((-s, lo, -s), (0, 0, 2 * s), (0, hi - lo, 0), 0)   # wall x=-s, normal -x
    b.quad((s, lo, -s), (0, hi - lo, 0), (0, 0, 2 * s), 0)    # wall x=+s, normal +x
    tri_v, tri_uv, tri_mat = b.arrays()
    return dict(
        name=f"slabview_{width}x{height}",
        tri_v=tri_v, tri_uv=tri_uv, tri_mat=tri_mat,
        mat_type=mat_type, mat_tex=mat_tex, mat_ior=mat_ior,
        n_tex=1, tex_res=1,
        emitter=dict(type=EMIT_QUAD, o=np.array([-5.0, 0.0, 5.0]), e1=np.array([10.0, 0.0, 0.0]),
                     e2=np.array([0.0, 0.0, -10.0])),
        camera=dict(pos=np.array([0.0, 1.5, 0.0]), target=np.array([0.0, 0.0, 0.0]),
                    up=np.array([0.0, 0.0, 1.0]), fov_deg=fov_deg, width=width, height=height),
        albedo=np.full((1, 1, 1, 3), 0.5), Le=np.full(3, float(Le)),
        albedo_target=None, heights_target=None,
    )


def directional_plane_scene(width=16, height=16, rho=0.6, tex_res=4, seed=SCENE_SEED, cam_h=2.0, fov_deg=60.0):
    """A textured directional emitter over a Lambertian plane, seen by a
    pinhole camera looking straight down (closed-form pin only).

    Plane y = 0, x,z in [-4, 4], albedo rho.  The emitter: a 0.9 x 0.7 quad
    at y = 1 from (-0.5, 1, -0.3), e1 along +x, e2 along +z, emitting a
    collimated beam straight down with a tex_res^2 RGB irradiance texture
    U(0.5, 1.5).  The emitter is not geometry (nothing occludes the camera).
    Camera at (0, cam_h, 0), up +z.  The beam lights the quad's footprint at
    normal incidence, so the expected image is a sum over texels of
    rho E_t / pi times the tent-filtered film area of the texel's footprint.
    """
    b = _Builder()
    b.quad((-4, 0, -4), (0, 0, 8), (8, 0, 0), 0)   # normal +y
    tri_v, tri_uv, tri_mat = b.arrays()
    rng = np.random.default_rng(seed + 29)
    Le = rng.uniform(0.5, 1.5, size=(tex_res, tex_res, 3))
    return dict(
        name="directional_plane",
        tri_v=tri_v, tri_uv=tri_uv, tri_mat=tri_mat,
        mat_type=np.array([MAT_LAMBERT], np.int32), mat_tex=np.array([0], np.int32),
        mat_ior=np.array([1.0]),
        n_tex=1, tex_res=1,
        emitter=dict(type=EMIT_DIRECTIONAL, o=np.array([-0.5, 1.0, -0.3]), e1=np.array([0.9, 0.0, 0.0]),
                     e2=np.array([0.0, 0.0, 0.7]), tex_res=tex_res),
        camera=dict(pos=np.array([0.0, cam_h, 0.0]), target=np.array([0.0, 0.0, 0.0]),
                    up=np.array([0.0, 0.0, 1.0]), fov_deg=fov_deg, width=width, height=height),
        hf=None,
        albedo=np.full((1, 1, 1, 3), rho), Le=Le.reshape(-1).copy(), heights=None,
        albedo_target=None, heights_target=None,
    )


def tumbler_scene(G=16, width=64, height=64, tex_res=8, seed=SCENE_SEED, target_seed=TARGET_SEED, ior=1.5):
    """Glass under a textured directional emitter (the Tumbler validation of
    the paper: differentiate the radiance texture of a directional emitter).

    The caustic scene's receiver and glass heightfield slab (heights
    N(0, 0.002) inside a zero ring), lit by a collimated beam from a 0.6 x 0.6
    quad at y = 1 pointing down, whose irradiance is a tex_res^2 RGB texture
    U(10, 30); the target texture is the same plus a seeded smooth pattern.
    Detached: the parameters are the emitter texture and the receiver albedo.
    """
    sc = caustic_scene(G=G, width=width, height=height, seed=seed, target_seed=target_seed, ior=ior)
    # drop the small area emitter's absorber quad: the beam source is not geometry
    sc["tri_v"], sc["tri_uv"], sc["tri_mat"] = sc["tri_v"][:-2], sc["tri_uv"][:-2], sc["tri_mat"][:-2]
    rng = np.random.default_rng(seed + 31)
    Le = rng.uniform(10.0, 30.0, size=(tex_res, tex_res, 3))
    xs = np.linspace(0.0, 1.0, tex_res)
    X, Z = np.meshgrid(xs, xs, indexing="xy")
    bump = 5.0 * np.sin(2 * math.pi * X)[..., None] * np.cos(math.pi * Z)[..., None] * np.array([1.0, 0.8, 0.6])
    sc.update(name=f"tumbler{G}_{width}x{height}",
              emitter=dict(type=EMIT_DIRECTIONAL, o=np.array([-0.3, 1.0, -0.3]), e1=np.array([0.6, 0.0, 0.0]),
                           e2=np.array([0.0, 0.0, 0.6]), tex_res=tex_res),
              Le=Le.reshape(-1).copy(), Le_target=(Le + bump).reshape(-1).copy())
    return sc


def plane_point_light_scene(width=32, height=32, rho=0.6, I0=5.0, light_h=0.8,
                            cam_h=2.0, fov_deg=60.0, roughness=None):
    """Point light over a large Lambertian plane seen by a pinhole camera.

    Plane y = 0 spanning x,z in [-4, 4] with one constant albedo rho (a 1x1
    texture); isotropic point light of intensity I0 at (0.3, light_h, -0.2);
    camera at (0, cam_h, 0) looking straight down with up = +z.  With one
    scattering vertex the expected image has a closed form (a pixel-filtered
    integral of rho/pi * I0 cos(theta_l) / r^2).  With a roughness the
    plane is a rough conductor of reflectance rho instead.
    """
    b = _Builder()
    b.quad((-4, 0, -4), (0, 0, 8), (8, 0, 0), 0)   # normal +y
    tri_v, tri_uv, tri_mat = b.arrays()
    cond = roughness is not None
    return dict(
        name="plane_point",
        tri_v=tri_v, tri_uv=tri_uv, tri_mat=tri_mat,
        mat_type=np.array([MAT_CONDUCTOR if cond else MAT_LAMBERT], np.int32), mat_tex=np.array([0], np.int32),
        mat_ior=np.array([float(roughness) if cond else 1.0]),
        n_tex=1, tex_res=1,
        emitter=dict(type=EMIT_POINT, o=np.array([0.3, light_h, -0.2]),
                     e1=np.zeros(3), e2=np.zeros(3)),
        camera=dict(pos=np.array([0.0, cam_h, 0.0]), target=np.array([0.0, 0.0, 0.0]),
                    up=np.array([0.0, 0.0, 1.0]), fov_deg=fov_deg, width=width, height=height),
        hf=None,
        albedo=np.full((1, 1, 1, 3), rho), Le=np.full(3, float(I0)), heights=None,
        albedo_target=None, heights_target=None,
    )


def two_plane_point_light_scene(width=8, height=8, rho_floor=0.7, rho_wall=0.5, I0=5.0,
                                light=(-0.3, 0.8, 0.1), fov_deg=30.0):
    """Point light, a Lambertian floor and a Lambertian wall, seen by a
    pinhole camera that sees only the wall.

    Floor: y = 0, x,z in [-1, 1], albedo rho_floor (texture 0), normal +y.
    Wall: x = 1, y in [0, 2], z in [-1, 1], albedo rho_wall (texture 1),
    normal -x.  Isotropic point light of intensity I0 at `light`.  Camera at
    (-0.5, 1, 0) looking along +x (up +y) with a narrow field of view: its
    view cone meets only the wall, and no floor point projects onto the film.
    The light paths light -> floor -> wall put their second vertex on the
    visible wall, so the depth-2 part of the image has a closed form (a
    pixel-filtered integral over the floor of the once-scattered radiance).
    """
    b = _Builder()
    b.quad((-1, 0, -1), (0, 0, 2), (2, 0, 0), 0)   # floor, normal +y
    b.quad((1, 0, -1), (0, 0, 2), (0, 2, 0), 1)    # wall, normal -x
    tri_v, tri_uv, tri_mat = b.arrays()
    albedo = np.zeros((2, 1, 1, 3))
    albedo[0] = rho_floor
    albedo[1] = rho_wall
    return dict(
        name="two_plane_point",
        tri_v=tri_v, tri_uv=tri_uv, tri_mat=tri_mat,
        mat_type=np.array([MAT_LAMBERT, MAT_LAMBERT], np.int32), mat_tex=np.array([0, 1], np.int32),
        mat_ior=np.array([1.0, 1.0]),
        n_tex=2, tex_res=1,
        emitter=dict(type=EMIT_POINT, o=np.array(light, float), e1=np.zeros(3), e2=np.zeros(3)),
        camera=dict(pos=np.array([-0.5, 1.0, 0.0]), target=np.array([1.0, 1.0, 0.0]),
                    up=np.array([0.0, 1.0, 0.0]), fov_deg=fov_deg, width=width, height=height),
        hf=None,
        albedo=albedo, Le=np.full(3, float(I0)), heights=None,
        albedo_target=None, heights_target=None,
    )


def batched_instances(n=48, seed=7):
    """Size table of a batch of uneven inverse-rendering instances.

    Half box, half caustic; heightfield side G log-uniform in [32, 256];
    film side log-uniform in [128, 1024] rounded to a multiple of 16; path
    count log-uniform in [1M, 32M]; depth uniform in [4, 12].
    """
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        kind = "box" if rng.uniform() < 0.5 else "caustic"
        G = int(round(math.exp(rng.uniform(math.log(32), math.log(256)))))
        film = int(round(math.exp(rng.uniform(math.log(128), math.log(1024))) / 16.0)) * 16
        paths = int(round(math.exp(rng.uniform(math.log(1 << 20), math.log(32 << 20)))))
        depth = int(rng.integers(4, 13))
        out.append(dict(kind=kind, G=G, film=film, n_paths=paths, depth=depth))
    return out


def guided_batch_instances(n=12, seed=11):
    """Size table of a batch of smooth-slab caustic instances for the guided
    batch: heightfield side G log-uniform in [32, 96], film side log-uniform
    in [128, 384] rounded to a multiple of 16, path count log-uniform in
    [1M, 4M], depth 6; each instance has its own scene and target seeds."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        G = int(round(math.exp(rng.uniform(math.log(32), math.log(96)))))
        film = int(round(math.exp(rng.uniform(math.log(128), math.log(384))) / 16.0)) * 16
        paths = int(round(math.exp(rng.uniform(math.log(1 << 20), math.log(4 << 20)))))
        out.append(dict(G=G, film=film, n_paths=paths, depth=6, scene_seed=SCENE_SEED + 101 * (k + 1),
                        target_seed=TARGET_SEED + 7 * (k + 1)))
    return out


GUIDE_SEED = 0x6D6C70
GUIDE_NPARAMS = 11433   # W1[64][6] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[41][64] b4[41]


def guide_weights(seed=GUIDE_SEED, out_scale=0.05):
    """Initial emission-guide weights, flat float64 [11433].

    Hidden layers: He-normal N(0, 2/fan_in), zero biases; output layer
    N(0, (out_scale^2)/fan_in) so that the first mixture is broad.
    """
    rng = np.random.default_rng(seed)
    parts = []
    for n_out, n_in, s in ((64, 6, math.sqrt(2.0 / 6)), (64, 64, math.sqrt(2.0 / 64)),
                           (64, 64, math.sqrt(2.0 / 64)), (41, 64, out_scale / math.sqrt(64))):
        parts.append(rng.normal(0.0, s, size=n_out * n_in))
        parts.append(np.zeros(n_out))
    w = np.concatenate(parts)
    assert w.size == GUIDE_NPARAMS
    return w


def guide_random_weights(seed, scale=1.0):
    """Weights with every entry (biases included) drawn N(0, scale^2/fan_in):
    a network whose mixtures are far from uniform, for parity tests."""
    rng = np.random.default_rng(seed)
    parts = []
    for n_out, n_in in ((64, 6), (64, 64), (64, 64), (41, 64)):
        s = scale * math.sqrt(2.0 / n_in)
        parts.append(rng.normal(0.0, s, size=n_out * n_in))
        parts.append(rng.normal(0.0, 0.3 * scale, size=n_out))
    return np.concatenate(parts)


def guide_sample_batch(sc, count, seed, zero_frac=0.25):
    """Synthetic training samples [count, 12]: x uniform in the emitter quad,
    its unit normal, a direction uniform on that hemisphere, a positive
    sampling density, a contribution S >= 0 (a fraction exactly zero)."""
    rng = np.random.default_rng(seed)
    em = sc["emitter"]
    o, e1, e2 = (np.asarray(em[k], np.float64) for k in ("o", "e1", "e2"))
    nrm = np.cross(e1, e2)
    nrm /= np.linalg.norm(nrm)
    u = rng.uniform(size=(count, 2))
    x = o + u[:, :1] * e1 + u[:, 1:2] * e2
    d = rng.normal(size=(count, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    d = np.where((d @ nrm)[:, None] < 0.0, -d, d)
    q = rng.uniform(0.05, 3.0, size=count)
    S = rng.exponential(1.0, size=count) * (rng.uniform(size=count) >= zero_frac)
    out = np.zeros((count, 12))
    out[:, 0:3], out[:, 3:6], out[:, 6:9], out[:, 9], out[:, 10] = x, nrm, d, q, S
    return out


def guide_aimed_weights(direction=(0.0, -1.0, 0.0), logk=2.0, spread=0.3, seed=GUIDE_SEED):
    """A guide whose 8 lobes point near `direction` (mean direction plus
    N(0, spread^2) per component), log-concentration `logk`, equal logits and
    mixing logit 1: the shape a guide trained on a scene below the emitter
    takes.  Hidden layers as guide_weights; only the output biases are set."""
    w = guide_weights(seed)
    rng = np.random.default_rng(seed + 1)
    b4 = w[GUIDE_NPARAMS - 41:]
    d = np.asarray(direction, np.float64)
    for k in range(8):
        b4[5 * k:5 * k + 3] = d + spread * rng.normal(size=3)
        b4[5 * k + 3] = logk
        b4[5 * k + 4] = 0.0
    b4[40] = 1.0
    return w
