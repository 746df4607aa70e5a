"""ctypes front end of the FP64 CPU oracle (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  The product path never does.

Functions mirror the oracle's C entry points:
  render(scene, ...)    light-tracing image (Sec. 3.1, Eq. 1-2, Eq. 20)
  gradient(scene, ...)  d<dI, I(theta)>/dtheta by taped reverse-mode AD
                        (naive) or of the ResLRB estimator (Eq. 11)
  loss_and_adjoint(I, T)  mean-squared error and dLoss/dI
  reservoir(w, u)       capacity-one weighted reservoir (Eq. 8)
  dielectric(...)       one smooth-dielectric scattering event (Fresnel
                        lobe choice, Snell refraction, mirror reflection)
  philox(seed, ctr)     Philox-4x32-10 block (Salmon et al. 2011)
  guide_*               the learned emission guide (an extension: MLP to a
                        folded vMF mixture, its sampler and density, the
                        training loss gradient) and plain Adam
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lt_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

ATTACHED = 1
SPLAT_SELECTED = 2
MODE_NAIVE = 0
MODE_RESLRB = 1


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (FP64, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class _Scene(C.Structure):
    _fields_ = [
        ("n_tris", C.c_int32), ("tri_v", C.POINTER(C.c_double)), ("tri_uv", C.POINTER(C.c_double)),
        ("tri_mat", C.POINTER(C.c_int32)),
        ("n_mats", C.c_int32), ("mat_type", C.POINTER(C.c_int32)), ("mat_tex", C.POINTER(C.c_int32)),
        ("mat_ior", C.POINTER(C.c_double)),
        ("n_tex", C.c_int32), ("tex_res", C.c_int32),
        ("em_type", C.c_int32), ("em_o", C.c_double * 3), ("em_e1", C.c_double * 3),
        ("em_e2", C.c_double * 3),
        ("cam_pos", C.c_double * 3), ("cam_target", C.c_double * 3), ("cam_up", C.c_double * 3),
        ("cam_fov_deg", C.c_double), ("width", C.c_int32), ("height", C.c_int32),
        ("hf_G", C.c_int32), ("hf_x0", C.c_double), ("hf_z0", C.c_double), ("hf_dx", C.c_double),
        ("hf_base", C.c_double), ("hf_mat", C.c_int32),
        ("em_tex_res", C.c_int32),
    ]


class _Args(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("n_paths", C.c_int64), ("max_depth", C.c_int32),
                ("flags", C.c_int32), ("n_threads", C.c_int32),
                ("path_list", C.POINTER(C.c_uint32)), ("n_list", C.c_int64),
                ("guide_w", C.POINTER(C.c_double)), ("guide_bf16", C.c_int32),
                ("guide_diffuse", C.c_int32), ("guide_flag", C.POINTER(C.c_uint8))]


GUIDE_NPARAMS = 11433
GUIDE_OUT = 41


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = C.CDLL(_LIB)
        dp, ip, up = C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_uint32)
        _lib.ora_render.argtypes = [C.POINTER(_Scene), C.POINTER(_Args), dp, dp, dp, dp, dp, dp, up, ip, dp, dp, up]
        _lib.ora_gradient.argtypes = [C.POINTER(_Scene), C.POINTER(_Args), C.c_int, dp, dp, dp, dp, dp, dp, dp, dp, dp]
        _lib.ora_reservoir.argtypes = [dp, dp, C.c_int, dp]
        _lib.ora_reservoir.restype = C.c_int
        _lib.ora_philox.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, up]
        _lib.ora_render.restype = C.c_int
        _lib.ora_gradient.restype = C.c_int
        _lib.ora_guide_eval.argtypes = [C.POINTER(_Scene), dp, dp, dp, C.c_int64, C.c_int, dp]
        _lib.ora_guide_pdf.argtypes = [dp, dp, dp, C.c_int64, dp]
        _lib.ora_guide_sample.argtypes = [dp, dp, dp, C.c_int64, dp, ip]
        _lib.ora_guide_emit.argtypes = [C.POINTER(_Scene), C.POINTER(_Args), dp, ip]
        _lib.ora_guide_emit.restype = C.c_int
        _lib.ora_guide_loss_grad.argtypes = [C.POINTER(_Scene), dp, dp, C.c_int64, C.c_int, dp, dp]
        _lib.ora_guide_table.argtypes = [C.POINTER(_Scene), C.POINTER(_Args), dp, dp, dp, C.POINTER(C.c_uint8)]
        _lib.ora_guide_table.restype = C.c_int64
        _lib.ora_guide_vertex_samples.argtypes = [C.POINTER(_Scene), C.POINTER(_Args), dp, dp, dp, dp, dp]
        _lib.ora_guide_vertex_samples.restype = C.c_int
        _lib.ora_ggx_terms.argtypes = [C.c_double, C.c_double, C.c_double, dp, dp]
        _lib.ora_conductor.argtypes = [dp, dp, C.c_double, C.c_double, C.c_double, dp, dp]
        _lib.ora_conductor.restype = C.c_int
        _lib.ora_conductor_conn.argtypes = [dp, dp, dp, C.c_double]
        _lib.ora_conductor_conn.restype = C.c_double
        _lib.ora_render_camera.argtypes = [C.POINTER(_Scene), C.POINTER(_Args), C.c_int, dp, dp, dp, dp, dp, up]
        _lib.ora_render_camera.restype = C.c_int
        _lib.ora_gradient_camera.argtypes = [C.POINTER(_Scene), C.POINTER(_Args), C.c_int, dp, dp, dp, dp, dp, dp, dp]
        _lib.ora_gradient_camera.restype = C.c_int
        _lib.ora_dielectric.argtypes = [dp, dp, dp, C.c_double, C.c_double, dp, ip, dp]
        _lib.ora_dielectric.restype = C.c_int
        assert _lib.ora_guide_nparams() == GUIDE_NPARAMS
    return _lib


def _p(a, t=C.c_double):
    return None if a is None else a.ctypes.data_as(C.POINTER(t))


class _Keep:
    """Holds the numpy arrays a ctypes struct points into."""

    def __init__(self):
        self.refs = []

    def f64(self, a):
        a = np.ascontiguousarray(a, np.float64)
        self.refs.append(a)
        return a

    def i32(self, a):
        a = np.ascontiguousarray(a, np.int32)
        self.refs.append(a)
        return a


def _scene(sc, keep):
    s = _Scene()
    tv, tuv, tm = keep.f64(sc["tri_v"]), keep.f64(sc["tri_uv"]), keep.i32(sc["tri_mat"])
    s.n_tris = tv.shape[0]
    s.tri_v, s.tri_uv, s.tri_mat = _p(tv), _p(tuv), _p(tm, C.c_int32)
    mt, mx, mi = keep.i32(sc["mat_type"]), keep.i32(sc["mat_tex"]), keep.f64(sc["mat_ior"])
    s.n_mats = mt.shape[0]
    s.mat_type, s.mat_tex, s.mat_ior = _p(mt, C.c_int32), _p(mx, C.c_int32), _p(mi)
    s.n_tex, s.tex_res = int(sc["n_tex"]), int(sc["tex_res"])
    em = sc["emitter"]
    s.em_type = int(em["type"])
    s.em_tex_res = int(em.get("tex_res", 0))
    for k in range(3):
        s.em_o[k], s.em_e1[k], s.em_e2[k] = em["o"][k], em["e1"][k], em["e2"][k]
    cam = sc["camera"]
    for k in range(3):
        s.cam_pos[k], s.cam_target[k], s.cam_up[k] = cam["pos"][k], cam["target"][k], cam["up"][k]
    s.cam_fov_deg = float(cam["fov_deg"])
    s.width, s.height = int(cam["width"]), int(cam["height"])
    hf = sc.get("hf")
    if hf is not None:
        s.hf_G, s.hf_x0, s.hf_z0 = int(hf["G"]), float(hf["x0"]), float(hf["z0"])
        s.hf_dx, s.hf_base, s.hf_mat = float(hf["dx"]), float(hf["base"]), int(hf["mat"])
    else:
        s.hf_G = 0
    return s


def _args(seed, n_paths, depth, flags, threads, path_list, keep, guide_w=None, guide_bf16=True,
          guide_diffuse=False):
    a = _Args()
    if guide_w is not None:
        gw = keep.f64(guide_w)
        assert gw.size == GUIDE_NPARAMS
        a.guide_w, a.guide_bf16 = _p(gw), int(bool(guide_bf16))
    else:
        a.guide_w, a.guide_bf16 = None, 0
    a.guide_diffuse = int(bool(guide_diffuse) and guide_w is not None)
    a.guide_flag = None
    a.seed, a.n_paths, a.max_depth, a.flags, a.n_threads = int(seed), int(n_paths), int(depth), int(flags), int(threads)
    if path_list is not None:
        pl = np.ascontiguousarray(path_list, np.uint32)
        keep.refs.append(pl)
        a.path_list, a.n_list = _p(pl, C.c_uint32), pl.shape[0]
    else:
        a.path_list, a.n_list = None, 0
    return a


def _params(sc, albedo, Le, heights, keep, normal_map=None):
    albedo = keep.f64(sc["albedo"] if albedo is None else albedo)
    Le = keep.f64(sc["Le"] if Le is None else Le)
    if heights is None:
        heights = sc.get("heights")
    heights = None if heights is None else keep.f64(heights)
    if normal_map is None:
        normal_map = sc.get("normal_map")
    normal_map = None if normal_map is None else keep.f64(normal_map)
    return albedo, Le, heights, normal_map


def render(sc, seed, n_paths, depth, albedo=None, Le=None, heights=None, flags=0,
           path_list=None, slices=False, per_path=False, threads=0, guide_w=None, guide_bf16=True,
           normal_map=None, guide_diffuse=False, guide_flag=None):
    """FP64 light-tracing image [H,W,3] (plus optional per-depth slices,
    per-path signature / reservoir index R / weight W / ill-conditioning
    flag, and total flux).
    guide_w: emission-guide weights (guided emission), else cosine emission;
    guide_diffuse: Lambertian vertices scatter from the guide table too;
    guide_flag: optional bool per guide-table entry (test bookkeeping):
    per_path's "gflag" marks the paths that scatter from a marked entry.
    normal_map: [G*G*2] shading slopes of a normal-mapped heightfield
    (default: the scene's, if any; else slopes from the heights)."""
    lib = _load()
    keep = _Keep()
    s = _scene(sc, keep)
    a = _args(seed, n_paths, depth, flags, threads, path_list, keep, guide_w, guide_bf16, guide_diffuse)
    alb, le, h, nm = _params(sc, albedo, Le, heights, keep, normal_map)
    if guide_flag is not None:
        gf = np.ascontiguousarray(guide_flag, np.uint8)
        keep.refs.append(gf)
        a.guide_flag = _p(gf, C.c_uint8)
    H, W = int(sc["camera"]["height"]), int(sc["camera"]["width"])
    img = np.zeros((H, W, 3))
    sl = np.zeros((depth, H, W, 3)) if slices else None
    n = len(path_list) if path_list is not None else int(n_paths)
    sig = np.zeros(n, np.uint32) if per_path else None
    R = np.zeros(n, np.int32) if per_path else None
    Wr = np.zeros(n) if per_path else None
    info = np.zeros(n, np.uint32) if per_path else None
    flux = np.zeros(3)
    rc = lib.ora_render(C.byref(s), C.byref(a), _p(alb), _p(le), _p(h), _p(nm), _p(img), _p(sl),
                        _p(sig, C.c_uint32), _p(R, C.c_int32), _p(Wr), _p(flux), _p(info, C.c_uint32))
    if rc != 0:
        raise ValueError("oracle render rejected its arguments")
    out = dict(image=img, flux=flux)
    if slices:
        out["slices"] = sl
    if per_path:
        out.update(sig=sig, R=R, W=Wr, illc=(info & 2) != 0, gflag=(info & 4) != 0)
    return out


def gradient(sc, seed, n_paths, depth, dI, mode=MODE_NAIVE, albedo=None, Le=None, heights=None,
             flags=0, path_list=None, threads=0, guide_w=None, guide_bf16=True, normal_map=None,
             guide_diffuse=False):
    """Gradient of <dI, I(theta)> w.r.t. albedo texels, emitter radiance and
    (attached) heights and normal-map slopes, by taped reverse-mode AD of
    each light path.  With guide_w the emission (and with guide_diffuse the
    Lambertian scatter) is guided and its density is held fixed (detached)."""
    lib = _load()
    keep = _Keep()
    s = _scene(sc, keep)
    a = _args(seed, n_paths, depth, flags, threads, path_list, keep, guide_w, guide_bf16, guide_diffuse)
    alb, le, h, nm = _params(sc, albedo, Le, heights, keep, normal_map)
    dI = keep.f64(dI)
    g_alb = np.zeros_like(alb)
    g_le = np.zeros_like(le)
    g_h = np.zeros_like(h) if h is not None else None
    g_n = np.zeros_like(nm) if nm is not None else None
    rc = lib.ora_gradient(C.byref(s), C.byref(a), int(mode), _p(alb), _p(le), _p(h), _p(nm), _p(dI),
                          _p(g_alb), _p(g_le), _p(g_h), _p(g_n))
    if rc != 0:
        raise ValueError("oracle gradient rejected its arguments")
    return dict(albedo=g_alb, Le=g_le, heights=g_h, normal_map=g_n)


def render_camera(sc, seed, n_paths, depth, spec_only=True, albedo=None, Le=None, heights=None, path_list=None,
                  threads=0, per_path=False):
    """Camera-side image [H,W,3] of the bidirectional combination: n_paths
    camera samples (a multiple of W*H), each pixel averaging n_paths/(W*H);
    spec_only: only samples whose first vertex is specular (the paths the
    light tracer cannot connect), else every path (a full path tracer with
    next-event estimation, the reference of the tests)."""
    lib = _load()
    keep = _Keep()
    s = _scene(sc, keep)
    a = _args(seed, n_paths, depth, 0, threads, path_list, keep)
    alb, le, h, nm = _params(sc, albedo, Le, heights, keep)
    H, W = int(sc["camera"]["height"]), int(sc["camera"]["width"])
    img = np.zeros((H, W, 3))
    n = len(path_list) if path_list is not None else int(n_paths)
    sig = np.zeros(n, np.uint32) if per_path else None
    if lib.ora_render_camera(C.byref(s), C.byref(a), int(bool(spec_only)), _p(alb), _p(le), _p(h), _p(nm), _p(img),
                             _p(sig, C.c_uint32)) != 0:
        raise ValueError("camera samples need a quad or point emitter and n_paths a multiple of the pixel count")
    out = dict(image=img)
    if per_path:
        out["sig"] = sig
    return out


def gradient_camera(sc, seed, n_paths, depth, dI, spec_only=True, albedo=None, Le=None, heights=None,
                    path_list=None, threads=0):
    """Gradient of <dI, I_camera> w.r.t. albedo texels and emitter radiance
    (detached) by taped reverse-mode AD of each camera sample."""
    lib = _load()
    keep = _Keep()
    s = _scene(sc, keep)
    a = _args(seed, n_paths, depth, 0, threads, path_list, keep)
    alb, le, h, nm = _params(sc, albedo, Le, heights, keep)
    dI = keep.f64(dI)
    g_alb, g_le = np.zeros_like(alb), np.zeros_like(le)
    if lib.ora_gradient_camera(C.byref(s), C.byref(a), int(bool(spec_only)), _p(alb), _p(le), _p(h), _p(nm), _p(dI),
                               _p(g_alb), _p(g_le)) != 0:
        raise ValueError("camera samples need a quad or point emitter and n_paths a multiple of the pixel count")
    return dict(albedo=g_alb, Le=g_le)


def loss_and_adjoint(image, target):
    """Mean squared error over all 3*W*H entries and its image adjoint."""
    image = np.asarray(image, np.float64)
    target = np.asarray(target, np.float64)
    n = image.size
    diff = image - target
    return float(np.sum(diff * diff) / n), 2.0 * diff / n


def reservoir(w, u):
    lib = _load()
    w = np.ascontiguousarray(w, np.float64)
    u = np.ascontiguousarray(u, np.float64)
    Wr = C.c_double(0.0)
    R = lib.ora_reservoir(_p(w), _p(u), len(w), C.byref(Wr))
    return R, Wr.value


def dielectric(w_in, ng, ns, ior, u_lobe):
    """One smooth-dielectric scattering event (the oracle's own step):
    returns (code, wo, reflect, F) with code 0 ok, 7 arrival behind the
    shading normal, 8 new direction on the wrong side of the geometric
    normal; wo the outgoing unit direction, F the Fresnel reflectance."""
    lib = _load()
    w_in, ng, ns = (np.ascontiguousarray(a, np.float64) for a in (w_in, ng, ns))
    wo = np.zeros(3)
    refl = C.c_int32(0)
    F = C.c_double(0.0)
    code = lib.ora_dielectric(_p(w_in), _p(ng), _p(ns), float(ior), float(u_lobe), _p(wo), C.byref(refl),
                              C.byref(F))
    return int(code), wo, bool(refl.value), F.value


def ggx_terms(a, cm, cv):
    """GGX D(m) at m.n = cm and Smith G1 at v.n = cv for roughness a."""
    lib = _load()
    D, G1 = C.c_double(), C.c_double()
    lib.ora_ggx_terms(float(a), float(cm), float(cv), C.byref(D), C.byref(G1))
    return D.value, G1.value


def conductor(w_in, n, a, u0, u1):
    """One rough-conductor reflection of wi (unit, pointing away from the
    surface on the side of n): (code, wo, weight f (wo.n)/p over F0); code 7
    (wi misses the drawn microfacet), 8 (wo below the surface), else 0."""
    lib = _load()
    wi = np.ascontiguousarray(w_in, np.float64)
    nn = np.ascontiguousarray(n, np.float64)
    wo = np.zeros(3)
    wgt = C.c_double()
    code = lib.ora_conductor(_p(wi), _p(nn), float(a), float(u0), float(u1), _p(wo), C.byref(wgt))
    return code, wo, wgt.value


def conductor_conn(w_in, wc, n, a):
    """The conductor's connection factor f (wc.n)/F0 = D(h) G1(wi) G1(wc)/(4 wi.n)."""
    lib = _load()
    wi, c, nn = (np.ascontiguousarray(v, np.float64) for v in (w_in, wc, n))
    return lib.ora_conductor_conn(_p(wi), _p(c), _p(nn), float(a))


def philox(seed, ctr):
    lib = _load()
    out = np.zeros(4, np.uint32)
    lib.ora_philox(int(seed), *(int(c) for c in ctr), _p(out, C.c_uint32))
    return out


# ----------------------------------------------------------------- guide
def guide_eval(sc, w, x, n, bf16=True):
    """Raw network outputs [count, 41] at positions x and unit normals n."""
    lib = _load()
    keep = _Keep()
    s = _scene(sc, keep)
    w, x, n = keep.f64(w), keep.f64(x), keep.f64(n)
    out = np.zeros((x.shape[0], GUIDE_OUT))
    lib.ora_guide_eval(C.byref(s), _p(w), _p(x), _p(n), x.shape[0], int(bool(bf16)), _p(out))
    return out


def guide_pdf(o, n, wd):
    """Folded mixture density at directions wd [count, 3] for outputs o [count, 41]."""
    lib = _load()
    o, n, wd = (np.ascontiguousarray(a, np.float64) for a in (o, n, wd))
    pdf = np.zeros(o.shape[0])
    lib.ora_guide_pdf(_p(o), _p(n), _p(wd), o.shape[0], _p(pdf))
    return pdf


def guide_sample(o, n, g):
    """Directions drawn from outputs o [count, 41] with uniforms g [count, 3];
    returns (directions [count, 3], component [count]: 0 cosine, k+1 lobe k)."""
    lib = _load()
    o, n, g = (np.ascontiguousarray(a, np.float64) for a in (o, n, g))
    wd = np.zeros((o.shape[0], 3))
    comp = np.zeros(o.shape[0], np.int32)
    lib.ora_guide_sample(_p(o), _p(n), _p(g), o.shape[0], _p(wd), _p(comp, C.c_int32))
    return wd, comp


def guide_emit(sc, seed, n_paths, guide_w, path_list=None, bf16=True):
    """Guided emission of each path: dict(x, w, pdf, factor, comp)."""
    lib = _load()
    keep = _Keep()
    s = _scene(sc, keep)
    a = _args(seed, n_paths, 1, 0, 1, path_list, keep, guide_w, bf16)
    n = len(path_list) if path_list is not None else int(n_paths)
    rec = np.zeros((n, 8))
    comp = np.zeros(n, np.int32)
    if lib.ora_guide_emit(C.byref(s), C.byref(a), _p(rec), _p(comp, C.c_int32)) != 0:
        raise ValueError("guided emission needs an area emitter and weights")
    return dict(x=rec[:, 0:3], w=rec[:, 3:6], pdf=rec[:, 6], factor=rec[:, 7], comp=comp)


def guide_table(sc, guide_w, bf16=True):
    """The diffuse guide table: raw network outputs per entry [2T, 41]
    (entry 2 texel + side), texel centres x, n [T, 3] and coverage ok [T]."""
    lib = _load()
    keep = _Keep()
    s = _scene(sc, keep)
    a = _args(1, 1, 1, 0, 1, None, keep, guide_w, bf16)
    T = int(sc["n_tex"]) * int(sc["tex_res"]) ** 2
    raw, x, n = np.zeros((2 * T, GUIDE_OUT)), np.zeros((T, 3)), np.zeros((T, 3))
    ok = np.zeros(T, np.uint8)
    rc = lib.ora_guide_table(C.byref(s), C.byref(a), _p(raw), _p(x), _p(n), _p(ok, C.c_uint8))
    assert rc == T
    return dict(raw=raw, x=x, n=n, ok=ok.astype(bool))


def guide_vertex_samples(sc, seed, n_paths, depth, guide_w, path_list=None, bf16=True, threads=0,
                         albedo=None, Le=None):
    """Diffuse-guide training samples [n, 12] (x, n, w, q, S, comp) of each
    path's first guided Lambertian scatter; zero rows for paths without one."""
    lib = _load()
    keep = _Keep()
    s = _scene(sc, keep)
    a = _args(seed, n_paths, depth, 0, threads, path_list, keep, guide_w, bf16, True)
    alb, le, h, nm = _params(sc, albedo, Le, None, keep)
    n = len(path_list) if path_list is not None else int(n_paths)
    out = np.zeros((n, 12))
    if lib.ora_guide_vertex_samples(C.byref(s), C.byref(a), _p(alb), _p(le), _p(h), _p(nm), _p(out)) != 0:
        raise ValueError("diffuse guide samples need an area emitter and weights")
    return out


def guide_loss_grad(sc, w, samples, bf16=True):
    """Training loss -sum (S/q_s) log q(w|x,n) / sum (S/q_s) and its parameter
    gradient.  samples [B, 12] = x (3), n (3), w (3), sampling density q_s, S, unused."""
    lib = _load()
    keep = _Keep()
    s = _scene(sc, keep)
    w, smp = keep.f64(w), keep.f64(samples)
    grad = np.zeros(GUIDE_NPARAMS)
    loss = C.c_double(0.0)
    lib.ora_guide_loss_grad(C.byref(s), _p(w), _p(smp), smp.shape[0], int(bool(bf16)), _p(grad), C.byref(loss))
    return loss.value, grad


def adam(w, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) with bias correction; returns new (w, m, v)."""
    w, g, m, v = (np.asarray(a, np.float64) for a in (w, g, m, v))
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
