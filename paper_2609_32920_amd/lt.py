"""Python binding of the HIP light-tracing library (liblt.so).

Argument marshalling only: every step of the path runs in the library's
gfx950 kernels.  PyTorch provides device memory and the stream.  The
binding refuses to run when the library is missing; there is no CPU
fallback.

The functions carry the C ABI's names (include/lt.h):
  lt_create / lt_scene_upload / lt_trace / lt_loss_l2 /
  lt_backward_naive / lt_backward_reslrb / lt_backward_lrb3 / lt_backward_lrb2 /
  lt_camera_trace / lt_camera_backward_prb /
  lt_guide_eval / lt_guide_emit / lt_guide_vertex_samples / lt_guide_grad / lt_guide_adam /
  lt_guide_train_step /
  lt_batch_create / lt_batch_step / lt_batch_autotune
and ``LightTrace`` wraps forward + a chosen reverse mode as a
``torch.autograd.Function``; ``CameraTrace`` does the same for the camera
side of the bidirectional combination.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblt.so")
# diagnostic build with event counters (byte model of the roofline only)
COUNTERS_LIB_PATH = os.path.join(_HERE, "liblt_counters.so")

LT_OK, LT_ERR_ARG, LT_ERR_OOM, LT_ERR_HIP, LT_ERR_STATE, LT_ERR_UNSUPPORTED = range(6)
ATTACHED, SPLAT_SELECTED, RECORD_TAPE, RECORD_RESERVOIR, CONTRIB_ADJOINT, RECORD_SPLATS = 1, 2, 4, 8, 16, 32
GUIDE_DIFFUSE = 64
CAMERA_ALL = 128
_STATUS = {1: "LT_ERR_ARG", 2: "LT_ERR_OOM", 3: "LT_ERR_HIP", 4: "LT_ERR_STATE", 5: "LT_ERR_UNSUPPORTED"}


class LTError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class SceneDesc(C.Structure):
    _fields_ = [
        ("n_tris", C.c_int32), ("tri_v", C.POINTER(C.c_double)), ("tri_uv", C.POINTER(C.c_double)),
        ("tri_mat", C.POINTER(C.c_int32)),
        ("n_mats", C.c_int32), ("mat_type", C.POINTER(C.c_int32)), ("mat_tex", C.POINTER(C.c_int32)),
        ("mat_ior", C.POINTER(C.c_double)),
        ("n_tex", C.c_int32), ("tex_res", C.c_int32),
        ("em_type", C.c_int32), ("em_o", C.c_double * 3), ("em_e1", C.c_double * 3), ("em_e2", C.c_double * 3),
        ("cam_pos", C.c_double * 3), ("cam_target", C.c_double * 3), ("cam_up", C.c_double * 3),
        ("cam_fov_deg", C.c_double), ("width", C.c_int32), ("height", C.c_int32),
        ("hf_G", C.c_int32), ("hf_x0", C.c_double), ("hf_z0", C.c_double), ("hf_dx", C.c_double),
        ("hf_base", C.c_double), ("hf_mat", C.c_int32), ("em_tex_res", C.c_int32),
    ]


class TraceArgs(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("n_paths", C.c_int64), ("max_depth", C.c_int32),
                ("flags", C.c_uint32), ("path_mask", C.c_void_p), ("path_sig", C.c_void_p),
                ("path_info", C.c_void_p), ("path_contrib", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [("albedo", C.c_void_p), ("emitter_L", C.c_void_p), ("heights", C.c_void_p),
                ("guide_w", C.c_void_p), ("normal_map", C.c_void_p)]


GUIDE_NPARAMS = 11433
GUIDE_NOUT = 41
GUIDE_SAMPLE_FLOATS = 12   # lt_guide_sample: x[3] n[3] w[3] pdf S comp


class Grads(C.Structure):
    _fields_ = [("albedo", C.c_void_p), ("emitter_L", C.c_void_p), ("heights", C.c_void_p),
                ("normal_map", C.c_void_p)]


class Tuning(C.Structure):
    _fields_ = [("block", C.c_int32), ("blocks_per_cu", C.c_int32), ("lds_grad", C.c_int32),
                ("lrb3_split", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("guard_triggers", C.c_uint64), ("nonfinite", C.c_uint64)]


class Instance(C.Structure):
    _fields_ = [("ctx", C.c_void_p), ("args", TraceArgs), ("params", Params), ("target", C.c_void_p),
                ("image", C.c_void_p), ("d_image", C.c_void_p), ("loss", C.c_void_p), ("grads", Grads)]


_libs = {}


def library(path=LIB_PATH):
    """Load liblt.so (raises if it has not been built)."""
    if path not in _libs:
        if not os.path.exists(path):
            raise RuntimeError(f"HIP library not built: {path} (run __graft_entry__.build())")
        lib = C.CDLL(path)
        vp = C.c_void_p
        sig = {
            "lt_create": ([C.c_int, vp, C.POINTER(vp)], C.c_int),
            "lt_destroy": ([vp], None),
            "lt_last_error": ([vp], C.c_char_p),
            "lt_set_stream": ([vp, vp], C.c_int),
            "lt_set_tuning": ([vp, C.POINTER(Tuning)], C.c_int),
            "lt_get_tuning": ([vp, C.POINTER(Tuning)], C.c_int),
            "lt_set_memory_cap": ([vp, C.c_uint64], C.c_int),
            "lt_get_stats": ([vp, C.POINTER(Stats)], C.c_int),
            "lt_read_counters": ([vp, C.POINTER(C.c_uint64), C.c_int], C.c_int),
            "lt_scene_upload": ([vp, C.POINTER(SceneDesc)], C.c_int),
            "lt_side_state_bytes": ([vp, C.POINTER(TraceArgs)], C.c_size_t),
            "lt_workspace_bytes": ([vp, C.POINTER(TraceArgs)], C.c_size_t),
            "lt_trace": ([vp, C.POINTER(TraceArgs), C.POINTER(Params), vp, vp, C.c_size_t], C.c_int),
            "lt_loss_l2": ([vp, vp, vp, C.c_int64, vp, vp], C.c_int),
            "lt_backward_naive": ([vp, C.POINTER(TraceArgs), C.POINTER(Params), vp, vp, C.c_size_t,
                                   C.POINTER(Grads)], C.c_int),
            "lt_backward_reslrb": ([vp, C.POINTER(TraceArgs), C.POINTER(Params), vp, vp, C.c_size_t,
                                    C.POINTER(Grads)], C.c_int),
            "lt_backward_lrb3": ([vp, C.POINTER(TraceArgs), C.POINTER(Params), vp, C.POINTER(Grads)], C.c_int),
            "lt_backward_lrb2": ([vp, C.POINTER(TraceArgs), C.POINTER(Params), vp, vp, C.c_size_t,
                                  C.POINTER(Grads)], C.c_int),
            "lt_backward_lrb3_noalloc": ([vp, C.POINTER(TraceArgs), C.POINTER(Params), vp, C.POINTER(Grads)],
                                         C.c_int),
            "lt_camera_trace": ([vp, C.POINTER(TraceArgs), C.POINTER(Params), vp], C.c_int),
            "lt_camera_backward_prb": ([vp, C.POINTER(TraceArgs), C.POINTER(Params), vp, C.POINTER(Grads)],
                                       C.c_int),
            "lt_guide_eval": ([vp, vp, vp, vp, C.c_int64, vp], C.c_int),
            "lt_guide_emit": ([vp, C.POINTER(TraceArgs), C.POINTER(Params), vp, vp], C.c_int),
            "lt_guide_vertex_samples": ([vp, C.POINTER(TraceArgs), C.POINTER(Params), vp], C.c_int),
            "lt_guide_grad": ([vp, vp, vp, C.c_int64, vp, vp], C.c_int),
            "lt_guide_adam": ([vp, vp, vp, vp, vp, C.c_int32, C.c_float, C.c_float, C.c_float, C.c_float], C.c_int),
            "lt_guide_train_step": ([vp, C.POINTER(TraceArgs), vp, vp, vp, C.c_int64, vp, vp, vp, vp, C.c_int32,
                                     C.c_float, C.c_float, C.c_float, C.c_float], C.c_int),
            "lt_batch_create": ([C.c_int, vp, C.POINTER(vp)], C.c_int),
            "lt_batch_destroy": ([vp], None),
            "lt_batch_last_error": ([vp], C.c_char_p),
            "lt_batch_step": ([vp, C.POINTER(Instance), C.c_int32, C.c_int32], C.c_int),
            "lt_batch_set_tuning": ([vp, C.POINTER(Tuning)], C.c_int),
            "lt_batch_get_tuning": ([vp, C.POINTER(Tuning)], C.c_int),
            "lt_batch_autotune": ([vp, C.POINTER(Instance), C.c_int32, C.c_char_p, C.POINTER(Tuning)], C.c_int),
        }
        for name, (argt, rest) in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = argt
            fn.restype = rest
        _libs[path] = lib
    return _libs[path]


def exported_symbols():
    return ["lt_create", "lt_destroy", "lt_last_error", "lt_set_stream", "lt_set_tuning", "lt_get_tuning",
            "lt_set_memory_cap", "lt_get_stats", "lt_read_counters", "lt_scene_upload", "lt_side_state_bytes",
            "lt_workspace_bytes", "lt_trace", "lt_loss_l2", "lt_backward_naive", "lt_backward_reslrb",
            "lt_backward_lrb3", "lt_backward_lrb2", "lt_backward_lrb3_noalloc", "lt_guide_eval", "lt_guide_emit", "lt_guide_grad", "lt_guide_adam",
            "lt_guide_train_step", "lt_guide_vertex_samples", "lt_camera_trace", "lt_camera_backward_prb",
            "lt_batch_create", "lt_batch_destroy", "lt_batch_last_error", "lt_batch_step", "lt_batch_set_tuning",
            "lt_batch_get_tuning", "lt_batch_autotune"]


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dev_f32(x, device):
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=torch.float32).contiguous()
    return torch.as_tensor(np.asarray(x, np.float32), device=device).contiguous()


class Context:
    """One library context bound to a device; calls run on torch's current
    stream of that device."""

    def __init__(self, device=0, counters=False):
        self.lib = library(COUNTERS_LIB_PATH if counters else LIB_PATH)
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        h = C.c_void_p()
        st = self.lib.lt_create(self.device.index or 0, None, C.byref(h))
        if st != LT_OK:
            raise LTError(st, "lt_create failed")
        self.h = h
        self.scene = None

    def __del__(self):
        try:
            if getattr(self, "h", None):
                self.lib.lt_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def _status(self, st):
        if st != LT_OK:
            raise LTError(st, self.lib.lt_last_error(self.h).decode())

    def _stream(self):
        s = torch.cuda.current_stream(self.device)
        self._status(self.lib.lt_set_stream(self.h, C.c_void_p(s.cuda_stream)))

    def set_tuning(self, block=128, blocks_per_cu=10, lds_grad=1, lrb3_split=2):
        t = Tuning(block, blocks_per_cu, lds_grad, lrb3_split)
        self._status(self.lib.lt_set_tuning(self.h, C.byref(t)))

    def get_tuning(self):
        t = Tuning()
        self._status(self.lib.lt_get_tuning(self.h, C.byref(t)))
        return dict(block=t.block, blocks_per_cu=t.blocks_per_cu, lds_grad=t.lds_grad, lrb3_split=t.lrb3_split)

    def read_counters(self, reset=True):
        """Event counts of the LT_COUNTERS build (see lt_read_counters)."""
        out = (C.c_uint64 * 16)()
        self._status(self.lib.lt_read_counters(self.h, out, int(reset)))
        names = ["rays", "shadow_rays", "nodes", "tris", "splats", "gathers", "grad_values", "paths",
                 "tape_written", "tape_read"]
        return {k: int(out[i]) for i, k in enumerate(names)}

    def set_memory_cap(self, nbytes):
        self._status(self.lib.lt_set_memory_cap(self.h, int(nbytes)))

    def stats(self):
        s = Stats()
        self._status(self.lib.lt_get_stats(self.h, C.byref(s)))
        return dict(guard_triggers=s.guard_triggers, nonfinite=s.nonfinite)

    # ------------------------------------------------------------ scene
    def scene_upload(self, sc):
        keep = []

        def f64(a):
            a = np.ascontiguousarray(a, np.float64)
            keep.append(a)
            return a.ctypes.data_as(C.POINTER(C.c_double))

        def i32(a):
            a = np.ascontiguousarray(a, np.int32)
            keep.append(a)
            return a.ctypes.data_as(C.POINTER(C.c_int32))

        d = SceneDesc()
        d.n_tris = int(np.asarray(sc["tri_v"]).shape[0])
        d.tri_v, d.tri_uv, d.tri_mat = f64(sc["tri_v"]), f64(sc["tri_uv"]), i32(sc["tri_mat"])
        d.n_mats = int(len(sc["mat_type"]))
        d.mat_type, d.mat_tex, d.mat_ior = i32(sc["mat_type"]), i32(sc["mat_tex"]), f64(sc["mat_ior"])
        d.n_tex, d.tex_res = int(sc["n_tex"]), int(sc["tex_res"])
        em = sc["emitter"]
        d.em_type = int(em["type"])
        d.em_tex_res = int(em.get("tex_res", 0))
        cam = sc["camera"]
        for k in range(3):
            d.em_o[k], d.em_e1[k], d.em_e2[k] = float(em["o"][k]), float(em["e1"][k]), float(em["e2"][k])
            d.cam_pos[k], d.cam_target[k], d.cam_up[k] = (float(cam["pos"][k]), float(cam["target"][k]),
                                                          float(cam["up"][k]))
        d.cam_fov_deg = float(cam["fov_deg"])
        d.width, d.height = int(cam["width"]), int(cam["height"])
        hf = sc.get("hf")
        if hf is not None:
            d.hf_G, d.hf_x0, d.hf_z0 = int(hf["G"]), float(hf["x0"]), float(hf["z0"])
            d.hf_dx, d.hf_base, d.hf_mat = float(hf["dx"]), float(hf["base"]), int(hf["mat"])
        self._stream()
        self._status(self.lib.lt_scene_upload(self.h, C.byref(d)))
        self.scene = sc
        self.W, self.H = d.width, d.height
        return self

    # ------------------------------------------------------------ passes
    def args(self, seed, n_paths, depth, flags=0, mask=None, sig=None, info=None, contrib=None):
        a = TraceArgs()
        a.seed, a.n_paths, a.max_depth, a.flags = int(seed), int(n_paths), int(depth), int(flags)
        a.path_mask = None if mask is None else mask.data_ptr()
        a.path_sig = None if sig is None else sig.data_ptr()
        a.path_info = None if info is None else info.data_ptr()
        a.path_contrib = None if contrib is None else contrib.data_ptr()
        return a

    def _sizes(self):
        sc = self.scene
        if sc is None:
            raise LTError(LT_ERR_STATE, "no scene uploaded")
        hf = sc.get("hf")
        G = int(hf["G"]) if hf is not None else 0
        R = int(sc["emitter"].get("tex_res", 0))
        self.n_le = 3 * (R * R if R > 0 else 1)
        return int(sc["n_tex"]) * int(sc["tex_res"]) ** 2 * 3, G * G

    def _check(self, t, name, numel):
        """A parameter or gradient array the kernels read or write through a
        raw pointer: float32, contiguous, on this context's device, with the
        element count the uploaded scene implies."""
        if t is None:
            return
        if not isinstance(t, torch.Tensor):
            raise ValueError(f"{name} must be a torch tensor")
        if t.dtype != torch.float32:
            raise ValueError(f"{name} must be float32, got {t.dtype}")
        if t.device.type != "cuda" or (t.device.index or 0) != (self.device.index or 0):
            raise ValueError(f"{name} must live on {self.device}, got {t.device}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if t.numel() != numel:
            raise ValueError(f"{name} has {t.numel()} elements, the scene needs {numel}")

    def params(self, albedo, Le, heights=None, guide_w=None, normal_map=None):
        n_alb, n_h = self._sizes()
        self._check(albedo, "albedo", n_alb)
        self._check(Le, "Le", self.n_le)
        if heights is not None:
            self._check(heights, "heights", n_h)
        self._check(guide_w, "guide_w", GUIDE_NPARAMS)
        self._check(normal_map, "normal_map", 2 * n_h)
        return Params(albedo.data_ptr(), Le.data_ptr(), None if heights is None else heights.data_ptr(),
                      None if guide_w is None else guide_w.data_ptr(),
                      None if normal_map is None else normal_map.data_ptr())

    def side_state_bytes(self, a):
        return int(self.lib.lt_side_state_bytes(self.h, C.byref(a)))

    def workspace_bytes(self, a):
        return int(self.lib.lt_workspace_bytes(self.h, C.byref(a)))

    def trace(self, a, p, image, side=None):
        self._stream()
        nb = 0 if side is None else side.numel() * side.element_size()
        self._status(self.lib.lt_trace(self.h, C.byref(a), C.byref(p), _ptr(image), _ptr(side), nb))

    def loss_l2(self, image, target, d_image, loss):
        self._stream()
        self._status(self.lib.lt_loss_l2(self.h, _ptr(image), _ptr(target), image.numel(), _ptr(d_image),
                                        _ptr(loss)))

    def _grads(self, g_albedo, g_Le, g_heights, g_normal_map=None):
        n_alb, n_h = self._sizes()
        self._check(g_albedo, "g_albedo", n_alb)
        self._check(g_Le, "g_Le", self.n_le)
        self._check(g_heights, "g_heights", n_h)
        self._check(g_normal_map, "g_normal_map", 2 * n_h)
        return Grads(None if g_albedo is None else g_albedo.data_ptr(),
                     None if g_Le is None else g_Le.data_ptr(),
                     None if g_heights is None else g_heights.data_ptr(),
                     None if g_normal_map is None else g_normal_map.data_ptr())

    def backward_naive(self, a, p, d_image, tape, g_albedo, g_Le, g_heights=None,
                     g_normal_map=None):
        self._stream()
        g = self._grads(g_albedo, g_Le, g_heights, g_normal_map)
        nb = tape.numel() * tape.element_size()
        self._status(self.lib.lt_backward_naive(self.h, C.byref(a), C.byref(p), _ptr(d_image), _ptr(tape), nb,
                                               C.byref(g)))

    def backward_reslrb(self, a, p, d_image, records, g_albedo, g_Le, g_heights=None,
                     g_normal_map=None):
        self._stream()
        g = self._grads(g_albedo, g_Le, g_heights, g_normal_map)
        nb = records.numel() * records.element_size()
        self._status(self.lib.lt_backward_reslrb(self.h, C.byref(a), C.byref(p), _ptr(d_image), _ptr(records),
                                                nb, C.byref(g)))

    def backward_lrb2(self, a, p, d_image, records, g_albedo, g_Le):
        self._stream()
        g = self._grads(g_albedo, g_Le, None)
        nb = records.numel() * records.element_size()
        self._status(self.lib.lt_backward_lrb2(self.h, C.byref(a), C.byref(p), _ptr(d_image), _ptr(records), nb,
                                               C.byref(g)))

    def backward_lrb3(self, a, p, d_image, g_albedo, g_Le, g_heights=None, g_normal_map=None):
        self._stream()
        g = self._grads(g_albedo, g_Le, g_heights, g_normal_map)
        self._status(self.lib.lt_backward_lrb3(self.h, C.byref(a), C.byref(p), _ptr(d_image), C.byref(g)))

    def backward_lrb3_noalloc(self, a, p, d_image, g_albedo, g_Le, g_heights=None, g_normal_map=None):
        """lt_backward_lrb3_noalloc: the LRB-3 backward with its working memory
        in the library's static device scratch (no allocation)."""
        self._stream()
        g = self._grads(g_albedo, g_Le, g_heights, g_normal_map)
        self._status(self.lib.lt_backward_lrb3_noalloc(self.h, C.byref(a), C.byref(p), _ptr(d_image), C.byref(g)))

    def camera_trace(self, a, p, image):
        """lt_camera_trace: adds the camera samples' estimate to image."""
        self._stream()
        self._status(self.lib.lt_camera_trace(self.h, C.byref(a), C.byref(p), _ptr(image)))

    def camera_backward_prb(self, a, p, d_image, g_albedo, g_Le):
        """lt_camera_backward_prb: path-replay gradients of the camera samples
        (accumulated)."""
        self._stream()
        g = self._grads(g_albedo, g_Le, None)
        self._status(self.lib.lt_camera_backward_prb(self.h, C.byref(a), C.byref(p), _ptr(d_image), C.byref(g)))

    # ------------------------------------------------------------ guide
    def guide_eval(self, guide_w, x, n, out):
        """Raw network outputs out [count, 41] at x, n [count, 3] (device float32)."""
        self._stream()
        self._status(self.lib.lt_guide_eval(self.h, _ptr(guide_w), _ptr(x), _ptr(n), x.shape[0], _ptr(out)))

    def guide_emit(self, a, p, samples, contrib=None):
        """Guided emission of paths [0, n_paths) as samples [n_paths, 12]."""
        self._stream()
        self._status(self.lib.lt_guide_emit(self.h, C.byref(a), C.byref(p), _ptr(contrib), _ptr(samples)))

    def guide_vertex_samples(self, a, p, samples):
        """Diffuse-guide training samples [n_paths, 12]: each path's first
        guided Lambertian scatter with the luminance of its later connections."""
        self._stream()
        self._status(self.lib.lt_guide_vertex_samples(self.h, C.byref(a), C.byref(p), _ptr(samples)))

    def guide_grad(self, guide_w, samples, grad, loss=None):
        """Training loss and gradient over samples [count, 12] (device float32)."""
        self._stream()
        self._status(self.lib.lt_guide_grad(self.h, _ptr(guide_w), _ptr(samples), samples.shape[0], _ptr(grad),
                                           _ptr(loss)))

    def guide_adam(self, w, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self._stream()
        self._status(self.lib.lt_guide_adam(self.h, _ptr(w), _ptr(grad), _ptr(m), _ptr(v), int(step), float(lr),
                                           float(beta1), float(beta2), float(eps)))

    def guide_train_step(self, a, guide_w, contrib, samples, grad, m, v, step, lr, loss=None, beta1=0.9,
                         beta2=0.999, eps=1e-8):
        """Emission samples paired with contrib, loss gradient and one Adam
        step on guide_w in place (samples: [n_samples, 12] device float32)."""
        self._stream()
        self._status(self.lib.lt_guide_train_step(self.h, C.byref(a), _ptr(guide_w), _ptr(contrib), _ptr(samples),
                                                 samples.shape[0], _ptr(grad), _ptr(m), _ptr(v), _ptr(loss),
                                                 int(step), float(lr), float(beta1), float(beta2), float(eps)))


class Batch:
    """Runner of batched optimisation steps (lt_batch_*) on torch's current
    stream of `device`.  An instance is a dict with keys ctx (Context), seed,
    n_paths, depth, attached (bool), albedo, Le, heights, guide (tensors or
    None), target, image, d_image, loss, g_albedo, g_Le, g_heights, and
    optionally mask (uint8 [n_paths] on the device, as lt_trace's path mask)."""

    def __init__(self, device=0):
        self.lib = library(LIB_PATH)
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        h = C.c_void_p()
        s = torch.cuda.current_stream(self.device)
        st = self.lib.lt_batch_create(self.device.index or 0, C.c_void_p(s.cuda_stream), C.byref(h))
        if st != LT_OK:
            raise LTError(st, "lt_batch_create failed")
        self.h = h

    def __del__(self):
        try:
            if getattr(self, "h", None):
                self.lib.lt_batch_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def _check(self, st):
        if st != LT_OK:
            raise LTError(st, self.lib.lt_batch_last_error(self.h).decode())

    @staticmethod
    def table(instances):
        arr = (Instance * len(instances))()
        for k, d in enumerate(instances):
            ctx = d["ctx"]
            arr[k].ctx = ctx.h
            arr[k].args = ctx.args(d["seed"], d["n_paths"], d["depth"], ATTACHED if d.get("attached") else 0,
                                   d.get("mask"))
            arr[k].params = ctx.params(d["albedo"], d["Le"], d.get("heights"), d.get("guide"), d.get("normal_map"))
            arr[k].target, arr[k].image = d["target"].data_ptr(), d["image"].data_ptr()
            arr[k].d_image, arr[k].loss = d["d_image"].data_ptr(), d["loss"].data_ptr()
            arr[k].grads = ctx._grads(d["g_albedo"], d.get("g_Le"), d.get("g_heights"), d.get("g_normal_map"))
        return arr

    def step(self, instances, use_graph=True, table=None):
        arr = table if table is not None else self.table(instances)
        self._check(self.lib.lt_batch_step(self.h, arr, len(arr), int(bool(use_graph))))

    def set_tuning(self, block=256, blocks_per_cu=4, lds_grad=1):
        t = Tuning(block, blocks_per_cu, lds_grad, 0)
        self._check(self.lib.lt_batch_set_tuning(self.h, C.byref(t)))

    def get_tuning(self):
        t = Tuning()
        self._check(self.lib.lt_batch_get_tuning(self.h, C.byref(t)))
        return dict(block=t.block, blocks_per_cu=t.blocks_per_cu, lds_grad=t.lds_grad)

    def autotune(self, instances, cache_path=None):
        arr = self.table(instances)
        t = Tuning()
        self._check(self.lib.lt_batch_autotune(self.h, arr, len(arr),
                                               None if cache_path is None else str(cache_path).encode(), C.byref(t)))
        return dict(block=t.block, blocks_per_cu=t.blocks_per_cu, lds_grad=t.lds_grad)


# C-ABI names as module-level functions -------------------------------------
def lt_create(device=0):
    return Context(device)


def lt_scene_upload(ctx, scene):
    return ctx.scene_upload(scene)


def lt_trace(ctx, args, params, image, side=None):
    return ctx.trace(args, params, image, side)


def lt_loss_l2(ctx, image, target, d_image, loss):
    return ctx.loss_l2(image, target, d_image, loss)


def lt_backward_naive(ctx, args, params, d_image, tape, g_albedo, g_Le, g_heights=None):
    return ctx.backward_naive(args, params, d_image, tape, g_albedo, g_Le, g_heights)


def lt_backward_reslrb(ctx, args, params, d_image, records, g_albedo, g_Le, g_heights=None):
    return ctx.backward_reslrb(args, params, d_image, records, g_albedo, g_Le, g_heights)


def lt_backward_lrb2(ctx, args, params, d_image, records, g_albedo, g_Le):
    return ctx.backward_lrb2(args, params, d_image, records, g_albedo, g_Le)


def lt_backward_lrb3(ctx, args, params, d_image, g_albedo, g_Le, g_heights=None):
    return ctx.backward_lrb3(args, params, d_image, g_albedo, g_Le, g_heights)


def lt_camera_trace(ctx, args, params, image):
    return ctx.camera_trace(args, params, image)


def lt_camera_backward_prb(ctx, args, params, d_image, g_albedo, g_Le):
    return ctx.camera_backward_prb(args, params, d_image, g_albedo, g_Le)


def lt_guide_eval(ctx, guide_w, x, n, out):
    return ctx.guide_eval(guide_w, x, n, out)


def lt_guide_emit(ctx, args, params, samples, contrib=None):
    return ctx.guide_emit(args, params, samples, contrib)


def lt_guide_vertex_samples(ctx, args, params, samples):
    return ctx.guide_vertex_samples(args, params, samples)


def lt_guide_grad(ctx, guide_w, samples, grad, loss=None):
    return ctx.guide_grad(guide_w, samples, grad, loss)


def lt_guide_adam(ctx, w, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    return ctx.guide_adam(w, grad, m, v, step, lr, beta1, beta2, eps)


def lt_guide_train_step(ctx, a, guide_w, contrib, samples, grad, m, v, step, lr, loss=None, beta1=0.9,
                        beta2=0.999, eps=1e-8):
    return ctx.guide_train_step(a, guide_w, contrib, samples, grad, m, v, step, lr, loss, beta1, beta2, eps)


def lt_batch_create(device=0):
    return Batch(device)


def lt_batch_step(batch, instances, use_graph=True):
    return batch.step(instances, use_graph)


def lt_batch_autotune(batch, instances, cache_path=None):
    return batch.autotune(instances, cache_path)


# ------------------------------------------------------------ autograd
MODES = ("naive", "reslrb", "lrb3", "lrb2")


class CameraTrace(torch.autograd.Function):
    """image = CameraTrace.apply(albedo, Le, heights, ctx, seed, n_samples, depth, flags, mask)

    The camera side of the bidirectional combination: lt_camera_trace into a
    zeroed image forward, lt_camera_backward_prb with the incoming image
    adjoint backward (path replay: nothing is kept between the two but the
    arguments).  Without CAMERA_ALL in flags only samples whose first vertex
    is specular contribute, so that
        LightTrace.apply(...) + CameraTrace.apply(...)
    estimates the whole image, each path through exactly one of the two.
    Detached: albedo and Le receive gradients, heights (the geometry the
    samples see, or None) none.  mask (optional, uint8 [n_samples]):
    samples whose byte is 0 contribute nothing.
    """

    @staticmethod
    def forward(fctx, albedo, Le, heights, ctx, seed, n_samples, depth, flags=0, mask=None):
        if mask is not None and (mask.dtype != torch.uint8 or mask.numel() != n_samples or not mask.is_contiguous()):
            raise ValueError("mask must be a contiguous uint8 tensor with one byte per sample")
        a = ctx.args(seed, n_samples, depth, flags, mask)
        p = ctx.params(albedo, Le, heights)
        image = torch.zeros((ctx.H, ctx.W, 3), dtype=torch.float32, device=albedo.device)
        ctx.camera_trace(a, p, image)
        fctx.lt = (ctx, seed, n_samples, depth, flags, mask)
        fctx.save_for_backward(albedo, Le, heights if heights is not None else torch.empty(0, device=albedo.device))
        return image

    @staticmethod
    def backward(fctx, grad_image):
        ctx, seed, n_samples, depth, flags, mask = fctx.lt
        albedo, Le, heights = fctx.saved_tensors
        heights = heights if heights.numel() else None
        a = ctx.args(seed, n_samples, depth, flags, mask)
        p = ctx.params(albedo, Le, heights)
        dI = grad_image.to(torch.float32).contiguous()
        g_alb = torch.zeros_like(albedo)
        g_le = torch.zeros_like(Le)
        ctx.camera_backward_prb(a, p, dI, g_alb, g_le)
        return g_alb, g_le, None, None, None, None, None, None, None


class LightTrace(torch.autograd.Function):
    """image = LightTrace.apply(albedo, Le, heights, ctx, seed, n_paths, depth, mode, flags, mask)

    Forward runs lt_trace (recording the tape for "naive", the reservoir
    records for "reslrb" or the splat records for "lrb2", the buffered
    two-pass variant); backward runs the matching lt_backward_* with the
    incoming image adjoint.  Seed replay is the recomputation: "lrb3" keeps
    no side state at all.  mask (optional, uint8 [n_paths] on the device):
    paths whose byte is 0 contribute nothing to the image or the gradients.
    """

    @staticmethod
    def forward(fctx, albedo, Le, heights, ctx, seed, n_paths, depth, mode="lrb3", flags=0, mask=None):
        if mode not in MODES:
            raise ValueError(mode)
        if mask is not None and (mask.dtype != torch.uint8 or mask.numel() != n_paths or not mask.is_contiguous()):
            raise ValueError("mask must be a contiguous uint8 tensor with one byte per path")
        rec = {"naive": RECORD_TAPE, "reslrb": RECORD_RESERVOIR, "lrb2": RECORD_SPLATS}.get(mode, 0)
        a = ctx.args(seed, n_paths, depth, flags | rec, mask)
        p = ctx.params(albedo, Le, heights)
        nb = ctx.side_state_bytes(a)
        side = torch.empty(max(nb, 1), dtype=torch.uint8, device=albedo.device) if nb else None
        image = torch.empty((ctx.H, ctx.W, 3), dtype=torch.float32, device=albedo.device)
        ctx.trace(a, p, image, side)
        fctx.lt = (ctx, seed, n_paths, depth, mode, flags | rec, side, mask)
        fctx.save_for_backward(albedo, Le, heights if heights is not None else torch.empty(0, device=albedo.device))
        return image

    @staticmethod
    def backward(fctx, grad_image):
        ctx, seed, n_paths, depth, mode, flags, side, mask = fctx.lt
        albedo, Le, heights = fctx.saved_tensors
        heights = heights if heights.numel() else None
        a = ctx.args(seed, n_paths, depth, flags, mask)
        p = ctx.params(albedo, Le, heights)
        dI = grad_image.to(torch.float32).contiguous()
        g_alb = torch.zeros_like(albedo)
        g_le = torch.zeros_like(Le)
        g_h = torch.zeros_like(heights) if heights is not None else None
        if mode == "naive":
            ctx.backward_naive(a, p, dI, side, g_alb, g_le, g_h)
        elif mode == "reslrb":
            ctx.backward_reslrb(a, p, dI, side, g_alb, g_le, g_h)
        elif mode == "lrb2":
            ctx.backward_lrb2(a, p, dI, side, g_alb, g_le)
        else:
            ctx.backward_lrb3(a, p, dI, g_alb, g_le, g_h)
        return g_alb, g_le, g_h, None, None, None, None, None, None, None
