"""ctypes binding of ``libmfadvr.so`` (C ABI declared in include/mfa_dvr.h).

Argument marshalling only: every step of rendering and evaluation runs in
the library's HIP kernels.  The functions carry the C names; descriptors are
built from any object with the fields of the C structs (for example the
records in ``workloads``), device buffers are torch CUDA tensors, and a
non-zero status raises ``MFAError``.  The library must have been built
(``python -m paper_2204_11762_amd.build``); importing this module without it
raises, there is no fallback.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmfadvr.so")

MFA_OK = 0
MFA_ERR_INVALID = -1
MFA_ERR_MODEL = -2
MFA_ERR_NOMEM = -3
MFA_ERR_DEVICE = -4
MFA_ERR_HANDLE = -5
MFA_ERR_TIMEOUT = -6
STATUS_NAMES = {0: "MFA_OK", -1: "MFA_ERR_INVALID", -2: "MFA_ERR_MODEL", -3: "MFA_ERR_NOMEM",
                -4: "MFA_ERR_DEVICE", -5: "MFA_ERR_HANDLE", -6: "MFA_ERR_TIMEOUT"}
MFA_STORE_F32 = 0
MFA_STORE_BF16 = 1
MFA_STORE_F16 = 2
MFA_CAMERA_ORTHO = 0
MFA_CAMERA_PERSP = 1

EXPORTED = ("mfa_create", "mfa_destroy", "mfa_set_memory_budget", "mfa_model_upload",
            "mfa_model_free", "mfa_model_bytes", "mfa_render", "mfa_render_curvature",
            "mfa_eval_points", "mfa_eval_hessian", "mfa_kernel_timing", "mfa_kernel_times",
            "mfa_measure_fma_peak", "mfa_autotune", "mfa_batch_create", "mfa_batch_render",
            "mfa_batch_free", "mfa_server_create", "mfa_server_submit", "mfa_server_wait",
            "mfa_server_destroy", "mfa_validate_model", "mfa_validate_render", "mfa_last_error",
            "mfa_version", "mfa_render_noalloc", "mfa_model_set_tuning")


class MFAError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.message = message


class ModelDesc(C.Structure):
    _fields_ = [("degree", C.c_int32 * 3), ("store", C.c_int32), ("n_ctrl", C.c_int64 * 3),
                ("knots", C.POINTER(C.c_double) * 3), ("ctrl", C.POINTER(C.c_double)),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("weights", C.POINTER(C.c_double))]


class Camera(C.Structure):
    _fields_ = [("kind", C.c_int32), ("width", C.c_int32), ("height", C.c_int32),
                ("reserved", C.c_int32), ("eye", C.c_double * 3), ("target", C.c_double * 3),
                ("up", C.c_double * 3), ("fov_y_deg", C.c_double), ("ortho_half_w", C.c_double),
                ("ortho_half_h", C.c_double)]


class TF(C.Structure):
    _fields_ = [("n", C.c_int32), ("reserved", C.c_int32), ("rgba", C.POINTER(C.c_float)),
                ("v_lo", C.c_double), ("v_hi", C.c_double)]


class CurvatureTF(C.Structure):
    _fields_ = [("m", C.c_int32), ("reserved", C.c_int32), ("rgba", C.POINTER(C.c_float)),
                ("k_lo", C.c_double), ("k_hi", C.c_double)]


class RenderParams(C.Structure):
    _fields_ = [("step", C.c_double), ("ert_alpha", C.c_double), ("shading", C.c_int32),
                ("shininess", C.c_int32), ("headlight", C.c_int32), ("reserved", C.c_int32),
                ("ka", C.c_double), ("kd", C.c_double), ("ks", C.c_double),
                ("light_dir", C.c_double * 3)]


class RenderRequest(C.Structure):
    _fields_ = [("model", C.c_int64), ("camera", C.POINTER(Camera)), ("tf", C.POINTER(TF)),
                ("params", C.POINTER(RenderParams)), ("rgba_dev", C.c_void_p),
                ("samples_dev", C.c_void_p)]


class TuneResult(C.Structure):
    _fields_ = [("round_spans", C.c_float), ("candidates", C.c_int32), ("best_ms", C.c_float),
                ("default_ms", C.c_float), ("lanes_per_ray", C.c_int32)]


class ServerConfig(C.Structure):
    _fields_ = [("streams", C.c_int32), ("max_batch", C.c_int32), ("max_bytes", C.c_int64)]


class RequestInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("batch_size", C.c_int32), ("submit_ns", C.c_int64),
                ("launch_ns", C.c_int64), ("done_ns", C.c_int64), ("deferred", C.c_int32),
                ("reserved", C.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2204_11762_amd.build` (no CPU fallback exists)")
    lib = C.CDLL(LIB_PATH)
    st = C.c_int32
    vp = C.c_void_p
    i64 = C.c_int64
    sig = {
        "mfa_create": (st, [C.c_int32, C.POINTER(vp)]),
        "mfa_destroy": (st, [vp]),
        "mfa_set_memory_budget": (st, [vp, i64]),
        "mfa_model_upload": (st, [vp, C.POINTER(ModelDesc), C.POINTER(i64)]),
        "mfa_model_free": (st, [vp, i64]),
        "mfa_model_bytes": (st, [vp, i64, C.POINTER(i64)]),
        "mfa_render": (st, [vp, i64, C.POINTER(Camera), C.POINTER(TF), C.POINTER(RenderParams),
                            vp, vp, vp]),
        "mfa_render_noalloc": (st, [vp, i64, C.POINTER(Camera), C.POINTER(TF),
                                    C.POINTER(RenderParams), vp, vp, vp]),
        "mfa_render_curvature": (st, [vp, i64, C.POINTER(Camera), C.POINTER(TF),
                                      C.POINTER(CurvatureTF), C.POINTER(RenderParams),
                                      vp, vp, vp]),
        "mfa_eval_points": (st, [vp, i64, i64, vp, vp, vp, vp]),
        "mfa_eval_hessian": (st, [vp, i64, i64, vp, vp, vp, vp, vp]),
        "mfa_kernel_timing": (st, [vp, C.c_int32]),
        "mfa_autotune": (st, [vp, i64, C.POINTER(Camera), C.POINTER(TF), C.POINTER(RenderParams),
                              vp, C.c_int32, vp, C.POINTER(TuneResult)]),
        "mfa_model_set_tuning": (st, [vp, i64, C.c_float, C.c_int32]),
        "mfa_batch_create": (st, [vp, C.POINTER(RenderRequest), C.c_int32, C.POINTER(i64)]),
        "mfa_batch_render": (st, [vp, i64, vp]),
        "mfa_batch_free": (st, [vp, i64]),
        "mfa_server_create": (st, [vp, C.POINTER(ServerConfig), C.POINTER(vp)]),
        "mfa_server_submit": (st, [vp, C.POINTER(RenderRequest), C.POINTER(i64)]),
        "mfa_server_wait": (st, [vp, i64, i64, C.POINTER(RequestInfo)]),
        "mfa_server_destroy": (st, [vp]),
        "mfa_kernel_times": (st, [vp, vp, i64, C.POINTER(i64)]),
        "mfa_measure_fma_peak": (st, [vp, C.POINTER(C.c_double)]),
        "mfa_validate_model": (st, [C.POINTER(ModelDesc)]),
        "mfa_validate_render": (st, [C.POINTER(Camera), C.POINTER(TF), C.POINTER(RenderParams)]),
        "mfa_last_error": (C.c_char_p, []),
        "mfa_version": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def last_error() -> str:
    return lib.mfa_last_error().decode()


def _check(status: int) -> None:
    if status != MFA_OK:
        raise MFAError(status, last_error())


# ---------------------------------------------------------------------------
# descriptor marshalling
# ---------------------------------------------------------------------------

class _Keep:
    """Host arrays referenced by a descriptor, kept alive for the call."""

    def __init__(self):
        self.refs = []

    def f64(self, a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        self.refs.append(a)
        return a.ctypes.data_as(C.POINTER(C.c_double))

    def f32(self, a):
        a = np.ascontiguousarray(a, dtype=np.float32)
        self.refs.append(a)
        return a.ctypes.data_as(C.POINTER(C.c_float))


def model_desc(spec, store: int = MFA_STORE_F32, keep: _Keep | None = None) -> tuple:
    """(ModelDesc, keep) from an object with degree, knots, ctrl, lo, hi.
    ``ctrl`` is (n_z, n_y, n_x), x fastest."""
    keep = keep or _Keep()
    d = ModelDesc()
    ctrl = np.asarray(spec.ctrl)
    nz, ny, nx = ctrl.shape
    for k in range(3):
        d.degree[k] = int(spec.degree[k])
        d.knots[k] = keep.f64(spec.knots[k])
        d.lo[k] = float(spec.lo[k])
        d.hi[k] = float(spec.hi[k])
    d.n_ctrl[0], d.n_ctrl[1], d.n_ctrl[2] = nx, ny, nz
    d.ctrl = keep.f64(ctrl.reshape(-1))
    w = getattr(spec, "weights", None)
    if w is not None:
        w = np.asarray(w, dtype=np.float64)
        if w.shape != ctrl.shape:
            raise ValueError("weights must have the shape of ctrl")
        d.weights = keep.f64(w.reshape(-1))
    d.store = int(store)
    return d, keep


def camera_struct(cam) -> Camera:
    c = Camera()
    c.kind = MFA_CAMERA_ORTHO if cam.kind == "ortho" else MFA_CAMERA_PERSP
    c.width, c.height = int(cam.width), int(cam.height)
    for k in range(3):
        c.eye[k] = float(cam.eye[k])
        c.target[k] = float(cam.target[k])
        c.up[k] = float(cam.up[k])
    c.fov_y_deg = float(cam.fov_y_deg)
    c.ortho_half_w = float(cam.ortho_half_w)
    c.ortho_half_h = float(cam.ortho_half_h)
    return c


def tf_struct(tf, keep: _Keep | None = None) -> tuple:
    keep = keep or _Keep()
    t = TF()
    table = np.asarray(tf.table, dtype=np.float32)
    t.n = int(table.shape[0])
    t.rgba = keep.f32(table.reshape(-1))
    t.v_lo = float(tf.v_lo)
    t.v_hi = float(tf.v_hi)
    return t, keep


def params_struct(p) -> RenderParams:
    r = RenderParams()
    r.step = float(p.step)
    r.ert_alpha = float(p.ert_alpha)
    r.shading = int(bool(p.shading))
    r.shininess = int(p.shininess)
    r.headlight = int(bool(p.headlight))
    r.ka, r.kd, r.ks = float(p.ka), float(p.kd), float(p.ks)
    for k in range(3):
        r.light_dir[k] = float(p.light_dir[k])
    return r


# ---------------------------------------------------------------------------
# entry points (same names as the C ABI)
# ---------------------------------------------------------------------------

def mfa_version() -> str:
    return lib.mfa_version().decode()


def mfa_create(device: int = 0) -> int:
    ctx = C.c_void_p()
    _check(lib.mfa_create(int(device), C.byref(ctx)))
    return ctx.value


def mfa_destroy(ctx: int) -> None:
    _check(lib.mfa_destroy(ctx))


def mfa_set_memory_budget(ctx: int, nbytes: int) -> None:
    _check(lib.mfa_set_memory_budget(ctx, int(nbytes)))


def mfa_validate_model(spec, store: int = MFA_STORE_F32) -> None:
    d, keep = model_desc(spec, store)
    _check(lib.mfa_validate_model(C.byref(d)))


def mfa_validate_render(camera, tf, params) -> None:
    t, keep = tf_struct(tf)
    _check(lib.mfa_validate_render(C.byref(camera_struct(camera)), C.byref(t),
                                   C.byref(params_struct(params))))


def mfa_model_upload(ctx: int, spec, store: int = MFA_STORE_F32) -> int:
    d, keep = model_desc(spec, store)
    h = C.c_int64()
    _check(lib.mfa_model_upload(ctx, C.byref(d), C.byref(h)))
    return h.value


def mfa_model_free(ctx: int, model: int) -> None:
    _check(lib.mfa_model_free(ctx, int(model)))


def mfa_model_bytes(ctx: int, model: int) -> int:
    b = C.c_int64()
    _check(lib.mfa_model_bytes(ctx, int(model), C.byref(b)))
    return b.value


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _dev_tensor(t, dtype, shape, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} tensor of shape {tuple(shape)}")
    return t.data_ptr()


def mfa_render(ctx: int, model: int, camera, tf, params, rgba, samples=None, stream=None) -> None:
    """Render into ``rgba`` (H, W, 4) float32; ``samples`` an int64 tensor of
    one element or None."""
    import torch
    out = _dev_tensor(rgba, torch.float32, (camera.height, camera.width, 4), "rgba")
    sp = None
    if samples is not None:
        sp = _dev_tensor(samples, torch.int64, (1,), "samples")
    t, keep = tf_struct(tf)
    _check(lib.mfa_render(ctx, int(model), C.byref(camera_struct(camera)), C.byref(t),
                          C.byref(params_struct(params)), out, sp, _stream_ptr(stream)))


def mfa_render_noalloc(ctx: int, model: int, camera, tf, params, rgba, samples=None,
                       stream=None) -> None:
    """As mfa_render, without device allocation (the library's fixed
    scratch array; overlapping calls on one GPU race)."""
    import torch
    out = _dev_tensor(rgba, torch.float32, (camera.height, camera.width, 4), "rgba")
    sp = None
    if samples is not None:
        sp = _dev_tensor(samples, torch.int64, (1,), "samples")
    t, keep = tf_struct(tf)
    _check(lib.mfa_render_noalloc(ctx, int(model), C.byref(camera_struct(camera)), C.byref(t),
                                  C.byref(params_struct(params)), out, sp, _stream_ptr(stream)))


def curvature_struct(ctf, keep: _Keep | None = None) -> tuple:
    """(CurvatureTF, keep) from an object with table (m, m, 4), k_lo, k_hi."""
    keep = keep or _Keep()
    table = np.asarray(ctf.table, dtype=np.float32)
    c = CurvatureTF()
    c.m = int(table.shape[0])
    c.rgba = keep.f32(table.reshape(-1))
    c.k_lo = float(ctf.k_lo)
    c.k_hi = float(ctf.k_hi)
    return c, keep


def mfa_render_curvature(ctx: int, model: int, camera, tf, curvature, params, rgba,
                         samples=None, stream=None) -> None:
    """Render with a curvature transfer function (``curvature``: table
    (m, m, 4), k_lo, k_hi) into ``rgba`` (H, W, 4) float32."""
    import torch
    out = _dev_tensor(rgba, torch.float32, (camera.height, camera.width, 4), "rgba")
    sp = None
    if samples is not None:
        sp = _dev_tensor(samples, torch.int64, (1,), "samples")
    t, keep = tf_struct(tf)
    c, keep = curvature_struct(curvature, keep)
    _check(lib.mfa_render_curvature(ctx, int(model), C.byref(camera_struct(camera)), C.byref(t),
                                    C.byref(c), C.byref(params_struct(params)), out, sp,
                                    _stream_ptr(stream)))


def mfa_autotune(ctx: int, model: int, camera, tf, params, rgba, repeats: int = 5, stream=None):
    """Tune the model's round length and lanes per ray on one request (rgba
    is overwritten); returns the TuneResult."""
    import torch
    out = _dev_tensor(rgba, torch.float32, (camera.height, camera.width, 4), "rgba")
    t, keep = tf_struct(tf)
    res = TuneResult()
    _check(lib.mfa_autotune(ctx, int(model), C.byref(camera_struct(camera)), C.byref(t),
                            C.byref(params_struct(params)), out, int(repeats), _stream_ptr(stream),
                            C.byref(res)))
    return res


def mfa_model_set_tuning(ctx: int, model: int, round_spans: float, lanes_per_ray: int) -> None:
    """Set the model's round length and lanes per ray (what mfa_autotune
    chooses)."""
    _check(lib.mfa_model_set_tuning(ctx, int(model), float(round_spans), int(lanes_per_ray)))


def mfa_batch_create(ctx: int, requests) -> int:
    """Prepare a batch from ``requests``: a sequence of (model, camera, tf,
    params, rgba, samples) with ``rgba`` an (H, W, 4) float32 CUDA tensor and
    ``samples`` a one-element int64 CUDA tensor or None.  The tensors must
    outlive the batch."""
    import torch
    reqs = list(requests)
    arr = (RenderRequest * len(reqs))()
    keep = []
    for i, (model, cam, tf, params, rgba, samples) in enumerate(reqs):
        c = camera_struct(cam)
        t, k = tf_struct(tf)
        p = params_struct(params)
        keep += [c, t, k, p]
        arr[i].model = int(model)
        arr[i].camera = C.pointer(c)
        arr[i].tf = C.pointer(t)
        arr[i].params = C.pointer(p)
        arr[i].rgba_dev = _dev_tensor(rgba, torch.float32, (cam.height, cam.width, 4), "rgba")
        arr[i].samples_dev = (None if samples is None
                              else _dev_tensor(samples, torch.int64, (1,), "samples"))
    h = C.c_int64()
    _check(lib.mfa_batch_create(ctx, arr, len(reqs), C.byref(h)))
    return h.value


def mfa_batch_render(ctx: int, batch: int, stream=None) -> None:
    _check(lib.mfa_batch_render(ctx, int(batch), _stream_ptr(stream)))


def mfa_batch_free(ctx: int, batch: int) -> None:
    _check(lib.mfa_batch_free(ctx, int(batch)))


def _request_struct(model, cam, tf, params, rgba, samples, keep):
    import torch
    c = camera_struct(cam)
    t, k = tf_struct(tf)
    p = params_struct(params)
    keep += [c, t, k, p]
    r = RenderRequest()
    r.model = int(model)
    r.camera = C.pointer(c)
    r.tf = C.pointer(t)
    r.params = C.pointer(p)
    r.rgba_dev = _dev_tensor(rgba, torch.float32, (cam.height, cam.width, 4), "rgba")
    r.samples_dev = None if samples is None else _dev_tensor(samples, torch.int64, (1,), "samples")
    return r


def mfa_server_create(ctx: int, streams: int = 0, max_batch: int = 0, max_bytes: int = 0) -> int:
    cfg = ServerConfig(int(streams), int(max_batch), int(max_bytes))
    h = C.c_void_p()
    _check(lib.mfa_server_create(ctx, C.byref(cfg), C.byref(h)))
    return h.value


def mfa_server_submit(server: int, model, camera, tf, params, rgba, samples=None) -> int:
    """Queue one request; the tensors must stay alive until it is waited for."""
    keep = []
    r = _request_struct(model, camera, tf, params, rgba, samples, keep)
    t = C.c_int64()
    _check(lib.mfa_server_submit(server, C.byref(r), C.byref(t)))
    return t.value


def mfa_server_wait(server: int, ticket: int, timeout_us: int = -1):
    """Wait for a request; returns its RequestInfo, or None on time-out."""
    info = RequestInfo()
    st = lib.mfa_server_wait(server, int(ticket), int(timeout_us), C.byref(info))
    if st == MFA_ERR_TIMEOUT:
        return None
    _check(st)
    return info


def mfa_server_destroy(server: int) -> None:
    _check(lib.mfa_server_destroy(server))


def mfa_kernel_timing(ctx: int, enable: bool) -> None:
    """Start (True) or stop (False) recording the ray-casting kernel's
    duration on every later mfa_render call; either discards the record."""
    _check(lib.mfa_kernel_timing(ctx, 1 if enable else 0))


def mfa_measure_fma_peak(ctx: int) -> float:
    """Measured FP32 FMA rate of the device (TFLOP/s), synchronous."""
    out = C.c_double()
    _check(lib.mfa_measure_fma_peak(ctx, C.byref(out)))
    return out.value


def mfa_kernel_times(ctx: int, cap: int = 1 << 16):
    """Durations (ms, float32 numpy array, in call order) of the recorded
    render kernels; waits for them and clears the record."""
    import numpy as np
    buf = np.zeros(max(int(cap), 0), dtype=np.float32)
    n = C.c_int64()
    _check(lib.mfa_kernel_times(ctx, buf.ctypes.data if cap > 0 else None, int(cap),
                                C.byref(n)))
    return buf[:min(n.value, int(cap))].copy()


def mfa_eval_points(ctx: int, model: int, xyz, value, grad=None, stream=None) -> None:
    """Value (n,) and world gradient (n, 3) float32 at world points xyz (n, 3) float64."""
    import torch
    n = int(xyz.shape[0])
    px = _dev_tensor(xyz, torch.float64, (n, 3), "xyz")
    pv = _dev_tensor(value, torch.float32, (n,), "value")
    pg = None if grad is None else _dev_tensor(grad, torch.float32, (n, 3), "grad")
    _check(lib.mfa_eval_points(ctx, int(model), n, px, pv, pg, _stream_ptr(stream)))


def mfa_eval_hessian(ctx: int, model: int, xyz, value, hess, grad=None, stream=None) -> None:
    """Value (n,), world Hessian (n, 6: xx yy zz xy xz yz) and optionally the
    world gradient (n, 3), float32, at world points xyz (n, 3) float64."""
    import torch
    n = int(xyz.shape[0])
    px = _dev_tensor(xyz, torch.float64, (n, 3), "xyz")
    pv = _dev_tensor(value, torch.float32, (n,), "value")
    ph = _dev_tensor(hess, torch.float32, (n, 6), "hess")
    pg = None if grad is None else _dev_tensor(grad, torch.float32, (n, 3), "grad")
    _check(lib.mfa_eval_hessian(ctx, int(model), n, px, pv, pg, ph, _stream_ptr(stream)))
