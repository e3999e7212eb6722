"""Python binding of the C ABI in include/nis.h (``libnis.so``).

Every function of the ABI is exposed under its own name (``nis_create``,
``nis_load_medium``, ...) with ctypes marshalling only; all computation runs
in the library's HIP kernels.  ``Context`` wraps the calls with numpy host
arrays and torch device tensors.  torch is used for device memory and streams
only; it is imported before the library is loaded so that both use the same
HIP runtime instance.

The library must have been built (``paper_2401_14051_amd.build.build()``);
importing this module raises if ``libnis.so`` is missing -- there is no
fallback implementation.
"""

import ctypes
import os
import struct

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnis.so")

NIS_OK = 0
NIS_E_INVALID = -1
NIS_E_STATE = -2
NIS_E_NOMEM = -3
NIS_E_DEVICE = -4
NIS_E_UNSUPPORTED = -5
NIS_E_INTERNAL = -6
NIS_FP32, NIS_BF16, NIS_FP8 = 0, 1, 2
NIS_EAGER = 1
NOALLOC_MAX_POINTS = 8192   # NIS_NOALLOC_MAX_POINTS
NIS_TEMPLATES_LATTICE, NIS_TEMPLATES_PAPER = 0, 1
NIS_BACKBONE_MLP, NIS_BACKBONE_PAPER = 0, 1
MODULE_FLOATS = 56706      # floats of the backbone-module block of the weight blob
TPL_SITES = 266
NIS_QUEUED, NIS_RUNNING = 1, 2
LAYERS, SITES, STATS, DESCRIPTOR = 12, 225, 8, 1057
PRECISIONS = {"fp32": NIS_FP32, "bf16": NIS_BF16, "fp8": NIS_FP8}

_fp = ctypes.POINTER(ctypes.c_float)
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64

class nis_camera(ctypes.Structure):
    _fields_ = [("eye", ctypes.c_double * 3), ("target", ctypes.c_double * 3),
                ("up", ctypes.c_double * 3), ("vfov_deg", ctypes.c_double),
                ("ortho_z", ctypes.c_double), ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class nis_server_cfg(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("precision", ctypes.c_int32),
                ("max_inflight", ctypes.c_int32), ("batch_gather", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class nis_frame_req(ctypes.Structure):
    _fields_ = [("medium", ctypes.c_int32), ("camera", nis_camera),
                ("light_dir", ctypes.c_float * 3), ("radiance", ctypes.c_float),
                ("g", ctypes.c_float), ("seed", ctypes.c_uint64)]


class nis_frame_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("channels", ctypes.c_int32), ("n_points", ctypes.c_int64), ("d_image", ctypes.c_void_p),
                ("t_submit", ctypes.c_double), ("t_start", ctypes.c_double),
                ("t_done", ctypes.c_double)]


class nis_query_item(ctypes.Structure):
    _fields_ = [("medium", ctypes.c_int32), ("reserved", ctypes.c_int32), ("d_points", ctypes.c_void_p),
                ("d_view_dirs", ctypes.c_void_p), ("n", ctypes.c_int64), ("d_radiance_out", ctypes.c_void_p)]


_u64 = ctypes.c_uint64

_SIGNATURES = {
    "nis_create": [_i32, ctypes.POINTER(_vp)],
    "nis_destroy": [_vp],
    "nis_load_medium": [_vp, _vp, _i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                        ctypes.POINTER(_i32)],
    "nis_rebuild_pyramid": [_vp, _i32, _vp],
    "nis_set_medium_params": [_vp, _i32, ctypes.c_float, ctypes.c_float, ctypes.c_float],
    "nis_unload_medium": [_vp, _i32],
    "nis_set_light": [_vp, _i32, _vp, ctypes.c_float, _i32],
    "nis_light_footprint": [_i32, _vp, ctypes.POINTER(_i64), _vp],
    "nis_set_phase_lobes": [_vp, _i32, _i32, _vp, _vp],
    "nis_set_volume_phase": [_vp, _i32, _i32],
    "nis_set_albedo_rgb": [_vp, _i32, _vp],
    "nis_set_weights": [_vp, _vp, ctypes.c_size_t],
    "nis_set_precision": [_vp, _i32],
    "nis_query": [_vp, _i32, _vp, _vp, _i64, _vp],
    "nis_query_device": [_vp, _i32, _vp, _vp, _i64, _vp, _vp],
    "nis_query_device_noalloc": [_vp, _i32, _vp, _vp, _i64, _vp, _vp],
    "nis_query_batch": [_vp, _vp, _i32, _vp],
    "nis_calibrate_fp8": [_vp, _i32, _vp, _vp, _i64, _vp],
    "nis_set_templates": [_vp, _i32],
    "nis_set_backbone": [_vp, _i32],
    "nis_debug_template_features": [_vp, _i32, _vp, _vp, _i64, _vp, _vp, _vp, _vp, _vp],
    "nis_query_rgb": [_vp, _i32, _vp, _vp, _i64, _vp],
    "nis_query_rgb_device": [_vp, _i32, _vp, _vp, _i64, _vp, _vp],
    "nis_medium_info": [_vp, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i64)],
    "nis_debug_pyramid": [_vp, _i32, _vp, _i64],
    "nis_debug_path_density": [_vp, _i32, _i32, _vp, _i64, ctypes.POINTER(_i32)],
    "nis_debug_path_pairs": [_vp, _i32, _i32, _vp, _i64],
    "nis_debug_features": [_vp, _i32, _vp, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp],
    "nis_debug_network": [_vp, _i32, _vp, _vp, _i64, _vp, _vp],
    "nis_frame_points": [_vp, _i32, ctypes.POINTER(nis_camera), _u64, _vp, _vp, _vp, _vp, _vp],
    "nis_render": [_vp, _i32, ctypes.POINTER(nis_camera), _u64, _vp, _vp],
    "nis_render_rgb": [_vp, _i32, ctypes.POINTER(nis_camera), _u64, _vp, _vp],
    "nis_server_start": [_vp, ctypes.POINTER(nis_server_cfg)],
    "nis_submit_frame": [_vp, ctypes.POINTER(nis_frame_req), ctypes.POINTER(_u64)],
    "nis_poll": [_vp, _u64, ctypes.POINTER(nis_frame_result)],
    "nis_wait": [_vp, _u64, ctypes.POINTER(nis_frame_result)],
    "nis_release": [_vp, _u64],
    "nis_frame_memory": [_vp, ctypes.POINTER(nis_frame_req), _i32, ctypes.POINTER(_u64)],
    "nis_server_stop": [_vp],
    "nis_profile": [_vp, _i32],
    "nis_profile_report": [_vp, _vp, ctypes.c_size_t],
}

EXPORTS = tuple(_SIGNATURES) + ("nis_last_error",)


class NisError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("nis error %d: %s" % (code, msg))
        self.code = code


def _load():
    try:
        import torch  # noqa: F401  (the HIP runtime torch loaded is the one the library binds to)
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError("libnis.so is not built (run paper_2401_14051_amd.build.build())")
    lib = ctypes.CDLL(LIB_PATH)
    for name, args in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = _i32
    lib.nis_last_error.argtypes = []
    lib.nis_last_error.restype = ctypes.c_char_p
    return lib


_lib = _load()


def nis_last_error():
    return _lib.nis_last_error().decode()


def _check(code):
    if code != NIS_OK:
        raise NisError(code, nis_last_error())
    return code


def _wrap(name):
    fn = getattr(_lib, name)

    def call(*args):
        return fn(*args)
    call.__name__ = name
    call.__doc__ = "Raw ABI call %s (returns the int32 status)." % name
    return call


for _n in _SIGNATURES:
    globals()[_n] = _wrap(_n)


# ---------------------------------------------------------------------------
# weight blob

_GROUP_ORDER = ("w1", "b1", "w2", "b2", "s1", "c1", "s2", "c2")


def pack_weights(params, fp8_scales=None, modules=None):
    """Serialise a parameter dict (see ``workloads.weights``) into the blob
    layout documented at nis_set_weights; ``modules`` is the list of arrays
    of the backbone modules (``workloads.weights.he_init_modules``)."""
    width, n_linear = int(params["width"]), int(params["n_linear"])
    has_fp8 = fp8_scales is not None
    mod = None
    if modules is not None:
        mod = np.concatenate([np.asarray(a, np.float32).ravel() for a in modules])
        if mod.size != MODULE_FLOATS:
            raise ValueError("the module block holds %d floats, not %d" % (mod.size, MODULE_FLOATS))
    header = struct.pack("<4s5I2f2I6I", b"NISW", 1, DESCRIPTOR, width, n_linear, 2,
                         float(params["lam"]), float(params["gamma"]), 1 if has_fp8 else 0,
                         0 if mod is None else 1, *([0] * 6))
    parts = []
    for g in ("diffuse", "highlight"):
        for k in _GROUP_ORDER:
            parts.append(np.asarray(params["groups"][g][k], np.float32).ravel())
    for A, b in zip(params["A"], params["beta"]):
        parts.append(np.asarray(A, np.float32).ravel())
        parts.append(np.asarray(b, np.float32).ravel())
    if has_fp8:
        parts.append(np.asarray(fp8_scales, np.float32).ravel())
    if mod is not None:
        parts.append(mod)
    return header + np.concatenate(parts).astype("<f4").tobytes()


# ---------------------------------------------------------------------------
# convenience wrapper

def camera(width, height, vfov_deg=45.0, eye=(0.5, 0.5, 2.0), target=(0.5, 0.5, 0.5),
           up=(0.0, 1.0, 0.0), ortho_z=1.0):
    """An ``nis_camera``; vfov_deg=0 gives the orthographic camera."""
    c = nis_camera()
    c.eye[:] = [float(v) for v in eye]
    c.target[:] = [float(v) for v in target]
    c.up[:] = [float(v) for v in up]
    c.vfov_deg = float(vfov_deg)
    c.ortho_z = float(ortho_z)
    c.width, c.height = int(width), int(height)
    return c


def light_footprint(n, direction):
    """Device bytes of one light's state for an n^3 medium: {"total": bytes,
    "levels": path-density pair bytes of each level}.  Host-only."""
    d = np.ascontiguousarray(direction, np.float32)
    total = _i64()
    levels = np.zeros(11, np.int64)
    _check(_lib.nis_light_footprint(int(n), _ptr(d), ctypes.byref(total), _ptr(levels)))
    L = int(n).bit_length()
    return {"total": total.value, "levels": [int(v) for v in levels[:L]]}


def _memcpy_d2d(dst, src, nbytes):
    """Device-to-device copy through the HIP runtime the library links
    (dlsym on the library's handle also searches its dependencies)."""
    fn = _lib.hipMemcpy
    fn.argtypes = [_vp, _vp, ctypes.c_size_t, ctypes.c_int]
    fn.restype = ctypes.c_int
    rc = fn(_vp(dst), _vp(src), nbytes, 3)     # hipMemcpyDeviceToDevice
    if rc != 0:
        raise NisError(NIS_E_DEVICE, "hipMemcpy failed with HIP error %d" % rc)


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if isinstance(a, np.ndarray) else ctypes.c_void_p(a)


def _dptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Context:
    """One library context on a HIP device."""

    def __init__(self, device=0):
        h = ctypes.c_void_p()
        _check(_lib.nis_create(device, ctypes.byref(h)))
        self.h = h
        self.device = device

    def close(self):
        # at interpreter exit the module's globals may already be cleared
        if getattr(self, "h", None) and _lib is not None:
            _lib.nis_destroy(self.h)
            self.h = None

    __del__ = close

    def load_medium(self, density, sigma_t, albedo, g):
        d = np.ascontiguousarray(density, dtype=np.float32)
        n = d.shape[0]
        if d.shape != (n, n, n):
            raise ValueError("density must be n^3")
        mid = _i32()
        _check(_lib.nis_load_medium(self.h, _ptr(d), n, sigma_t, albedo, g, ctypes.byref(mid)))
        return mid.value

    def rebuild_pyramid(self, medium, stream=None):
        _check(_lib.nis_rebuild_pyramid(self.h, medium, _vp(stream)))

    def set_medium_params(self, medium, sigma_t, albedo, g):
        _check(_lib.nis_set_medium_params(self.h, medium, sigma_t, albedo, g))

    def unload_medium(self, medium):
        _check(_lib.nis_unload_medium(self.h, medium))

    def set_phase_lobes(self, medium, lobes):
        """Multi-lobe HG phase (eq. 6) from a sequence of (weight, g) pairs."""
        w = np.ascontiguousarray([float(a) for a, _ in lobes], np.float32)
        g = np.ascontiguousarray([float(b) for _, b in lobes], np.float32)
        _check(_lib.nis_set_phase_lobes(self.h, medium, len(w), _ptr(w), _ptr(g)))

    def set_volume_phase(self, medium, enable=True):
        """Volume phases (eq. 9) in the phase features, or point phases."""
        _check(_lib.nis_set_volume_phase(self.h, medium, 1 if enable else 0))

    def set_albedo_rgb(self, medium, albedo_rgb):
        """One albedo per colour channel (red, green, blue), each in [0,1]."""
        a = np.ascontiguousarray(albedo_rgb, dtype=np.float32).reshape(3)
        _check(_lib.nis_set_albedo_rgb(self.h, medium, _ptr(a)))

    def set_light(self, medium, direction, radiance=1.0, eager=False):
        d = np.ascontiguousarray(direction, dtype=np.float32)
        _check(_lib.nis_set_light(self.h, medium, _ptr(d), radiance, NIS_EAGER if eager else 0))

    def set_weights(self, params=None, blob=None, fp8_scales=None, modules=None):
        if blob is None:
            blob = pack_weights(params, fp8_scales, modules)
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(_lib.nis_set_weights(self.h, buf, len(blob)))

    def set_precision(self, precision):
        if isinstance(precision, str):
            precision = PRECISIONS[precision]
        _check(_lib.nis_set_precision(self.h, precision))

    def query(self, medium, points, dirs):
        """Host arrays in, host radiance out (synchronous)."""
        p = np.ascontiguousarray(points, dtype=np.float32)
        d = np.ascontiguousarray(dirs, dtype=np.float32)
        out = np.empty(p.shape[0], np.float32)
        _check(_lib.nis_query(self.h, medium, _ptr(p), _ptr(d), p.shape[0], _ptr(out)))
        return out

    def query_device(self, medium, points, dirs, out, stream=None):
        """torch device tensors in/out, queued on ``stream`` (a HIP stream
        handle; None = the current torch stream)."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(points.device).cuda_stream
        _check(_lib.nis_query_device(self.h, medium, _dptr(points), _dptr(dirs), points.shape[0],
                                     _dptr(out), _vp(stream)))

    def query_batch(self, queries, stream=None):
        """Several device queries in one launch: ``queries`` is a list of
        (medium, points, dirs, out) with torch device tensors; queued on
        ``stream`` (None = the current torch stream)."""
        import torch
        items = (nis_query_item * len(queries))()
        for it, (medium, points, dirs, out) in zip(items, queries):
            it.medium = medium
            it.reserved = 0
            it.d_points = points.data_ptr()
            it.d_view_dirs = dirs.data_ptr()
            it.n = points.shape[0]
            it.d_radiance_out = out.data_ptr()
        if stream is None:
            dev = queries[0][1].device if queries else torch.device("cuda", self.device)
            stream = torch.cuda.current_stream(dev).cuda_stream
        _check(_lib.nis_query_batch(self.h, items, len(queries), _vp(stream)))

    def calibrate_fp8(self, medium, points, dirs, stream=None):
        """Static FP8 activation scales from the FP32 path over these points
        (torch device tensors [n, 3]); synchronous."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(points.device).cuda_stream
        _check(_lib.nis_calibrate_fp8(self.h, medium, _dptr(points), _dptr(dirs), points.shape[0], _vp(stream)))

    def query_device_noalloc(self, medium, points, dirs, out, stream=None):
        """As query_device through the entry point that allocates nothing (its
        scratch is the library's fixed per-GPU array; at most
        NOALLOC_MAX_POINTS points)."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(points.device).cuda_stream
        _check(_lib.nis_query_device_noalloc(self.h, medium, _dptr(points), _dptr(dirs), points.shape[0],
                                             _dptr(out), _vp(stream)))

    def query_rgb(self, medium, points, dirs):
        """As query, one radiance per colour channel: host [n, 3]."""
        p = np.ascontiguousarray(points, dtype=np.float32)
        d = np.ascontiguousarray(dirs, dtype=np.float32)
        out = np.empty((p.shape[0], 3), np.float32)
        _check(_lib.nis_query_rgb(self.h, medium, _ptr(p), _ptr(d), p.shape[0], _ptr(out)))
        return out

    def query_rgb_device(self, medium, points, dirs, out, stream=None):
        """As query_device with ``out`` a device tensor [n, 3]."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(points.device).cuda_stream
        _check(_lib.nis_query_rgb_device(self.h, medium, _dptr(points), _dptr(dirs), points.shape[0],
                                         _dptr(out), _vp(stream)))

    def frame_points(self, medium, cam, seed, stream=None):
        """Collisions of a frame as torch device tensors (points [P,3], dirs [P,3],
        pixel [P]); synchronises ``stream`` to read P."""
        import torch
        dev = torch.device("cuda", self.device)
        npix = cam.width * cam.height
        pts = torch.empty(npix, 3, dtype=torch.float32, device=dev)
        dirs = torch.empty(npix, 3, dtype=torch.float32, device=dev)
        pix = torch.empty(npix, dtype=torch.int32, device=dev)
        cnt = torch.zeros(1, dtype=torch.int32, device=dev)
        if stream is None:
            stream = torch.cuda.current_stream(dev).cuda_stream
        _check(_lib.nis_frame_points(self.h, medium, ctypes.byref(cam), seed, _dptr(pts),
                                     _dptr(dirs), _dptr(pix), _dptr(cnt), _vp(stream)))
        n = int(cnt.item())
        return pts[:n], dirs[:n], pix[:n]

    def render(self, medium, cam, seed, out=None, stream=None):
        """A frame image (torch float32 [height, width]) queued on ``stream``."""
        import torch
        dev = torch.device("cuda", self.device)
        if out is None:
            out = torch.empty(cam.height, cam.width, dtype=torch.float32, device=dev)
        if stream is None:
            stream = torch.cuda.current_stream(dev).cuda_stream
        _check(_lib.nis_render(self.h, medium, ctypes.byref(cam), seed, _dptr(out), _vp(stream)))
        return out

    def render_rgb(self, medium, cam, seed, out=None, stream=None):
        """An RGB frame image (torch float32 [height, width, 3]) queued on ``stream``."""
        import torch
        dev = torch.device("cuda", self.device)
        if out is None:
            out = torch.empty(cam.height, cam.width, 3, dtype=torch.float32, device=dev)
        if stream is None:
            stream = torch.cuda.current_stream(dev).cuda_stream
        _check(_lib.nis_render_rgb(self.h, medium, ctypes.byref(cam), seed, _dptr(out), _vp(stream)))
        return out

    # -- frame server --

    def server_start(self, budget_bytes, precision="bf16", max_inflight=4, batch_gather=False):
        cfg = nis_server_cfg(int(budget_bytes), PRECISIONS.get(precision, precision), int(max_inflight),
                             1 if batch_gather else 0, 0)
        _check(_lib.nis_server_start(self.h, ctypes.byref(cfg)))

    @staticmethod
    def frame_request(medium, cam, light_dir, radiance=1.0, g=0.85, seed=0):
        req = nis_frame_req()
        req.medium = medium
        req.camera = cam
        req.light_dir[:] = [float(v) for v in light_dir]
        req.radiance = float(radiance)
        req.g = float(g)
        req.seed = int(seed)
        return req

    def frame_memory(self, medium, cam, light_dir, precision="bf16"):
        req = self.frame_request(medium, cam, light_dir)
        b = _u64()
        _check(_lib.nis_frame_memory(self.h, ctypes.byref(req), PRECISIONS.get(precision, precision),
                                     ctypes.byref(b)))
        return b.value

    def submit(self, medium, cam, light_dir, radiance=1.0, g=0.85, seed=0):
        req = self.frame_request(medium, cam, light_dir, radiance, g, seed)
        fid = _u64()
        _check(_lib.nis_submit_frame(self.h, ctypes.byref(req), ctypes.byref(fid)))
        return fid.value

    def poll(self, fid):
        r = nis_frame_result()
        _check(_lib.nis_poll(self.h, fid, ctypes.byref(r)))
        return r

    def wait(self, fid):
        r = nis_frame_result()
        _check(_lib.nis_wait(self.h, fid, ctypes.byref(r)))
        return r

    def frame_image(self, result):
        """Copy of a finished frame's image as a torch tensor ([height, width],
        or [height, width, 3] for a medium with a coloured albedo)."""
        import torch
        n = result.width * result.height * result.channels
        shape = (result.height, result.width) + ((3,) if result.channels == 3 else ())
        out = torch.empty(*shape, dtype=torch.float32, device=torch.device("cuda", self.device))
        if n:
            torch.cuda.synchronize(out.device)
            _memcpy_d2d(out.data_ptr(), result.d_image, n * 4)
        return out

    def release(self, fid):
        _check(_lib.nis_release(self.h, fid))

    def server_stop(self):
        _check(_lib.nis_server_stop(self.h))

    def profile(self, enable=True):
        _check(_lib.nis_profile(self.h, 1 if enable else 0))

    def profile_report(self):
        """{kernel: (launches, total_ms)} for the kernels recorded since profile()."""
        buf = ctypes.create_string_buffer(1 << 16)
        _check(_lib.nis_profile_report(self.h, buf, len(buf)))
        out = {}
        for line in buf.value.decode().splitlines():
            name, cnt, ms = line.split()
            out[name] = (int(cnt), float(ms))
        return out

    def medium_info(self, medium):
        lv, nf = _i32(), _i64()
        _check(_lib.nis_medium_info(self.h, medium, ctypes.byref(lv), ctypes.byref(nf)))
        return lv.value, nf.value

    def pyramid(self, medium):
        levels, nf = self.medium_info(medium)
        out = np.empty(nf, np.float32)
        _check(_lib.nis_debug_pyramid(self.h, medium, _ptr(out), nf))
        res, off = [], 0
        n0 = 1 << (levels - 1)          # edges halve from n0 down to 1
        for m in range(levels):
            nm = n0 >> m
            res.append(out[off:off + nm ** 3].reshape(nm, nm, nm))
            off += nm ** 3
        return res

    def path_density(self, medium, level):
        dims = (_i32 * 5)()
        _check(_lib.nis_debug_path_density(self.h, medium, level, None, 0, dims))
        nu, nv, nj = dims[1] - dims[0] + 1, dims[3] - dims[2] + 1, dims[4]
        out = np.empty(nu * nv * nj, np.float32)
        _check(_lib.nis_debug_path_density(self.h, medium, level, _ptr(out), out.size, dims))
        return out.reshape(nj, nv, nu), (dims[0], dims[1], dims[2], dims[3])

    def path_pairs(self, medium, level):
        """Path-density pairs of one level as [J][V' = 0..n_V][U][2]."""
        dims = (_i32 * 5)()
        _check(_lib.nis_debug_path_density(self.h, medium, level, None, 0, dims))
        nu, nv, nj = dims[1] - dims[0] + 1, dims[3] - dims[2] + 1, dims[4]
        out = np.empty(2 * nu * (nv + 1) * nj, np.float32)
        _check(_lib.nis_debug_path_pairs(self.h, medium, level, _ptr(out), out.size))
        return out.reshape(nj, nv + 1, nu, 2)

    def features(self, medium, points, dirs):
        """Gather-stage outputs for torch device tensors (returns torch tensors)."""
        import torch
        n = points.shape[0]
        dev = points.device
        z = lambda *s: torch.zeros(*s, dtype=torch.float32, device=dev)
        out = {"tbar": z(n, LAYERS, SITES), "rho": z(n, LAYERS, SITES), "phi": z(n, SITES),
               "stats": z(n, LAYERS, STATS), "tp": z(n), "f0": z(n)}
        _check(_lib.nis_debug_features(self.h, medium, _dptr(points), _dptr(dirs), n,
                                       *[_dptr(out[k]) for k in ("tbar", "rho", "phi", "stats",
                                                                 "tp", "f0")]))
        return out

    def set_templates(self, kind):
        """"lattice" (default) or "paper" (the sphere and cone templates)."""
        if isinstance(kind, str):
            kind = {"lattice": NIS_TEMPLATES_LATTICE, "paper": NIS_TEMPLATES_PAPER}[kind]
        _check(_lib.nis_set_templates(self.h, kind))

    def set_backbone(self, kind):
        """"mlp" (default) or "paper" (the layer-by-layer modules before the
        MLP; needs the paper's templates and weights with the module block)."""
        if isinstance(kind, str):
            kind = {"mlp": NIS_BACKBONE_MLP, "paper": NIS_BACKBONE_PAPER}[kind]
        _check(_lib.nis_set_backbone(self.h, kind))

    def template_features(self, medium, points, dirs):
        """Gather-stage outputs at the paper's templates (torch tensors)."""
        import torch
        n = points.shape[0]
        z = lambda *s: torch.zeros(*s, dtype=torch.float32, device=points.device)
        out = {"tbar": z(n, TPL_SITES), "rho": z(n, TPL_SITES), "phi": z(n, TPL_SITES),
               "stats": z(n, LAYERS, STATS), "f0": z(n)}
        _check(_lib.nis_debug_template_features(self.h, medium, _dptr(points), _dptr(dirs), n,
                                                *[_dptr(out[k]) for k in ("tbar", "rho", "phi", "stats", "f0")]))
        return out

    def network(self, medium, points, dirs, want_desc=True):
        import torch
        n = points.shape[0]
        desc = torch.zeros(n, DESCRIPTOR, dtype=torch.float32, device=points.device) if want_desc else None
        y = torch.zeros(n, dtype=torch.float32, device=points.device)
        _check(_lib.nis_debug_network(self.h, medium, _dptr(points), _dptr(dirs), n, _dptr(desc),
                                      _dptr(y)))
        return desc, y
