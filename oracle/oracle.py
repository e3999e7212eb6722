"""ctypes wrapper of the FP64 CPU oracle (``nis_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
benchmark's CPU-baseline leg.  The HIP library never uses it.

``build()`` compiles ``liboracle.so`` next to this file with gcc
(-O2 -fno-fast-math -ffp-contract=off -fopenmp).  Parameters are the dicts
produced by ``workloads.weights``; they are flattened here into the oracle's
own FP64 layout.
"""

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "nis_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

LAYERS, SITES, STATS, FEAT, DESC = 12, 225, 8, 80, 1057
GROUP_ORDER = ("w1", "b1", "w2", "b2", "s1", "c1", "s2", "c2")

_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force=False):
    """Compile the oracle shared library (always when ``force``)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-fno-fast-math", "-ffp-contract=off",
                               "-fopenmp", "-fPIC", "-shared", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        L.om_create.restype = ctypes.c_void_p
        L.om_create.argtypes = [_fp, ctypes.c_int]
        L.om_free.argtypes = [ctypes.c_void_p]
        L.om_levels.argtypes = [ctypes.c_void_p]
        L.om_level_offset.restype = ctypes.c_int64
        L.om_level_offset.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.om_pyramid.restype = _dp
        L.om_pyramid.argtypes = [ctypes.c_void_p]
        L.om_set_light.argtypes = [ctypes.c_void_p, _fp]
        L.om_light_frame.argtypes = [ctypes.c_void_p, _ip, _dp, _dp]
        L.om_path_density.restype = _dp
        L.om_path_density.argtypes = [ctypes.c_void_p, ctypes.c_int, _ip]
        L.om_sample_rho.restype = ctypes.c_double
        L.om_sample_rho.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp]
        L.om_sample_D.restype = ctypes.c_double
        L.om_sample_D.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp]
        L.om_hg.restype = ctypes.c_double
        L.om_hg.argtypes = [ctypes.c_double, ctypes.c_double]
        L.om_mhg.restype = ctypes.c_double
        L.om_mhg.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_double]
        L.om_hg_cone.restype = ctypes.c_double
        L.om_hg_cone.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.om_volume_init.argtypes = []
        L.om_set_threads.argtypes = [ctypes.c_int]
        L.om_get_threads.restype = ctypes.c_int
        L.om_get_threads.argtypes = []
        L.om_features.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_int, _dp, _dp, ctypes.c_int,
                                  ctypes.c_double,
                                  _fp, _fp, ctypes.c_int64, _dp, _dp, _dp, _dp, _dp, _dp]
        L.om_cnn_se.argtypes = [_dp, _dp, _dp]
        L.om_descriptor.argtypes = [_dp, _dp, _dp, ctypes.c_double, _dp]
        L.om_mlp.restype = ctypes.c_double
        L.om_mlp.argtypes = [_dp, ctypes.c_int, ctypes.c_int, _dp]
        L.om_query.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_int, _dp, _dp,
                               ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp, ctypes.c_int,
                               ctypes.c_int, _fp, _fp, ctypes.c_int64, _dp, _dp, _dp, _dp]
        L.om_tpl_count_of.restype = ctypes.c_int
        L.om_tpl_count_of.argtypes = [ctypes.c_int]
        L.om_tpl_unit.argtypes = [ctypes.c_int, ctypes.c_int, _dp]
        L.om_tpl_D.restype = ctypes.c_double
        L.om_tpl_D.argtypes = [ctypes.c_int]
        L.om_tpl_radius.restype = ctypes.c_double
        L.om_tpl_radius.argtypes = [ctypes.c_int]
        L.om_tpl_light_extent.restype = ctypes.c_double
        L.om_tpl_light_extent.argtypes = [_dp, _dp]
        L.om_tpl_features.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_int, _dp, _dp, ctypes.c_double,
                                      _fp, _fp, ctypes.c_int64, _dp, _dp, _dp, _dp, _dp]
        L.om_tpl_descriptor.argtypes = [_dp, _dp, _dp, _dp, ctypes.c_double, _dp]
        L.om_tpl_query.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_int, _dp, _dp,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp, ctypes.c_int,
                                   ctypes.c_int, _fp, _fp, ctypes.c_int64, _dp, _dp, _dp, _dp]
        L.om_modules_size.restype = ctypes.c_int64
        L.om_modules_size.argtypes = []
        L.om_modules.argtypes = [_dp, _dp, ctypes.c_double, _dp]
        L.om_tpl_modules_query.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_int, _dp,
                                           _dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp,
                                           ctypes.c_int, ctypes.c_int, _dp, _fp, _fp, ctypes.c_int64, _dp, _dp, _dp]
        _lib = L
    return _lib


def flatten_modules(modules):
    """The oracle's FP64 block of the modules' weights (workloads.weights.he_init_modules order)."""
    flat = np.concatenate([np.asarray(a, np.float64).ravel() for a in modules])
    if flat.size != lib().om_modules_size():
        raise ValueError("module block has %d values, expected %d" % (flat.size, lib().om_modules_size()))
    return flat


def modules(mods, feat, albedo):
    """The paper's backbone modules: template features (894, descriptor
    layout) -> the modules' descriptor (1057)."""
    out = np.zeros(DESC)
    f = np.zeros(DESC)
    f[:len(feat)] = feat
    lib().om_modules(_ptr(flatten_modules(mods), _dp), _ptr(f, _dp), float(albedo), _ptr(out, _dp))
    return out


# ---- the paper's templates (Sec. III.B.2, eq. 2-4) ----
TPL_SITES = 266


def tpl_counts():
    """Points per template layer: 8 diffuse sphere layers, 4 highlight cone layers."""
    return [lib().om_tpl_count_of(k) for k in range(LAYERS)]


def tpl_unit(layer):
    """Unit template points of a layer as an [n, 3] array (diffuse: world axes;
    highlight: (t along l, x1, x2) in the frame of l)."""
    n = lib().om_tpl_count_of(layer)
    out = np.zeros((n, 3))
    u = np.zeros(3)
    for k in range(n):
        lib().om_tpl_unit(layer, k, _ptr(u, _dp))
        out[k] = u
    return out


def tpl_D(layer):
    """eq. (3): mean nearest-neighbour distance of the layer's unit points."""
    return lib().om_tpl_D(layer)


def tpl_radius(layer):
    """eq. (4): radius of diffuse layer i in unit-cube lengths."""
    return lib().om_tpl_radius(layer)


def tpl_light_extent(l, x):
    """Distance from x towards the light to where that ray leaves the unit cube."""
    return lib().om_tpl_light_extent(_ptr(_f64(l), _dp), _ptr(_f64(x), _dp))


def set_threads(n):
    """Threads of the oracle's OpenMP loops from now on."""
    lib().om_set_threads(int(n))


def get_threads():
    return lib().om_get_threads()


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, t):
    return None if a is None else a.ctypes.data_as(t)


def hg(g, mu):
    """Henyey-Greenstein phase value (eq. 5)."""
    return lib().om_hg(float(g), float(mu))


def lobes(phase):
    """(weights, asymmetries) as float64 arrays of a phase given either as one
    asymmetry g (plain HG, eq. 5) or as a sequence of (weight, g) lobes (eq. 6)."""
    if np.ndim(phase) == 0:
        return np.array([1.0]), np.array([float(phase)])
    lw = np.array([float(w) for w, _ in phase])
    lg = np.array([float(g) for _, g in phase])
    return lw, lg


def hg_cone(g, mu0, beta):
    """Volume phase of one HG lobe (eq. 9): its mean over a cone of half-angle
    beta around a direction d, for mu0 = w . d."""
    lib().om_volume_init()
    return lib().om_hg_cone(float(g), float(mu0), float(beta))


def mhg(phase, mu):
    """Multi-lobe HG phase value (eq. 6) of a phase as accepted by lobes()."""
    lw, lg = lobes(phase)
    return lib().om_mhg(len(lw), _ptr(lw, _dp), _ptr(lg, _dp), float(mu))


def flatten_params(params):
    """The oracle's own flat FP64 layout of a ``workloads.weights`` dict."""
    parts = []
    for name in ("diffuse", "highlight"):
        for key in GROUP_ORDER:
            parts.append(np.asarray(params["groups"][name][key], np.float64).ravel())
    for A, b in zip(params["A"], params["beta"]):
        parts.append(np.asarray(A, np.float64).ravel())
        parts.append(np.asarray(b, np.float64).ravel())
    return np.concatenate(parts)


def group_block(params, name):
    return np.concatenate([np.asarray(params["groups"][name][k], np.float64).ravel()
                           for k in GROUP_ORDER])


def cnn_se(params, group, lattice):
    """80 attention-weighted CNN features of one 9x5x5 lattice."""
    out = np.zeros(FEAT)
    blk = group_block(params, group)
    lib().om_cnn_se(_ptr(blk, _dp), _ptr(_f64(lattice).ravel(), _dp), _ptr(out, _dp))
    return out


def descriptor(params, tbar, stats, albedo):
    """1057-entry descriptor from per-layer lattices [12][225] and stats [12][8]."""
    flat = flatten_params(params)
    out = np.zeros(DESC)
    lib().om_descriptor(_ptr(flat, _dp), _ptr(_f64(tbar).ravel(), _dp),
                        _ptr(_f64(stats).ravel(), _dp), float(albedo), _ptr(out, _dp))
    return out


def mlp(params, desc):
    flat = flatten_params(params)
    return lib().om_mlp(_ptr(flat, _dp), int(params["width"]), int(params["n_linear"]),
                        _ptr(_f64(desc), _dp))


class Medium:
    """A density grid with its FP64 pyramid and, after ``set_light``, its
    FP64 path-density fields."""

    def __init__(self, density):
        density = _f32(density)
        n = density.shape[0]
        if density.shape != (n, n, n):
            raise ValueError("density must be n^3")
        self._keep = density
        self.h = lib().om_create(_ptr(density, _fp), n)
        if not self.h:
            raise ValueError("grid edge must be a power of two")
        self.n = n
        self.levels = lib().om_levels(self.h)

    def __del__(self):
        if getattr(self, "h", None):
            lib().om_free(self.h)
            self.h = None

    def level(self, m):
        nm = self.n >> m
        off = lib().om_level_offset(self.h, m)
        base = lib().om_pyramid(self.h)
        arr = np.ctypeslib.as_array(base, shape=(off + nm ** 3,))
        return arr[off:off + nm ** 3].reshape(nm, nm, nm).copy()

    def set_light(self, direction):
        d = _f32(direction)
        if lib().om_set_light(self.h, _ptr(d, _fp)) != 0:
            raise ValueError("light direction must be finite and non-zero")

    def light_frame(self):
        fr = (ctypes.c_int * 4)()
        sh = (ctypes.c_double * 2)()
        ll = (ctypes.c_double * 3)()
        lib().om_light_frame(self.h, fr, sh, ll)
        return {"a": fr[0], "b": fr[1], "c": fr[2], "sigma": fr[3],
                "sb": sh[0], "sc": sh[1], "l": np.array(list(ll))}

    def path_density(self, m):
        """(D [nJ][nV][nU] float64, (U_lo, U_hi, V_lo, V_hi))."""
        dims = (ctypes.c_int * 5)()
        p = lib().om_path_density(self.h, m, dims)
        nu, nv, nj = dims[1] - dims[0] + 1, dims[3] - dims[2] + 1, dims[4]
        arr = np.ctypeslib.as_array(p, shape=(nj * nv * nu,)).reshape(nj, nv, nu).copy()
        return arr, (dims[0], dims[1], dims[2], dims[3])

    def sample_rho(self, m, x):
        return lib().om_sample_rho(self.h, m, _ptr(_f64(x), _dp))

    def sample_D(self, m, x):
        return lib().om_sample_D(self.h, m, _ptr(_f64(x), _dp))

    def features(self, sigma_t, g, lam, pts, dirs, volume=False,
                 outputs=("tbar", "rho", "phi", "stats", "tp", "f0")):
        """Per-point features; g is one asymmetry or a sequence of (weight, g)
        lobes; volume selects the volume phase of eq. 9 for the phase features.
        Only the named outputs are kept (the others are computed, not stored)."""
        pts, dirs = _f32(pts), _f32(dirs)
        P = pts.shape[0]
        shapes = {"tbar": (P, LAYERS, SITES), "rho": (P, LAYERS, SITES), "phi": (P, SITES),
                  "stats": (P, LAYERS, STATS), "tp": (P,), "f0": (P,)}
        out = {k: np.zeros(shapes[k]) for k in outputs}
        lw, lg = lobes(g)
        lib().om_features(self.h, float(sigma_t), len(lw), _ptr(lw, _dp), _ptr(lg, _dp), int(bool(volume)),
                          float(lam), _ptr(pts, _fp),
                          _ptr(dirs, _fp), P, *[_ptr(out.get(k), _dp) for k in
                                                ("tbar", "rho", "phi", "stats", "tp", "f0")])
        return out

    def tpl_features(self, sigma_t, g, lam, pts, dirs):
        """Features at the paper's template points: tbar/rho/phi [P][266],
        stats [P][12][8], f0 [P] (point phase; g as in features())."""
        pts, dirs = _f32(pts), _f32(dirs)
        P = pts.shape[0]
        out = {"tbar": np.zeros((P, TPL_SITES)), "rho": np.zeros((P, TPL_SITES)), "phi": np.zeros((P, TPL_SITES)),
               "stats": np.zeros((P, LAYERS, STATS)), "f0": np.zeros(P)}
        lw, lg = lobes(g)
        lib().om_tpl_features(self.h, float(sigma_t), len(lw), _ptr(lw, _dp), _ptr(lg, _dp), float(lam),
                              _ptr(pts, _fp), _ptr(dirs, _fp), P,
                              *[_ptr(out[k], _dp) for k in ("tbar", "rho", "phi", "stats", "f0")])
        return out

    def tpl_query(self, params, pts, dirs, sigma_t, albedo, g, radiance=1.0, want_desc=False):
        """As query() with the paper's templates and their descriptor."""
        pts, dirs = _f32(pts), _f32(dirs)
        P = pts.shape[0]
        flat = flatten_params(params)
        L, y, F = np.zeros(P), np.zeros(P), np.zeros(P)
        desc = np.zeros((P, DESC)) if want_desc else None
        lw, lg = lobes(g)
        lib().om_tpl_query(self.h, float(sigma_t), float(albedo), len(lw), _ptr(lw, _dp), _ptr(lg, _dp),
                           float(params["lam"]), float(params["gamma"]), float(radiance), _ptr(flat, _dp),
                           int(params["width"]), int(params["n_linear"]), _ptr(pts, _fp), _ptr(dirs, _fp), P,
                           _ptr(L, _dp), _ptr(y, _dp), _ptr(F, _dp), _ptr(desc, _dp))
        out = {"L": L, "y": y, "F": F}
        if want_desc:
            out["desc"] = desc
        return out

    def tpl_modules_query(self, params, mods, pts, dirs, sigma_t, albedo, g, radiance=1.0, want_desc=False):
        """The paper's templates and backbone modules, then the MLP and decode."""
        pts, dirs = _f32(pts), _f32(dirs)
        P = pts.shape[0]
        flat = flatten_params(params)
        mp = flatten_modules(mods)
        L, y = np.zeros(P), np.zeros(P)
        desc = np.zeros((P, DESC)) if want_desc else None
        lw, lg = lobes(g)
        lib().om_tpl_modules_query(self.h, float(sigma_t), float(albedo), len(lw), _ptr(lw, _dp), _ptr(lg, _dp),
                                   float(params["lam"]), float(params["gamma"]), float(radiance), _ptr(flat, _dp),
                                   int(params["width"]), int(params["n_linear"]), _ptr(mp, _dp), _ptr(pts, _fp),
                                   _ptr(dirs, _fp), P, _ptr(L, _dp), _ptr(y, _dp), _ptr(desc, _dp))
        out = {"L": L, "y": y}
        if want_desc:
            out["desc"] = desc
        return out

    def query(self, params, pts, dirs, sigma_t, albedo, g, radiance=1.0, want_desc=False, volume=False):
        """Radiance, network output y and decoded F for each point; g is one
        asymmetry or a sequence of (weight, g) lobes."""
        pts, dirs = _f32(pts), _f32(dirs)
        P = pts.shape[0]
        flat = flatten_params(params)
        L, y, F = np.zeros(P), np.zeros(P), np.zeros(P)
        desc = np.zeros((P, DESC)) if want_desc else None
        lw, lg = lobes(g)
        lib().om_query(self.h, float(sigma_t), float(albedo), len(lw), _ptr(lw, _dp), _ptr(lg, _dp),
                       int(bool(volume)), float(params["lam"]),
                       float(params["gamma"]), float(radiance), _ptr(flat, _dp),
                       int(params["width"]), int(params["n_linear"]), _ptr(pts, _fp),
                       _ptr(dirs, _fp), P, _ptr(L, _dp), _ptr(y, _dp), _ptr(F, _dp),
                       _ptr(desc, _dp))
        out = {"L": L, "y": y, "F": F}
        if want_desc:
            out["desc"] = desc
        return out
