"""Shared set-up of the GPU parity tests: one library context, seeded inputs,
and the oracle fed with exactly the float32 values the library receives."""

import numpy as np

from oracle import oracle
from workloads import camera, configs, medium, weights


def f32(x):
    """The float32 value a float parameter becomes at the C ABI, as a double."""
    return float(np.float32(x))


def oracle_params(params):
    """Copy of ``params`` whose lambda/gamma are the float32 blob values."""
    p = dict(params)
    p["lam"] = f32(params["lam"])
    p["gamma"] = f32(params["gamma"])
    return p


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


class Scene:
    """A medium loaded both on the GPU and in the oracle, under one light.  g
    is one HG asymmetry or a sequence of (weight, g) lobes."""

    def __init__(self, ctx, density, light, sigma_t=8.0, albedo=0.99, g=0.85, radiance=1.0, volume=False):
        self.ctx = ctx
        self.volume = volume
        self.density = np.ascontiguousarray(density, np.float32)
        self.sigma_t, self.albedo, self.g, self.radiance = sigma_t, albedo, g, radiance
        if np.ndim(g) == 0:
            self.mid = ctx.load_medium(self.density, sigma_t, albedo, g)
        else:
            self.mid = ctx.load_medium(self.density, sigma_t, albedo, g[0][1])
            ctx.set_phase_lobes(self.mid, g)
        if volume:
            ctx.set_volume_phase(self.mid, True)
        self.ctx.set_light(self.mid, light, radiance)
        self.om = oracle.Medium(self.density)
        self.om.set_light(np.asarray(light, np.float32))

    def close(self):
        self.ctx.unload_medium(self.mid)

    def phase(self):
        """The phase as the library holds it (float32 values)."""
        if np.ndim(self.g) == 0:
            return f32(self.g)
        return [(f32(w), f32(g)) for w, g in self.g]

    def oracle_query(self, params, pts, dirs, want_desc=False):
        return self.om.query(oracle_params(params), pts, dirs, f32(self.sigma_t), f32(self.albedo),
                             self.phase(), f32(self.radiance), want_desc=want_desc, volume=self.volume)

    def oracle_tpl_features(self, params, pts, dirs):
        return self.om.tpl_features(f32(self.sigma_t), self.phase(), f32(params["lam"]), pts, dirs)

    def oracle_tpl_query(self, params, pts, dirs, want_desc=False):
        return self.om.tpl_query(oracle_params(params), pts, dirs, f32(self.sigma_t), f32(self.albedo),
                                 self.phase(), f32(self.radiance), want_desc=want_desc)

    def oracle_tpl_modules_query(self, params, mods, pts, dirs, want_desc=False):
        return self.om.tpl_modules_query(oracle_params(params), mods, pts, dirs, f32(self.sigma_t),
                                         f32(self.albedo), self.phase(), f32(self.radiance), want_desc=want_desc)

    def oracle_features(self, params, pts, dirs):
        return self.om.features(f32(self.sigma_t), self.phase(), f32(params["lam"]), pts, dirs, volume=self.volume)


def small_points(extra_random=300, seed=5):
    """The 32^3 orthographic frame's collisions plus random points, some of
    them outside the unit cube."""
    w = configs.SMALL
    d = w.density()
    p, dd, _ = w.points(d)
    rp, rd = camera.random_points(extra_random, seed=seed, lo=-0.3, hi=1.3)
    return d, np.concatenate([p, rp]), np.concatenate([dd, rd])


def set_precision(ctx, prec, mid=None, pts=None, dirs=None):
    """ctx.set_precision(prec); for FP8 the static activation scales are
    calibrated first, with the FP32 path over the given points of medium mid
    (nis_calibrate_fp8)."""
    if prec == "fp8":
        import torch
        tp = torch.from_numpy(np.ascontiguousarray(pts, np.float32)).cuda()
        td = torch.from_numpy(np.ascontiguousarray(dirs, np.float32)).cuda()
        ctx.calibrate_fp8(mid, tp, td)
    ctx.set_precision(prec)


__all__ = ["f32", "oracle_params", "rel_l2", "Scene", "small_points", "set_precision", "configs", "medium",
           "weights", "camera", "oracle"]
