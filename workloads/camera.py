"""Cameras and first-collision delta tracking: the frame's shading points.

A frame is produced by tracing one ray per pixel into the unit-cube medium and
keeping the first real collision found by delta (Woodcock) tracking.  Each
collision is a shading point p with the camera-ray direction omega at which
the in-scattered radiance is queried.  Rays that leave the box without a
collision produce no point.

Delta tracking here uses the piecewise-constant (nearest voxel) density
mu(x) = sigma_t * rho0[floor(x * N)] with majorant sigma_t * max(rho0); free
flights are -log(1 - u) / majorant and a tentative collision is accepted with
probability mu(x) / majorant.  Draw 2i is the i-th free flight and draw 2i+1
its acceptance test, both from ``rng.uniform(seed, pixel, draw)``.
"""

import math

import numpy as np

from . import rng


def orthographic_rays(res, z0=1.0):
    """res x res orthographic rays travelling along -z through pixel centres
    of the unit square at height ``z0``.  Returns (origins, dirs) float64."""
    px = (np.arange(res, dtype=np.float64) + 0.5) / res
    yy, xx = np.meshgrid(px, px, indexing="ij")       # row = y, column = x
    o = np.stack([xx.ravel(), yy.ravel(), np.full(res * res, z0)], axis=1)
    d = np.tile(np.array([0.0, 0.0, -1.0]), (res * res, 1))
    return o, d


def pinhole_rays(width, height, vfov_deg=45.0, eye=(0.5, 0.5, 2.0),
                 target=(0.5, 0.5, 0.5), up=(0.0, 1.0, 0.0)):
    """Pinhole rays through pixel centres; pixel index = row * width + col,
    row 0 at the top of the image.  Returns (origins, dirs) float64."""
    eye = np.asarray(eye, dtype=np.float64)
    f = np.asarray(target, dtype=np.float64) - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, dtype=np.float64))
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    t = math.tan(math.radians(vfov_deg) * 0.5)
    aspect = width / height
    col = (np.arange(width, dtype=np.float64) + 0.5) / width * 2.0 - 1.0
    row = 1.0 - (np.arange(height, dtype=np.float64) + 0.5) / height * 2.0
    rr, cc = np.meshgrid(row, col, indexing="ij")
    d = (f[None, :] + (cc.ravel() * aspect * t)[:, None] * r[None, :]
         + (rr.ravel() * t)[:, None] * u[None, :])
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = np.tile(eye, (width * height, 1))
    return o, d


def _box_interval(o, d):
    """Slab-test entry/exit parameters of rays against [0,1]^3."""
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / d
        t0 = (0.0 - o) * inv
        t1 = (1.0 - o) * inv
    tmin = np.nanmax(np.minimum(t0, t1), axis=1)
    tmax = np.nanmin(np.maximum(t0, t1), axis=1)
    return np.maximum(tmin, 0.0), tmax


def delta_track(density, sigma_t, origins, dirs, seed=0, max_steps=100000, pixels=None):
    """First real collision of each ray by delta tracking.

    Returns (points float32 [P,3], dirs float32 [P,3], pixel int64 [P]) for
    the rays that collide inside the box, in pixel order.  ``pixels`` (sorted
    int64, one per ray) tracks a subset of a frame's rays: the random numbers
    and the returned indices are those of these pixels.
    """
    ids = np.arange(origins.shape[0], dtype=np.int64) if pixels is None else np.asarray(pixels, np.int64)
    n = density.shape[0]
    rmax = float(density.max())
    npx = origins.shape[0]
    t_in, t_out = _box_interval(origins, dirs)
    alive = np.nonzero(t_in < t_out)[0]
    hit_t = np.full(npx, np.nan)
    if rmax <= 0.0 or sigma_t <= 0.0:
        return (np.zeros((0, 3), np.float32), np.zeros((0, 3), np.float32),
                np.zeros(0, np.int64))
    majorant = sigma_t * rmax
    t = t_in[alive].copy()
    step = 0
    while alive.size and step < max_steps:
        u_fly = rng.uniform(seed, ids[alive], 2 * step)
        u_acc = rng.uniform(seed, ids[alive], 2 * step + 1)
        t = t - np.log1p(-u_fly) / majorant
        inside = t < t_out[alive]
        x = origins[alive] + t[:, None] * dirs[alive]
        idx = np.clip(np.floor(x * n).astype(np.int64), 0, n - 1)
        rho = density[idx[:, 2], idx[:, 1], idx[:, 0]].astype(np.float64)
        accept = inside & (u_acc * majorant < sigma_t * rho)
        hit_t[alive[accept]] = t[accept]
        keep = inside & ~accept
        alive, t = alive[keep], t[keep]
        step += 1
    hit = np.nonzero(~np.isnan(hit_t))[0]
    pts = origins[hit] + hit_t[hit, None] * dirs[hit]
    return pts.astype(np.float32), dirs[hit].astype(np.float32), ids[hit]


def random_points(count, seed, lo=0.0, hi=1.0):
    """Uniform points in [lo, hi)^3 and uniform unit directions (float32)."""
    idx = np.arange(count, dtype=np.uint64)
    p = np.stack([rng.uniform(seed, idx, k) for k in range(3)], axis=1)
    p = lo + (hi - lo) * p
    z = 2.0 * rng.uniform(seed, idx, 3) - 1.0
    phi = 2.0 * math.pi * rng.uniform(seed, idx, 4)
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    d = np.stack([s * np.cos(phi), s * np.sin(phi), z], axis=1)
    return p.astype(np.float32), d.astype(np.float32)


def uniform_direction(seed, stream=0):
    """A uniform unit vector on the sphere (float64[3])."""
    z = 2.0 * float(rng.uniform(seed, stream, 0)) - 1.0
    phi = 2.0 * math.pi * float(rng.uniform(seed, stream, 1))
    s = math.sqrt(max(0.0, 1.0 - z * z))
    return np.array([s * math.cos(phi), s * math.sin(phi), z])
