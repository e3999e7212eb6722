"""Procedural density clouds: 4-octave value-noise fBm on an N^3 voxel grid.

The cloud stands in for the clouds, smoke and fog media the paper targets
(Introduction; Sec. III.B.4).  The noise is defined in unit-cube coordinates,
so grids of different resolution built from the same seed sample the same
cloud.

Recipe
------
* octave o = 0..3 has R_o = 4 * 2**o lattice cells per unit length and
  (R_o + 1)^3 node values drawn U[0,1) from ``numpy.random.default_rng(seed)``
  in octave order, node array indexed [z][y][x];
* each octave is evaluated at voxel centres (i + 1/2)/N by trilinear
  interpolation with smoothstep weights s(f) = f^2 (3 - 2 f);
* n = sum_o 2^-o v_o / sum_o 2^-o;
* rho = max_density * clamp((n - threshold) / (1 - threshold), 0, 1).

The grid is returned as float32 in [z][y][x] order with x fastest.
"""

import numpy as np

OCTAVES = 4
BASE_CELLS = 4


def _octave_axis(n, cells):
    """Per-axis lattice index and smoothstep weight at the voxel centres."""
    u = (np.arange(n, dtype=np.float64) + 0.5) / n * cells
    i0 = np.minimum(np.floor(u).astype(np.int64), cells - 1)
    f = u - i0
    s = f * f * (3.0 - 2.0 * f)
    return i0, s


def fbm_cloud(n, seed=0, threshold=0.4, max_density=1.0):
    """Return an (n, n, n) float32 density grid [z][y][x] of the fBm cloud."""
    if n < 1:
        raise ValueError("grid edge must be positive")
    rng = np.random.default_rng(seed)
    nodes = []
    for o in range(OCTAVES):
        r = BASE_CELLS * 2 ** o
        nodes.append(rng.random((r + 1, r + 1, r + 1)))
    amp = np.array([2.0 ** -o for o in range(OCTAVES)])
    amp = amp / amp.sum()

    acc = np.zeros((n, n, n), dtype=np.float64)
    for o in range(OCTAVES):
        i0, s = _octave_axis(n, BASE_CELLS * 2 ** o)
        v = nodes[o]
        # the trilinear blend is separable: interpolate x, then y, then z
        vx = v[:, :, i0] * (1.0 - s) + v[:, :, i0 + 1] * s             # (R+1, R+1, n)
        vxy = vx[:, i0, :] * (1.0 - s)[None, :, None] + vx[:, i0 + 1, :] * s[None, :, None]
        for z in range(n):
            acc[z] += amp[o] * (vxy[i0[z]] * (1.0 - s[z]) + vxy[i0[z] + 1] * s[z])
    dens = np.clip((acc - threshold) / (1.0 - threshold), 0.0, 1.0) * max_density
    return dens.astype(np.float32)


def constant(n, value):
    """Homogeneous slab of density ``value``."""
    return np.full((n, n, n), value, dtype=np.float32)
