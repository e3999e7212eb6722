"""The named workloads: medium, light, camera and network shapes.

``small``   32^3 cloud, 64x64 orthographic camera (<= 4096 points), MLP 6 x 128
``frame``   256^3 cloud, 1920x1080 pinhole camera (~1.2M points), MLP 10 x 200
``precision`` the ``frame`` workload with g swept over {0, 0.5, 0.85, 0.95}
``large``   512^3 cloud, albedo 0.999, g 0.9, 3840x2160 camera (~5M points)
``serving`` Poisson arrivals at 200 req/s over media of 64^3..512^3 and
            resolutions 256^2 / 720p / 1080p with random light and g

Shared medium parameters: sigma_t 8, albedo 0.99, g 0.85, light direction
(0.3, 0.9, 0.3) normalised, radiance 1, medium seed 0, point seed 0, weight
seed 1.
"""

from dataclasses import dataclass, field

import numpy as np

from . import camera, medium, weights

LIGHT_DIR = (0.3, 0.9, 0.3)


@dataclass
class Workload:
    name: str
    n: int
    sigma_t: float = 8.0
    albedo: float = 0.99
    g: float = 0.85
    light: tuple = LIGHT_DIR
    radiance: float = 1.0
    cam: str = "ortho"
    res: tuple = (64, 64)
    eye: tuple = (0.5, 0.5, 2.0)
    width: int = 128
    n_linear: int = 6
    medium_seed: int = 0
    point_seed: int = 0
    weight_seed: int = 1
    g_sweep: tuple = field(default_factory=tuple)

    def density(self):
        return medium.fbm_cloud(self.n, seed=self.medium_seed)

    def rays(self):
        if self.cam == "ortho":
            return camera.orthographic_rays(self.res[0])
        return camera.pinhole_rays(self.res[0], self.res[1], eye=self.eye)

    def points(self, density=None):
        """(points, dirs, pixel) of the frame's first collisions."""
        if density is None:
            density = self.density()
        o, d = self.rays()
        return camera.delta_track(density, self.sigma_t, o, d, seed=self.point_seed)

    def params(self):
        return weights.he_init(self.width, self.n_linear, seed=self.weight_seed)


SMALL = Workload("small", n=32)
# The pinhole eye sits at z = 1.65 (0.65 in front of the cube) so that a 1080p
# frame of the 256^3 cloud yields about 1.2M first collisions (1,206,872).
FRAME_EYE = (0.5, 0.5, 1.65)
FRAME = Workload("frame", n=256, cam="pinhole", res=(1920, 1080), eye=FRAME_EYE,
                 width=200, n_linear=10)
PRECISION = Workload("precision", n=256, cam="pinhole", res=(1920, 1080), eye=FRAME_EYE,
                     width=200, n_linear=10, g_sweep=(0.0, 0.5, 0.85, 0.95))
LARGE = Workload("large", n=512, albedo=0.999, g=0.9, cam="pinhole", res=(3840, 2160),
                 eye=FRAME_EYE, width=200, n_linear=10)

BY_NAME = {w.name: w for w in (SMALL, FRAME, PRECISION, LARGE)}


def serving_trace(seconds=60.0, rate=200.0, seed=7):
    """Poisson frame requests: list of dicts with arrival time (s), medium edge,
    resolution, light direction and g, all drawn from ``default_rng(seed)``."""
    r = np.random.default_rng(seed)
    t, out = 0.0, []
    sizes = (64, 128, 256, 512)
    resolutions = ((256, 256), (1280, 720), (1920, 1080))
    while True:
        t += r.exponential(1.0 / rate)
        if t >= seconds:
            break
        z = 2.0 * r.random() - 1.0
        phi = 2.0 * np.pi * r.random()
        s = np.sqrt(max(0.0, 1.0 - z * z))
        out.append({
            "t": t,
            "n": int(sizes[r.integers(len(sizes))]),
            "res": resolutions[r.integers(len(resolutions))],
            "light": (s * np.cos(phi), s * np.sin(phi), z),
            "g": float(r.uniform(0.3, 0.95)),
            "seed": int(r.integers(1 << 31)),
        })
    return out
