"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This package generates *inputs* only: density grids, light directions, shading
points with view directions, and network weights.  It holds none of the
in-scattering method's arithmetic (no pyramid, no transmittance, no template
sampling, no network evaluation), so that the FP64 oracle and the HIP library
can both be fed from it without sharing any of the computation they are
compared on.

Modules
-------
rng      counter-based SplitMix64 uniform generator (Steele, Lea and Flood 2014)
medium   4-octave value-noise fBm density clouds
camera   orthographic and pinhole cameras plus first-collision delta tracking
weights  He-normal network parameters in the layout the method uses
configs  the five named workloads (32^3 CPU case, 256^3 1080p, precision
         sweep, 512^3 4K, serving trace)
"""

from . import rng, medium, camera, weights, configs  # noqa: F401
