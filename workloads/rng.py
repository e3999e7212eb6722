"""Counter-based uniform random numbers from the SplitMix64 mixer.

SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014) advances a 64-bit state by the golden-ratio constant
0x9E3779B97F4A7C15 and finalises it with two xor-shift-multiply rounds
(shifts 30, 27, 31; multipliers 0xBF58476D1CE4E5B9 and 0x94D049BB133111EB).

Here it is used as a stateless hash of a (seed, stream, draw) triple:

    h = mix(mix(mix(seed) ^ stream) ^ draw),   mix(x) = finalise(x + golden)

and the uniform variate is the top 53 bits of h scaled by 2**-53, so it lies in
[0, 1).  Everything is vectorised over numpy uint64 arrays with wrap-around
arithmetic.
"""

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def mix(x):
    """One SplitMix64 step applied to ``x`` (uint64 scalar or array)."""
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = x + _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def hash3(seed, stream, draw):
    """64-bit hash of (seed, stream, draw); arguments broadcast."""
    s = mix(np.uint64(seed))
    s = mix(s ^ np.asarray(stream, dtype=np.uint64))
    return mix(s ^ np.asarray(draw, dtype=np.uint64))


def uniform(seed, stream, draw):
    """U[0,1) doubles from the top 53 bits of ``hash3(seed, stream, draw)``."""
    h = hash3(seed, stream, draw)
    return (h >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
