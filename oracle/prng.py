"""SplitMix64 (Steele, Lea, Flood 2014; public-domain reference by S. Vigna).

Counter-based form: the i-th output (i = 0, 1, ...) for a seed s is
``mix(s + (i + 1) * 0x9E3779B97F4A7C15)`` with the published finaliser

    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB
    z =  z ^ (z >> 31)

all modulo 2**64.  Random draws of the method (k-means++ seeding, Rademacher
probe vectors, Lanczos start blocks) are defined in terms of this stream so the
oracle and the HIP library draw identical numbers.

Derived draws (stream layout shared with the library):

* ``uniform(seed, i)``   = (u64 >> 11) * 2**-53          in [0, 1)
* ``rademacher(seed, i)``= +1 if the top bit of u64 is 0, else -1
* ``gauss(seed, i)``     = sqrt(-2 ln(1 - u(2i))) * cos(2 pi u(2i+1))  (Box-Muller)
"""
from __future__ import annotations

import numpy as np

MASK = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def splitmix64(seed: int, i: int) -> int:
    z = (seed + (i + 1) * GAMMA) & MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def splitmix64_array(seed: int, start: int, count: int) -> np.ndarray:
    """Outputs ``start .. start+count-1`` as uint64 (vectorised, same definition)."""
    with np.errstate(over="ignore"):
        i = np.arange(start, start + count, dtype=np.uint64)
        z = np.uint64(seed & MASK) + (i + np.uint64(1)) * np.uint64(GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform(seed: int, start: int, count: int) -> np.ndarray:
    return (splitmix64_array(seed, start, count) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def rademacher(seed: int, start: int, count: int) -> np.ndarray:
    top = splitmix64_array(seed, start, count) >> np.uint64(63)
    return np.where(top == 0, 1.0, -1.0)


def gauss(seed: int, start: int, count: int) -> np.ndarray:
    u = uniform(seed, 2 * start, 2 * count)
    u1 = u[0::2]
    u2 = u[1::2]
    return np.sqrt(-2.0 * np.log(1.0 - u1)) * np.cos(2.0 * np.pi * u2)


def derive(seed: int, tag: int) -> int:
    """Sub-stream seed: first output of SplitMix64 keyed by seed xor tag."""
    return splitmix64((seed ^ tag) & MASK, 0)


# stream tags (shared layout with the library)
TAG_KPM = 0x4B504D            # Rademacher probe vectors for the DOS estimate
TAG_BOUNDS = 0x424E44         # start vector of the spectral-bounds Lanczos
TAG_LANCZOS = 0x4C4E43        # Lanczos / subspace start blocks (xor shift index << 32)
TAG_KMEANSPP = 0x4B4D50       # k-means++ seeding draws
