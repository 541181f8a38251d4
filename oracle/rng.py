"""Counter-based white noise for the initial conditions (the paper draws its ICs from
external simulations; this generator is the synthetic stand-in).

SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): the k-th output (k = 0, 1, ...) of
a generator seeded with s is mix64(s + (k + 1) * 0x9E3779B97F4A7C15) (mod 2^64) with
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
  z = (z ^ (z >> 27)) * 0x94D049BB133111EB
  z =  z ^ (z >> 31)
Grid point j (row-major j = (ix n + iy) n + iz) uses outputs 2j and 2j+1, mapped to
u = ((z >> 11) + 0.5) 2^-53 in (0, 1), and the Box-Muller cosine branch
g = sqrt(-2 ln u0) cos(2 pi u1) gives a standard normal deviate.
"""

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed, counter):
    """Vectorised SplitMix64 output number `counter` (uint64 array) for `seed`."""
    with np.errstate(over="ignore"):
        c = np.asarray(counter, dtype=np.uint64)
        z = np.uint64(seed) + (c + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def to_unit(z):
    return ((z >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53


def white_noise(seed, n):
    """Unit-variance Gaussian white noise on an n^3 grid, float64, shape (n, n, n)."""
    j = np.arange(n ** 3, dtype=np.uint64)
    u0 = to_unit(splitmix64(seed, 2 * j))
    u1 = to_unit(splitmix64(seed, 2 * j + np.uint64(1)))
    g = np.sqrt(-2.0 * np.log(u0)) * np.cos(2.0 * np.pi * u1)
    return g.reshape(n, n, n)
