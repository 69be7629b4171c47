"""Counter-based random numbers (SplitMix64, Steele, Lea and Flood 2014).

``splitmix64(c)`` maps a 64-bit counter to a 64-bit output with the published
SplitMix64 finaliser: add the golden-ratio increment, then the two
xor-shift-multiply rounds and a final xor-shift.  Everything is vectorised over
numpy ``uint64`` arrays; overflow wraps modulo 2**64 as the definition wants.
"""

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_S30 = np.uint64(30)
_S27 = np.uint64(27)
_S31 = np.uint64(31)
_S11 = np.uint64(11)


def splitmix64(counter):
    """SplitMix64 output for each 64-bit counter value (array or scalar)."""
    z = np.asarray(counter, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = z + _GAMMA
        z = (z ^ (z >> _S30)) * _M1
        z = (z ^ (z >> _S27)) * _M2
    return z ^ (z >> _S31)


def _key(seed, stream, a, b=None):
    """Mix (seed, stream, a[, b]) into one 64-bit counter per element."""
    a = np.asarray(a, dtype=np.uint64)
    with np.errstate(over="ignore"):
        k = splitmix64(np.uint64(seed) * np.uint64(0x100000001B3) + np.uint64(stream))
        k = splitmix64(k ^ a)
        if b is not None:
            k = splitmix64(k ^ (np.asarray(b, dtype=np.uint64) * np.uint64(0xD6E8FEB86659FD93)))
    return k


def uniform01(seed, stream, a, b=None):
    """Uniform on [0, 1) with 53 random bits: (h >> 11) * 2**-53."""
    h = _key(seed, stream, a, b)
    return (h >> _S11).astype(np.float64) * (1.0 / 9007199254740992.0)


def uniform_pm1(seed, stream, a, b=None):
    """Uniform on [-1, 1): 2u - 1 with u from :func:`uniform01`."""
    return 2.0 * uniform01(seed, stream, a, b) - 1.0


def randint_pm(seed, stream, lim, a, b=None):
    """Integers uniform on [-lim, lim] (as float64), from the same hash."""
    h = _key(seed, stream, a, b)
    span = np.uint64(2 * lim + 1)
    return (h % span).astype(np.int64).astype(np.float64) - float(lim)
