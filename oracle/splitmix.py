"""SplitMix64 (Steele, Lea and Flood, OOPSLA 2014), the counter-based generator both sides use
for the Lanczos start vector.

Test infrastructure only (see the package docstring).

splitmix64(x): z = x + 0x9E3779B97F4A7C15; z = (z ^ z>>30) * 0xBF58476D1CE4E5B9;
z = (z ^ z>>27) * 0x94D049BB133111EB; return z ^ z>>31   (all mod 2^64).
A 64-bit output h maps to a double in [0, 1) as (h >> 11) * 2^-53.
"""

from __future__ import annotations

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(x):
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = x + _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def unit_double(h):
    return (np.asarray(h, dtype=np.uint64) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def start_vector(seed: int, level: int, n: int):
    """v_g = u(splitmix64(seed ^ g ^ (level << 32))) - 1/2 for every global node index g < n."""
    g = np.arange(n, dtype=np.uint64)
    key = np.uint64(seed) ^ g ^ (np.uint64(level) << np.uint64(32))
    return unit_double(splitmix64(key)) - 0.5
