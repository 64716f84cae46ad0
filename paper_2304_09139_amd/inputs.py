"""Seeded synthetic inputs shared by the tests, the oracle checks and the benchmark.

This module only draws random numbers and formats them; it contains none of the
method's arithmetic.  The paper starts every quench from a Poisson point
process, i.e. independent uniform positions in the periodic box ("Simulations"
section).  Here each fractional coordinate is an exact 106-bit dyadic
u = a 2^-53 + b 2^-106 with a, b the top 53 bits of two SplitMix64 outputs
(Steele, Lea and Flood, OOPSLA 2014), stored as a normalised hi/lo pair:
hi = u rounded to the nearest double and lo = u - hi exactly.

Positions use the ``float64[2, d, N]`` layout (hi plane, lo plane) of the
library's C interface.
"""
from __future__ import annotations

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """Outputs offset .. offset+count-1 of the SplitMix64 stream started at ``seed``."""
    with np.errstate(over="ignore"):
        idx = np.arange(offset + 1, offset + count + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + idx * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def stream_seed(*keys: int) -> int:
    """Fold a tuple of integers (config id, replica, ...) into one 64-bit seed."""
    s = 0x243F6A8885A308D3
    for k in keys:
        s = int(splitmix64(s ^ (int(k) & 0xFFFFFFFFFFFFFFFF), 1)[0])
    return s


def uniform_positions(d: int, N: int, seed: int) -> np.ndarray:
    """iid uniform fractional positions in [0, 1)^d as float64[2, d, N]."""
    raw = splitmix64(seed, 2 * d * N).reshape(d, N, 2)
    a = (raw[..., 0] >> np.uint64(11)).astype(np.float64)   # 53-bit integers, exact
    b = (raw[..., 1] >> np.uint64(11)).astype(np.float64)
    ta = a * 2.0 ** -53                                     # exact scalings
    tb = b * 2.0 ** -106
    hi = ta + tb                                            # one rounding: nearest double to u
    lo = (ta - hi) + tb                                     # exact remainder u - hi
    out = np.empty((2, d, N), dtype=np.float64)
    out[0] = hi
    out[1] = lo
    return out


def config_positions(cfg_id: int, d: int, N: int, replica: int = 0) -> np.ndarray:
    """Positions for a named workload and replica (seed = stream_seed(cfg_id, replica))."""
    return uniform_positions(d, N, stream_seed(cfg_id, replica))


def batch_shapes(count: int, seed: int = 3, n_min: int = 500, n_max: int = 5000,
                 dims=(2, 3), chis=(0.2, 0.35, 0.45)) -> list[tuple[int, int, float]]:
    """A seeded mix of independent quench shapes (d, N, chi): d uniform over
    ``dims``, N = round(10^U) with U uniform on [log10 n_min, log10 n_max], chi
    uniform over ``chis`` -- many small independent runs, as in a sweep of
    Poisson starts."""
    raw = splitmix64(stream_seed(seed, count), 3 * count).reshape(count, 3)
    out = []
    lo, hi = np.log10(n_min), np.log10(n_max)
    for r in raw:
        d = dims[int(r[0] % np.uint64(len(dims)))]
        u = float(r[1] >> np.uint64(11)) * 2.0 ** -53
        N = int(round(10.0 ** (lo + (hi - lo) * u)))
        chi = chis[int(r[2] % np.uint64(len(chis)))]
        out.append((d, N, chi))
    return out


def serve_stream(count: int, seed: int = 5, n_min: int = 500, n_max: int = 5000, dims=(2, 3),
                 chi_min: float = 0.1, chi_max: float = 0.49) -> list[tuple[int, int, float, float]]:
    """A seeded stream of quench requests (d, N, chi, t): d uniform over ``dims``,
    N log-uniform on [n_min, n_max], chi uniform on [chi_min, chi_max], and
    arrival times t of a unit-rate Poisson process (exponential gaps -ln(1 - U))."""
    raw = splitmix64(stream_seed(seed, count), 4 * count).reshape(count, 4)
    out = []
    t = 0.0
    lo, hi = np.log10(n_min), np.log10(n_max)
    for r in raw:
        u = [float(x >> np.uint64(11)) * 2.0 ** -53 for x in r[1:]]
        d = dims[int(r[0] % np.uint64(len(dims)))]
        N = int(round(10.0 ** (lo + (hi - lo) * u[0])))
        chi = chi_min + (chi_max - chi_min) * u[1]
        t += -np.log1p(-u[2])
        out.append((d, N, chi, t))
    return out
