"""Seeded synthetic workloads (input generators only -- none of the sampler's
arithmetic lives here).  Shared by the tests and the benchmark.

The paper's experiments use synthetic (n, N) pairs only (N = 2^50, n swept);
these generators produce the batched and serving workloads: instance sizes n
log-uniform in [2^8, 2^22] and densities n/N log-uniform in [1e-6, 0.5].
Uniforms come from SplitMix64 (Steele, Lea, Flood 2014) with a fixed key, so
the tables do not depend on any library version.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

_MASK = (1 << 64) - 1
WORKLOAD_KEY = 0x5EED_0F_BA7C4  # fixed key of the batched / serving workloads


def _splitmix64(x: int) -> int:
    x = (x + 0x9E3779B97F4A7C15) & _MASK
    z = x
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31)


def uniform(key: int, i: int, j: int) -> float:
    """A uniform double in [0, 1) for (key, i, j)."""
    h = _splitmix64((key * 0x100000001B3 + i * 0x9E3779B1 + j) & _MASK)
    return (h >> 11) * 2.0**-53


@dataclass(frozen=True)
class Inst:
    n: int
    N: int
    seed: int


def batched_instances(count: int = 4096, n_lo_log2: int = 8, n_hi_log2: int = 22,
                      dens_lo: float = 1e-6, dens_hi: float = 0.5,
                      key: int = WORKLOAD_KEY, n_cap_log2: int | None = None) -> list:
    """Instance i: n = floor(2^(lo + (hi-lo) u1)), density d = dens_lo *
    (dens_hi/dens_lo)^u2, N = max(n, ceil(n / d)), seed = i."""
    out = []
    span = math.log10(dens_hi / dens_lo)
    for i in range(count):
        u1 = uniform(key, i, 1)
        u2 = uniform(key, i, 2)
        n = int(math.floor(2.0 ** (n_lo_log2 + (n_hi_log2 - n_lo_log2) * u1)))
        if n_cap_log2 is not None:
            n = min(n, 1 << n_cap_log2)
        d = dens_lo * 10.0 ** (span * u2)
        N = max(n, int(math.ceil(n / d)))
        out.append(Inst(n=n, N=N, seed=i))
    return out


def poisson_arrivals(count: int, rate_per_s: float, key: int = WORKLOAD_KEY) -> list:
    """Arrival times (seconds) of a Poisson process: gaps -ln(1-u)/rate."""
    t = 0.0
    times = []
    for i in range(count):
        u = uniform(key ^ 0xA77, i, 3)
        t += -math.log1p(-u) / rate_per_s
        times.append(t)
    return times


def segment_lengths(count: int = 4096, lo_log2: float = 16, hi_log2: float = 40,
                    key: int = WORKLOAD_KEY) -> list:
    """Sizes of the segments of an uneven universe (sharded data of uneven
    shard sizes): segment i holds floor(2^(lo + (hi-lo) u)) elements."""
    return [int(math.floor(2.0 ** (lo_log2 + (hi_log2 - lo_log2) * uniform(key ^ 0x5E6, i, 4))))
            for i in range(count)]
