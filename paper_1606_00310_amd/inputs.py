"""Seeded synthetic workloads shaped like the paper's benchmarks (Sec. III):
square or rectangular lattices of lateral size 2^k grown from a flat surface
with given p, q, number of MCS and seed.  This module holds parameters and
random draws of workload parameters only -- none of the model's arithmetic --
so both the GPU path and the CPU oracle's tests can use it.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    X: int
    Y: int
    p: float
    q: float
    n_mcs: int
    seed: int

    @property
    def sites(self) -> int:
        return self.X * self.Y


# The 128x128 validation run: p = 1/2 (one 64-bit draw per word), 1000 MCS.
SMALL = Workload("octahedron-128x128-p0.5-q0", 128, 128, 0.5, 0.0, 1000, 1)
# 2^12 x 2^12 with a two-digit mask (p = 0.11b, q = 0.01b share two draws).
MEDIUM = Workload("octahedron-4096x4096-p0.75-q0.25", 4096, 4096, 0.75, 0.25, 10_000, 7)
# The sweep-throughput workload: 2^16 x 2^16 (1 GiB of packed slopes) at p = 1
# (no random draws), and the p = 0.9375 variant (four-digit mask, two Philox
# calls per word).
HEADLINE = Workload("octahedron-65536x65536-p1-q0", 65536, 65536, 1.0, 0.0, 2000, 42)
HEADLINE_RANDOM = Workload("octahedron-65536x65536-p0.9375-q0", 65536, 65536, 0.9375, 0.0, 2000, 42)
# The paper's own throughput workload (Sec. III): 2^16 x 2^16 at p = 1/2
# (one 64-bit draw per word, half a Philox call).
HEADLINE_HALF = Workload("octahedron-65536x65536-p0.5-q0", 65536, 65536, 0.5, 0.0, 2000, 42)
# Lateral size 2^17 (the paper's cyan bar, Sec. III): 4 GiB of packed slopes.
WIDE = Workload("octahedron-131072x131072-p1-q0", 131072, 131072, 1.0, 0.0, 2000, 42)
# Arbitrary probabilities: one 32-bit uniform per site.
PERSITE = Workload("octahedron-16384x16384-p0.93-q0.07", 16384, 16384, 0.93, 0.07, 5000, 3)
PERSITE_SNAPSHOTS = (100, 1000)


def log_times(t_max: int = 10_000, per_decade: int = 10):
    """Distinct floor(10^(k/per_decade)) up to t_max: 1, 2, 3, 5, 6, 7, 10, ..."""
    out = []
    k = 0
    while True:
        t = int(np.floor(10 ** (k / per_decade) + 1e-9))
        if t > t_max:
            break
        if not out or t != out[-1]:
            out.append(t)
        k += 1
    return out


def autocorr_times(s: int, t_max: int = 5000):
    """Measurement times for C(t, s): s itself, the log-spaced times after s, and t_max."""
    ts = [s] + [t for t in log_times(t_max) if t > s]
    if ts[-1] != t_max:
        ts.append(t_max)
    return ts


@dataclass(frozen=True)
class EnsembleMember:
    L: int
    p: float
    n_mcs: int
    seed: int


def ensemble(n: int = 4096, rng_seed: int = 20160601, l_min_log2: int = 6, l_max_log2: int = 11,
             p_choices=(0.5, 0.75, 0.9375), mcs_log10=(2.0, 4.0), seed0: int = 1_000_000):
    """Independent realizations of uneven size: L = 2^U{6..11}, p from a small
    dyadic set, q = 0, MCS = round(10^U[2,4]), distinct seeds."""
    rng = np.random.default_rng(rng_seed)
    Ls = 2 ** rng.integers(l_min_log2, l_max_log2 + 1, size=n)
    ps = rng.choice(np.asarray(p_choices, dtype=np.float64), size=n)
    mcs = np.rint(10 ** rng.uniform(mcs_log10[0], mcs_log10[1], size=n)).astype(np.int64)
    return [EnsembleMember(int(Ls[i]), float(ps[i]), int(mcs[i]), seed0 + i) for i in range(n)]


def poisson_arrivals(n: int, rate_per_s: float, rng_seed: int = 7):
    """Arrival times (s) of n requests of a Poisson stream."""
    rng = np.random.default_rng(rng_seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=n))
