"""Seeded synthetic inputs (query ranges and request traces); no search arithmetic here.

SplitMix64 is the generator of Steele, Lea and Flood (OOPSLA 2014): state += 0x9E3779B97F4A7C15,
then the xor-shift-multiply finaliser.  Both the GPU side and the oracle side receive
the arrays produced here.
"""
import math

import numpy as np

MASK64 = (1 << 64) - 1


class SplitMix64:
    def __init__(self, seed):
        self.state = seed & MASK64

    def next(self):
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def unit(self):
        """Uniform in [0, 1) with 53 bits."""
        return (self.next() >> 11) * (1.0 / (1 << 53))


def batched_queries(n=4096, seed=2506, log2_min=10, log2_max=24, a_bits=40):
    """Range queries [a, a + L): L = floor(2^(log2_min + (log2_max - log2_min) u)), a uniform in [0, 2^a_bits)."""
    g = SplitMix64(seed)
    a = np.empty(n, dtype=np.uint64)
    L = np.empty(n, dtype=np.uint64)
    for i in range(n):
        u = g.unit()
        length = int(math.floor(2.0 ** (log2_min + (log2_max - log2_min) * u)))
        length = min(max(length, 1 << log2_min), 1 << log2_max)
        start = g.next() >> (64 - a_bits)
        a[i], L[i] = start, length
    return a, a + L


def served_trace(n=12000, seed=1099, rate=200.0, log2_min=12, log2_max=28, a_bits=40):
    """Poisson arrivals (rate per second) of range requests: (t_arrival, a, b) arrays."""
    g = SplitMix64(seed)
    t = np.empty(n, dtype=np.float64)
    a = np.empty(n, dtype=np.uint64)
    L = np.empty(n, dtype=np.uint64)
    now = 0.0
    for i in range(n):
        now += -math.log(1.0 - g.unit()) / rate
        u = g.unit()
        length = int(math.floor(2.0 ** (log2_min + (log2_max - log2_min) * u)))
        length = min(max(length, 1 << log2_min), 1 << log2_max)
        t[i] = now
        a[i] = g.next() >> (64 - a_bits)
        L[i] = length
    return t, a, a + L


def planted_queries():
    """Ranges that contain known pairs: prefixes [1, b) and windows around small family members."""
    qs = [(1, 1 << 12), (1, 1 << 16), (1, 1 << 20), (1, 1 << 24), (2, 9), (3, 9), (74, 1217), (34, 4376)]
    for k in range(2, 12):
        m, n = 2**k - 2, 2**(2 * k) - 2**(k + 1)
        qs.append((m, n + 1))
        qs.append((m + 1, n + 1))
    for k in range(0, 12):
        m, n = 2**k + 1, 2**(2 * k) + 2**(k + 1)
        qs.append((m, n + 1))
        qs.append((m, n))
    a = np.array([q[0] for q in qs], dtype=np.uint64)
    b = np.array([q[1] for q in qs], dtype=np.uint64)
    return a, b
