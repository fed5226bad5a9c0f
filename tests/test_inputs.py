"""The seeded input generators (shared by both sides; no search arithmetic)."""
import numpy as np

from paper_2506_01099_amd.inputs import SplitMix64, batched_queries, planted_queries, served_trace


def test_splitmix64_reference_values():
    # Published outputs of SplitMix64 for seed 0 (Steele, Lea & Flood; Vigna's reference code).
    g = SplitMix64(0)
    assert [g.next() for _ in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_batched_queries_shape_and_bounds():
    a, b = batched_queries()
    assert a.size == b.size == 4096
    L = (b - a).astype(np.int64)
    assert L.min() >= 2**10 and L.max() <= 2**24
    assert int(a.max()) < 2**40
    a2, b2 = batched_queries()
    assert np.array_equal(a, a2) and np.array_equal(b, b2)
    total = int(L.sum())
    assert 5e9 < total < 1e10  # E[L] = (2^24 - 2^10) / (14 ln 2) ~ 1.73e6


def test_served_trace_shape_and_rate():
    t, a, b = served_trace(n=2000)
    assert np.all(np.diff(t) > 0)
    rate = t.size / t[-1]
    assert 150 < rate < 260
    L = (b - a).astype(np.int64)
    assert L.min() >= 2**12 and L.max() <= 2**28


def test_planted_queries_are_valid():
    a, b = planted_queries()
    assert np.all(a >= 1) and np.all(b > a)
