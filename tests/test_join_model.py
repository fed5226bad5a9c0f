"""CPU checks of the numpy join model that the GPU candidate-count tests compare with.

The model (tests/join_model.py) restates the member test and the key grouping in
numpy.  Its member test must stay exact where x * (rad - 1) passes 2^63, which
happens for x near 2^32 and above: here it is compared with the rule evaluated on
Python integers, over windows whose bound b puts many squarefree x on both sides
of the product test.  The grouping is compared with brute-force pair counting.
"""
import numpy as np
import pytest

import join_model
import oracle
from test_member_test import may_pair


@pytest.mark.parametrize("a", [5, 1 << 20, 5 << 30, (1 << 40) - 3000])
def test_kept_is_exact_at_every_magnitude(a):
    n = 3000
    rad = oracle.radicals(a, a + n + 1).astype(np.int64)
    x = np.arange(a, a + n, dtype=np.int64)
    r0, r1 = rad[:n], rad[1:n + 1]
    # Bounds from just above 2a (every squarefree x dropped but the smallest) to the
    # 2^42 value limit; from x near 2^32 on the products x * (rad - 1) pass 2^63.
    for b in (2 * a + 7, min(a * 1000, (1 << 42) - 1)):
        got = join_model.kept(x, r0, r1, b)
        want = [may_pair(int(x[i]), int(r0[i]), int(r1[i]), b) for i in range(n)]
        assert got.tolist() == want, (a, b)
    if a > 1 << 32:
        sq = r0 == x
        assert max(int(x[i]) * (int(r1[i]) - 1) for i in np.flatnonzero(sq)) > 1 << 63


def test_candidates_is_pair_count():
    rng = np.random.default_rng(7)
    keys = rng.integers(0, 50, size=400).astype(np.uint64)
    brute = sum(1 for i in range(keys.size) for j in range(i + 1, keys.size) if keys[i] == keys[j])
    assert join_model.candidates(keys) == brute
    assert join_model.candidates(np.zeros(0, dtype=np.uint64)) == 0


M64 = (1 << 64) - 1


def _key64_int(lo, hi, grp):
    """key64 on Python integers: SplitMix64's output mix over (lo | grp << 43) * K xor hi."""
    z = ((((lo | (grp << 43)) * 0x9E3779B97F4A7C15) & M64) ^ hi)
    z ^= z >> 30
    z = (z * 0xBF58476D1CE4E5B9) & M64
    z ^= z >> 27
    z = (z * 0x94D049BB133111EB) & M64
    z ^= z >> 31
    return z


def _brute_groups(a, b, grp, group_of):
    """Pairs of kept x in [a, b) whose groups (a tuple from the key hash) agree, counted
    pair by pair on Python integers."""
    rad = [int(v) for v in oracle.radicals(a, b + 1)]
    groups = []
    for i in range(b - a):
        x, r0, r1 = a + i, rad[i], rad[i + 1]
        if not may_pair(x, r0, r1, b):
            continue
        h = _key64_int(min(r0, r1), max(r0, r1), grp)
        groups.append(group_of(h))
    return sum(1 for i in range(len(groups)) for j in range(i + 1, len(groups)) if groups[i] == groups[j]), len(groups)


@pytest.mark.parametrize("a,b,b1,b2,keep", [(1, 20001, 2, 3, 6), (1 << 20, (1 << 20) + 6000, 1, 4, 5),
                                            ((1 << 36) - 4000, 1 << 36, 0, 2, 7)])
def test_compact_keys_match_pairwise_count(a, b, b1, b2, keep):
    """The compact-word grouping (bucket = low b1 hash bits, partition = top b2 of the 53-bit
    fingerprint, kept = its low `keep` bits) against pair-by-pair counting on Python integers."""
    def group_of(h):
        fp = h >> 11
        return (h & ((1 << b1) - 1), fp >> (53 - b2), fp & ((1 << keep) - 1))

    want, n_kept = _brute_groups(a, b, 3, group_of)
    keys, got_kept = join_model.compact_keys(oracle.radicals(a, b + 1), a, b, 3, b1, b2, keep)
    assert got_kept == n_kept and want > 0
    assert join_model.candidates(keys) == want


@pytest.mark.parametrize("passes,fp_bits", [(1, 9), (3, 8)])
def test_group_keys_match_pairwise_count(passes, fp_bits):
    """The 12-byte-entry grouping (pass, bucket, query, top 11 and low fp_bits fingerprint bits)
    against pair-by-pair counting on Python integers, the pass taken from the 24-bit-multiply
    hash restated on integers."""
    a, b, b1, grp = 1, 12001, 2, 5

    def pass_of(lo, hi):
        m = 0xFFFFFF
        l0, l1, h0, h1 = lo & 0x1FFFFF, lo >> 21, hi & 0x1FFFFF, hi >> 21
        s = ((l0 & m) * 0x9E3779 + (l1 & m) * 0x7F4A7D + (h0 & m) * 0xC2B2AF + (h1 & m) * 0x85EBCB
             + (grp & m) * 0x27D4EB) & 0xFFFFFFFF
        s ^= s >> 15
        s = (s * 0x2C1B3C6D) & 0xFFFFFFFF
        s ^= s >> 12
        return sum(1 for p in range(1, passes) if s >= (p << 32) // passes)

    rad = [int(v) for v in oracle.radicals(a, b + 1)]
    groups = []
    for i in range(b - a):
        x, r0, r1 = a + i, rad[i], rad[i + 1]
        if not may_pair(x, r0, r1, b):
            continue
        lo, hi = min(r0, r1), max(r0, r1)
        h = _key64_int(lo, hi, grp)
        fp = h >> 11
        groups.append((pass_of(lo, hi), h & ((1 << b1) - 1), fp >> 42, fp & ((1 << fp_bits) - 1)))
    want = sum(1 for i in range(len(groups)) for j in range(i + 1, len(groups)) if groups[i] == groups[j])
    keys, n_kept = join_model.group_keys(oracle.radicals(a, b + 1), a, b, grp, b1, passes, fp_bits)
    assert n_kept == len(groups) and want > 0
    assert join_model.candidates(keys) == want
