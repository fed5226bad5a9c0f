"""Pins of the oracle against what the paper and the mathematics fix (CPU only).

Each pin is independent of the oracle's own code: brute force by the definition
with radicals from a smallest-prime-factor sieve, the closed forms of Theorem 1,
the printed Tables 1 and 2, the Moebius count of squarefree integers and
algebraic properties of the radical.
"""
import math

import numpy as np
import pytest

import oracle
from paper_facts import THEOREM1_LIMIT, golden, load_table, theorem1_pairs


def spf_radicals(limit):
    """rad(x) for 0 <= x <= limit from a smallest-prime-factor sieve (index 0 unused)."""
    spf = np.zeros(limit + 1, dtype=np.int64)
    for p in range(2, limit + 1):
        if spf[p] == 0:
            spf[p::p][spf[p::p] == 0] = p
    rad = np.zeros(limit + 1, dtype=np.int64)
    rad[1] = 1
    for x in range(2, limit + 1):
        y, r = x, 1
        while y > 1:
            p = spf[y]
            r *= p
            while y % p == 0:
                y //= p
        rad[x] = r
    return rad


def mobius(limit):
    mu = np.ones(limit + 1, dtype=np.int64)
    is_comp = np.zeros(limit + 1, dtype=bool)
    for p in range(2, limit + 1):
        if not is_comp[p]:
            is_comp[2 * p::p] = True
            mu[p::p] *= -1
            mu[p * p::p * p] = 0
    mu[0] = 0
    return mu


def squarefree_count(n):
    """#{1 <= x <= n : x squarefree} = sum_{d <= sqrt n} mu(d) floor(n / d^2)."""
    r = math.isqrt(n)
    mu = mobius(r)
    return int(sum(int(mu[d]) * (n // (d * d)) for d in range(1, r + 1)))


def primes_upto(n):
    s = np.ones(n + 1, dtype=bool)
    s[:2] = False
    for p in range(2, math.isqrt(n) + 1):
        if s[p]:
            s[p * p::p] = False
    return np.nonzero(s)[0]


# --- brute force by the definition -------------------------------------------------

def test_bruteforce_definition_upto_2_12():
    """Every m < n <= 2^12 checked against the two definitions (Section 1)."""
    N = 2**12
    r = spf_radicals(N + 1)
    expect = []
    for m in range(1, N):
        n = np.arange(m + 1, N + 1)
        first = (r[n] == r[m]) & (r[n + 1] == r[m + 1])
        second = (r[n + 1] == r[m]) & (r[n] == r[m + 1])
        assert not np.any(first & second)
        expect += [(m, int(k), 1) for k in n[first]]
        expect += [(m, int(k), 2) for k in n[second]]
    expect.sort()
    assert expect == oracle.search(N)
    assert expect == theorem1_pairs(N)
    assert len(expect) == 12


def test_small_radicals_match_sieve():
    r = spf_radicals(5000)
    assert np.array_equal(oracle.radicals(1, 5001).astype(np.int64), r[1:])


# --- Theorem 1 and the families of Section 1 ---------------------------------------------

@pytest.mark.parametrize("N", [2**16, 2**20])
def test_theorem1_complete_list(N):
    assert oracle.search(N) == theorem1_pairs(N)


@pytest.mark.slow
def test_theorem1_complete_list_2_24():
    got = oracle.search(2**24)
    assert got == theorem1_pairs(2**24)
    assert len(got) == 25


def test_counts_per_kind_2_20():
    got = oracle.search(2**20)
    assert sum(1 for p in got if p[2] == 1) == 10
    assert sum(1 for p in got if p[2] == 2) == 11


def test_families_and_exceptions_by_radical():
    """The closed forms of Section 1 satisfy the definitions (radicals by the oracle)."""
    for k in range(2, 21):
        m, n = 2**k - 2, 2**k * (2**k - 2)
        assert n == (m + 1) ** 2 - 1 == m * (m + 2)
        assert oracle.rad(m) == oracle.rad(n) and oracle.rad(m + 1) == oracle.rad(n + 1)
    for k in range(0, 21):
        m = 2**k + 1
        n = m * m - 1
        assert oracle.rad(m) == oracle.rad(n + 1) and oracle.rad(m + 1) == oracle.rad(n)
    assert oracle.rad(75) == oracle.rad(1215) == 15 and oracle.rad(76) == oracle.rad(1216) == 38
    assert oracle.rad(35) == oracle.rad(4375) == 35 and oracle.rad(36) == oracle.rad(4374) == 6


def test_group_of_three():
    """{2, 3, 8} share the set {2, 3}: all three pairs are reported."""
    got = oracle.search(8)
    assert got == [(2, 3, 2), (2, 8, 1), (3, 8, 2)]


def test_kinds_filter():
    full = oracle.search(2**20)
    assert oracle.search(2**20, kinds=1) == [p for p in full if p[2] == 1]
    assert oracle.search(2**20, kinds=2) == [p for p in full if p[2] == 2]
    with pytest.raises(ValueError):
        oracle.search(10, kinds=0)


@pytest.mark.parametrize("a,b", [(1, 9), (2, 9), (3, 9), (1, 8), (0, 100), (36, 4375), (35, 4375), (35, 4374),
                                 (1000, 2**20 + 1), (126, 16129), (127, 16129), (500, 501), (7, 7), (9, 3)])
def test_range_semantics(a, b):
    """A range [a, b) reports exactly the pairs with both members in it."""
    full = theorem1_pairs(2**20)
    assert oracle.search_range(a, b) == [p for p in full if p[0] >= max(a, 1) and p[1] < b]


def test_larger_member_non_squarefree():
    """For every pair but (2, 3) both n and n+1 are non-squarefree (rad(x) < x)."""
    for m, n, _ in oracle.search(2**20):
        if (m, n) == (2, 3):
            assert oracle.rad(n) == n
            continue
        assert oracle.rad(n) < n and oracle.rad(n + 1) < n + 1


# --- Tables 1 and 2 -----------------------------------------------------------------

def _prime_set_rad(fact):
    return math.prod(fact.keys())


@pytest.mark.parametrize("name,kind", [("paper_table1_first_kind.txt", 1), ("paper_table2_second_kind.txt", 2)])
def test_paper_tables(name, kind):
    rows = load_table(golden(name))
    small = set(int(p) for p in primes_upto(2**21))
    for m, n, facts in rows:
        if kind == 1:
            vals = (m, n, m + 1, n + 1)
        else:
            vals = (m, n + 1, m + 1, n)
        for v, f in zip(vals, facts):
            for p in f:
                assert v % p == 0
                assert p in small or all(p % q for q in small if q * q <= p)
            assert oracle.rad(v) == _prime_set_rad(f), (v, f)
        assert oracle.rad(vals[0]) == oracle.rad(vals[1])
        assert oracle.rad(vals[2]) == oracle.rad(vals[3])
    pairs = sorted((m, n, kind) for m, n, _ in rows)
    assert pairs == [p for p in theorem1_pairs(THEOREM1_LIMIT - 1) if p[2] == kind]


# --- radicals: Moebius count and properties -------------------------------------------

@pytest.mark.parametrize("N", [2**16, 2**20])
def test_squarefree_count_moebius(N):
    r = oracle.radicals(1, N + 1)
    x = np.arange(1, N + 1, dtype=np.uint64)
    assert int(np.count_nonzero(r == x)) == squarefree_count(N)


def test_squarefree_count_known_value():
    assert squarefree_count(2**20) == 637461


def test_rad_prime_powers():
    for p in [2, 3, 5, 7, 97, 65537, 131071, 524287, 1048573]:
        k = 1
        while p**k < 2**42:
            assert oracle.rad(p**k) == p
            k += 1


def test_rad_properties_random():
    """rad(x) | x, x | rad(x)^42, rad(x) squarefree; multiplicative on coprime pairs."""
    rng = np.random.default_rng(20250601)
    small = [int(p) for p in primes_upto(2**21)]
    xs = [int(v) for v in rng.integers(1, 2**42, size=40)] + [2**41 - 1, 2**42 - 1, 3**26, 2**40, 6**16]
    for x in xs:
        r = oracle.rad(x)
        assert x % r == 0
        assert pow(r, 42, x) == 0 if x > 1 else r == 1
        for p in small:
            if p * p > r:
                break
            assert r % (p * p) != 0
        # the cofactor above 2^21 (if any) is a single prime to the first power
    for _ in range(40):
        a, b = (int(v) for v in rng.integers(1, 2**20, size=2))
        if math.gcd(a, b) == 1:
            assert oracle.rad(a * b) == oracle.rad(a) * oracle.rad(b)


def test_radicals_range_matches_pointwise():
    lo = 2**36 - 50
    r = oracle.radicals(lo, lo + 100)
    assert [int(v) for v in r] == [oracle.rad(x) for x in range(lo, lo + 100)]


def test_bad_arguments():
    with pytest.raises(ValueError):
        oracle.rad(0)
    with pytest.raises(ValueError):
        oracle.radicals(0, 10)
    assert oracle.search_range(5, 5) == []
    assert oracle.search(1) == []


# --- Erdős's third condition (abstract, introduction) -------------------------------------

def test_no_listed_first_kind_pair_meets_the_third_condition():
    """The paper's argument for the family: m + 2 = 2^(k+1) is a power of two while
    n + 2 = (2^k - 1) 2^(k+2) + 2 is 2 mod 4, so rad(m+2) = 2 != rad(n+2); and for the
    exceptional pair m + 2 = 77 = 7 * 11 while n + 2 = 1217 is prime.  Checked with the
    oracle's radicals for every first-kind pair with n < 1.4e12."""
    for m, n, kind in theorem1_pairs(THEOREM1_LIMIT - 1):
        if kind != 1:
            continue
        if (m, n) == (75, 1215):
            assert oracle.rad(m + 2) == 77 and oracle.rad(n + 2) == 1217
        else:
            k = (m + 2).bit_length() - 1
            assert m + 2 == 2 ** k and (n + 2) % 4 == 2
            assert oracle.rad(m + 2) == 2 and oracle.rad(n + 2) != 2
        assert oracle.rad(m + 2) != oracle.rad(n + 2)


def _bruteforce_third(N, d, r):
    """First-kind pairs m < n <= N (Section 1's definition) that also have
    rad(m + d) = rad(n + d), straight from the definition over radicals r."""
    out = []
    for m in range(1, N):
        n = np.arange(m + 1, N + 1)
        first = (r[n] == r[m]) & (r[n + 1] == r[m + 1]) & (r[n + d] == r[m + d])
        out += [(m, int(k)) for k in n[first]]
    return out


@pytest.mark.parametrize("d", [0, 1, 2, 3, 4, 5, 6, 8])
def test_third_condition_bruteforce(d):
    """Kinds bit 4 with offset d against the definition for every m < n <= 2^12
    (radicals from a smallest-prime-factor sieve).  d = 2 is Erdos's question: no
    pair; d = 0 and d = 1 repeat the first two conditions: every first-kind pair."""
    N = 2**12
    r = spf_radicals(N + 9)
    want = _bruteforce_third(N, d, r)
    got = oracle.search(N, kinds=4, third_offset=d)
    assert got == [(m, n, 5) for m, n in want]
    firsts = [(m, n) for m, n, k in theorem1_pairs(N) if k == 1]
    if d in (0, 1):
        assert want == firsts
    if d == 2:
        assert want == []
    # The full mask: pairs meeting the third condition carry kind 5, the rest keep 1 or 2.
    full = oracle.search(N, kinds=7, third_offset=d)
    marked = set(want)
    assert full == [(m, n, 5 if (m, n) in marked else k) for m, n, k in theorem1_pairs(N)]
    assert oracle.search(N, kinds=5, third_offset=d) == [p for p in full if p[2] in (1, 5)]
    assert oracle.search(N, kinds=6, third_offset=d) == [p for p in full if p[2] in (2, 5)]


def test_third_condition_nontrivial_offset():
    """Offset 4 marks (2, 8) only (rad 6 = rad 12) among the pairs up to 2^12, so the
    marking is not all-or-nothing; worked out by hand from the factorizations."""
    assert oracle.search(2**12, kinds=4, third_offset=4) == [(2, 8, 5)]
    assert oracle.rad(6) == oracle.rad(12) == 6


def test_third_condition_range_and_default():
    """Range form and the default offset 2 (Erdos's question): nothing up to 2^20."""
    assert oracle.search(2**20, kinds=4) == []
    assert oracle.search(2**20, kinds=7) == oracle.search(2**20, kinds=3)
    assert oracle.search_range(3, 4000, kinds=4, third_offset=1) == [
        (m, n, 5) for m, n, k in theorem1_pairs(4000) if k == 1 and m >= 3]
