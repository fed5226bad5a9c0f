"""The member test that lets the sieve drop x which cannot belong to any pair.

The kernels keep x for the join only if it may be a member of a pair (m, n)
with m < n < b (both kinds):
  * the larger member n has n and n + 1 non-squarefree, except n = 3 in (2, 3);
  * if the smaller member m is squarefree, then m * spf(m) <= b, and likewise
    for m + 1 (spf = smallest prime factor, bounded below by the first of
    2, 3, 5, 7 dividing it, else 11).
These tests check that rule, restated here on its own, against every pair the
paper lists (Theorem 1, Tables 1 and 2, n < 1.4e12, radicals taken from the
printed factorizations) and against every pair the oracle finds up to 2^20,
each time with the tightest bound b = n + 1.  They also check, by brute
force over all m < n <= 2^12, the two facts the rule rests on.
"""
import math

import numpy as np
import pytest

import oracle
from paper_facts import golden, load_table


def spf_floor(y):
    for p in (2, 3, 5, 7):
        if y % p == 0:
            return p
    return 11


def may_pair(x, r0, r1, b):
    if x <= 3:
        return True
    if r0 == x and x * spf_floor(x) > b:
        return False
    if r1 == x + 1 and (x + 1) * spf_floor(x + 1) > b:
        return False
    return True


def _rad_from(fact):
    return math.prod(fact.keys())


@pytest.mark.parametrize("name,kind", [("paper_table1_first_kind.txt", 1), ("paper_table2_second_kind.txt", 2)])
def test_every_listed_pair_survives(name, kind):
    rows = load_table(golden(name))
    assert rows
    for m, n, facts in rows:
        if kind == 1:
            rm, rn, rm1, rn1 = (_rad_from(f) for f in facts)
        else:
            rm, rn1, rm1, rn = (_rad_from(f) for f in facts)
        b = n + 1
        assert may_pair(m, rm, rm1, b), (m, n)
        assert may_pair(n, rn, rn1, b), (m, n)


def test_every_oracle_pair_survives():
    pairs = oracle.search(2**20)
    assert len(pairs) == 21
    for m, n, _ in pairs:
        b = n + 1
        assert may_pair(m, oracle.rad(m), oracle.rad(m + 1), b)
        assert may_pair(n, oracle.rad(n), oracle.rad(n + 1), b)


def test_rule_facts_brute_force():
    """All m < n <= 2^12 with {rad m, rad m+1} = {rad n, rad n+1}: n, n+1 non-squarefree
    unless (m, n) = (2, 3); a squarefree m (or m+1) has n or n+1 = m * t (or (m+1) * t),
    t >= spf, with t = 1 only for (2, 3)."""
    N = 2**12
    r = [0] + [int(v) for v in oracle.radicals(1, N + 2)]
    groups = {}
    for x in range(1, N + 1):
        groups.setdefault(frozenset((r[x], r[x + 1])), []).append(x)
    seen = 0
    for xs in groups.values():
        for i, m in enumerate(xs):
            for n in xs[i + 1:]:
                seen += 1
                if (m, n) != (2, 3):
                    assert r[n] < n and r[n + 1] < n + 1
                assert may_pair(m, r[m], r[m + 1], n + 1)
                assert may_pair(n, r[n], r[n + 1], n + 1)
    assert seen == len([p for p in oracle.search(N)])


def test_rule_drops_most_integers():
    """The rule is worth having: at b = 2^20 + 1 it keeps under 30% of x in [1, 2^20]."""
    N = 2**20
    r = oracle.radicals(1, N + 2).astype(np.int64)
    kept = sum(1 for x in range(1, N + 1) if may_pair(x, int(r[x - 1]), int(r[x]), N + 1))
    assert 0.25 * N < kept < 0.30 * N
