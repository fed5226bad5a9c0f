"""The member test that lets the sieve drop x which cannot belong to any pair.

The kernels keep x for the join only if it may be a member of a pair (m, n)
with m < n < b (both kinds):
  * the larger member n has n and n + 1 non-squarefree, except n = 3 in (2, 3);
  * if the smaller member m is squarefree, then n or n + 1 is m * t with
    t >= max(2, rad(m + 1) - 1), so m * t <= b; likewise for m + 1 with rad(m).
These tests check that rule, restated here on its own, against every pair the
paper lists (Theorem 1, Tables 1 and 2, n < 1.4e12, radicals taken from the
printed factorizations) and against every pair the oracle finds up to 2^20,
each time with the tightest bound b = n + 1.  They also check, by brute
force over all m < n <= 2^12, the facts the rule rests on.
"""
import math

import numpy as np
import pytest

import oracle
from paper_facts import golden, load_table


def may_pair(x, r0, r1, b):
    if x <= 3:
        return True
    if r0 == x and x * max(2, r1 - 1) > b:
        return False
    if r1 == x + 1 and (x + 1) * max(2, r0 - 1) > b:
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
    unless (m, n) = (2, 3); a squarefree m has n or n+1 = m*t with t-1 (first kind) or
    t+1 (second kind) divisible by rad(m+1); the same for a squarefree m+1."""
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
                first = r[m] == r[n]
                if (m, n) != (2, 3):
                    assert r[n] < n and r[n + 1] < n + 1
                if r[m] == m:
                    big = n if first else n + 1
                    assert big % m == 0 and big // m >= 2
                    t = big // m
                    assert (t - 1 if first else t + 1) % r[m + 1] == 0
                if r[m + 1] == m + 1 and (m, n) != (2, 3):
                    big = n + 1 if first else n
                    assert big % (m + 1) == 0 and big // (m + 1) >= 2
                    t = big // (m + 1)
                    assert (t - 1 if first else t + 1) % r[m] == 0
                assert may_pair(m, r[m], r[m + 1], n + 1)
                assert may_pair(n, r[n], r[n + 1], n + 1)
    assert seen == len([p for p in oracle.search(N)])


def test_rule_keeps_about_the_non_squarefree_neighbours():
    """The rule is worth having: at b = 2^20 + 1 it keeps 10.9% of x in [1, 2^20], barely
    above the 10.68% whose x and x+1 are both non-squarefree."""
    N = 2**20
    r = oracle.radicals(1, N + 2).astype(np.int64)
    kept = nn = 0
    for x in range(1, N + 1):
        r0, r1 = int(r[x - 1]), int(r[x])
        kept += may_pair(x, r0, r1, N + 1)
        nn += r0 != x and r1 != x + 1
    assert nn <= kept < 0.11 * N
    assert 0.106 * N < nn < 0.108 * N
