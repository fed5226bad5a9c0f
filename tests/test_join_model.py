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
