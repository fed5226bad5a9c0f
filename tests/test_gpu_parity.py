"""GPU parity: the HIP path (through the C-ABI) against the oracle and the paper's pins.

Radicals are compared element by element with trial division; pair lists are
compared bit-exactly as sorted lists.  Full-size cases compare the pair list with
Theorem 1 (complete up to 1.4e12) and radicals sampled one by one.
"""
import math
import sys

import numpy as np
import pytest

import join_model
import oracle
from paper_facts import theorem1_pairs

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_2506_01099_amd import Benelux

    c = Benelux(device=0)
    yield c
    c.close()


def squarefree_count(n):
    r = math.isqrt(n)
    mu = np.ones(r + 1, dtype=np.int64)
    comp = np.zeros(r + 1, dtype=bool)
    for p in range(2, r + 1):
        if not comp[p]:
            comp[2 * p::p] = True
            mu[p::p] *= -1
            mu[p * p::p * p] = 0
    return int(sum(int(mu[d]) * (n // (d * d)) for d in range(1, r + 1)))


def member_count(N):
    """#{1 <= x <= N : x may be a member of a pair with n <= N}, by the rule of
    tests/test_member_test.py, vectorised over the oracle's radicals (exact in
    int64 for N <= 2^30)."""
    assert N <= 1 << 30
    r = oracle.radicals(1, N + 2).astype(np.int64)
    x = np.arange(1, N + 1, dtype=np.int64)
    return int(np.count_nonzero(join_model.kept(x, r[:N], r[1:N + 1], N + 1)))


def device_squarefree_count(ctx, N, chunk=1 << 28):
    """#{x <= N : rad(x) = x} from the library's radicals, sieved in chunks on the device."""
    import torch

    count = 0
    buf = torch.empty(chunk, dtype=torch.int64, device="cuda")
    xs = torch.empty(chunk, dtype=torch.int64, device="cuda")
    base = torch.arange(chunk, dtype=torch.int64, device="cuda")
    for lo in range(1, N + 1, chunk):
        hi = min(N + 1, lo + chunk)
        n = hi - lo
        ctx.radical_segment_dev(lo, hi, buf)
        torch.add(base, lo, out=xs)
        count += int((buf[:n] == xs[:n]).sum().item())
    return count


# --- radicals -----------------------------------------------------------------------

@pytest.mark.parametrize("lo,hi", [
    (1, 2), (1, 3), (5, 5), (1, 4097), (1, 4098), (1, (1 << 16) + 3), (1, (1 << 17) + 1),
    ((1 << 17) - 7, (1 << 17) + 9), ((1 << 20) - 100, (1 << 20) + 300),
    ((1 << 32) - 3000, (1 << 32) + 1000),
    ((1 << 36) - 300000, (1 << 36) + 300000),  # two segments of 2^18 and many tiles
    ((1 << 40) - 5000, (1 << 40) + 5000),
    ((1 << 42) - 20001, (1 << 42) - 1),
])
def test_radicals_match_oracle(ctx, lo, hi):
    say(f"radicals [{lo}, {hi})")
    got = ctx.radical_segment(lo, hi)
    want = oracle.radicals(lo, hi) if hi > lo else np.empty(0, dtype=np.uint64)
    assert got.dtype == np.uint64 and got.size == hi - lo
    assert np.array_equal(got, want)


def test_radicals_special_values(ctx):
    """Prime powers near the top of the table, 3^26, 2^41, p^2 for the largest table prime."""
    lim = math.isqrt((1 << 42) - 1)
    p = lim
    while any(p % d == 0 for d in range(2, math.isqrt(p) + 1)):
        p -= 1
    for v in [p * p, 3**26, 2**41, 5**17, 7**14, 2**41 - 1, p * (p - 2)]:
        lo = max(1, v - 300)
        hi = min((1 << 42) - 1, v + 300)
        say(f"radicals around {v}")
        got = ctx.radical_segment(lo, hi)
        assert np.array_equal(got, oracle.radicals(lo, hi)), v


def test_radicals_squarefree_count_2_24(ctx):
    N = 1 << 24
    r = ctx.radical_segment(1, N + 1)
    x = np.arange(1, N + 1, dtype=np.uint64)
    assert int(np.count_nonzero(r == x)) == squarefree_count(N)


def test_radicals_squarefree_count_2_30_on_device(ctx):
    """Aggregate pin at a size trial division cannot reach: #{x <= N : rad(x) = x} (Moebius)."""
    assert device_squarefree_count(ctx, 1 << 30, chunk=1 << 27) == squarefree_count(1 << 30)


@pytest.mark.parametrize("log2n,want", [(32, 2611027094), (36, 41776432306)])
def test_radicals_squarefree_count_full_size(ctx, log2n, want):
    """The sieve in aggregate over the whole headline ranges: the squarefree count up to
    2^32 and 2^36 equals the Moebius sum (value checked against the formula here too)."""
    N = 1 << log2n
    assert squarefree_count(N) == want
    say(f"squarefree count to 2^{log2n} on the device")
    assert device_squarefree_count(ctx, N) == want


def test_radicals_sampled_at_scale(ctx):
    rng = np.random.default_rng(36)
    for mag in (32, 36, 40, 41):
        xs = rng.integers(1 << (mag - 1), 1 << mag, size=12)
        for x in xs:
            x = int(x)
            got = ctx.radical_segment(x, x + 2)
            assert [int(v) for v in got] == [oracle.rad(x), oracle.rad(x + 1)], x


def test_radical_segment_dev_matches_host(ctx):
    import torch

    lo, hi = (1 << 33) + 17, (1 << 33) + 17 + 300000
    t = torch.empty(hi - lo, dtype=torch.int64, device="cuda")
    ctx.radical_segment_dev(lo, hi, t)
    torch.cuda.synchronize()
    assert np.array_equal(t.cpu().numpy().astype(np.uint64), ctx.radical_segment(lo, hi))


# --- searches -------------------------------------------------------------------------

@pytest.mark.parametrize("N", [1, 2, 3, 8, 100, 1215, 4096, 4374, 1 << 16, 1 << 20])
def test_search_matches_oracle(ctx, N):
    say(f"search N={N}")
    assert ctx.search(N) == oracle.search(N)


def test_search_2_24_matches_oracle(ctx):
    N = 1 << 24
    got = ctx.search(N)
    assert got == oracle.search(N)
    st = ctx.stats()
    assert st["integers"] == N
    assert st["entries"] == st["joined"] == member_count(N)


@pytest.mark.parametrize("N", [1 << 20, 1 << 24])
def test_fingerprint_collisions_are_dropped(ctx, N):
    """With 23 of the 53 fingerprint bits kept, different sets share fingerprints in
    the join; the verification recomputes the radicals and drops every such pair."""
    ctx.set_option("fp_bits", 12)
    try:
        got = ctx.search(N)
        st = ctx.stats()
        batch = ctx.search_batch(np.array([1, 70], dtype=np.uint64), np.array([N, 1300], dtype=np.uint64))
    finally:
        ctx.set_option("fp_bits", 0)
    assert got == oracle.search(N)
    assert st["candidates"] > st["pairs"] == len(got)
    assert batch == [oracle.search_range(1, N), oracle.search_range(70, 1300)]


@pytest.mark.parametrize("N", [1 << 20, 1 << 24])
def test_sort_join_matches_oracle(ctx, N):
    """The sort-join ablation (Algorithm 2 per partition, all pairs of a run) gives the
    same lists as the hash join and the oracle."""
    ctx.set_option("join", 1)
    try:
        got = ctx.search(N)
    finally:
        ctx.set_option("join", 0)
    assert got == oracle.search(N)


@pytest.mark.parametrize("N,log2s", [(1 << 20, 14), (1 << 24, 18), ((1 << 20) + 12345, 16)])
def test_paper_schedule_matches_oracle(ctx, N, log2s):
    """Algorithm 3's chunk schedule (chunks of s values overlapping by one, a table of
    4s slots per chunk, every earlier chunk sieved again and probed) finds the same
    pairs as the oracle, including pairs inside one chunk and across chunks."""
    ctx.set_option("schedule", 1)
    ctx.set_option("a3_chunk_log2", log2s)
    try:
        got = ctx.search(N)
        st = ctx.stats()
        rng = ctx.search_range(70, N // 3, 3)
        first = ctx.search(N, 1)
    finally:
        ctx.set_option("schedule", 0)
        ctx.set_option("a3_chunk_log2", 0)
    assert got == oracle.search(N)
    assert rng == oracle.search_range(70, N // 3, 3)
    assert first == [p for p in got if p[2] == 1]
    assert st["passes"] == -(-N // ((1 << log2s) - 1))  # one pass per chunk
    assert st["candidates"] >= len(got)


def test_paper_schedule_2_32_theorem1(ctx):
    """The paper's own configuration (chunks of 2^27, tables of 2^29 slots) up to 2^32."""
    say("Algorithm 3 schedule up to 2^32")
    ctx.set_option("schedule", 1)
    try:
        got = ctx.search(1 << 32)
        st = ctx.stats()
        with pytest.raises(Exception):
            ctx.search_batch(np.array([1], dtype=np.uint64), np.array([100], dtype=np.uint64))
    finally:
        ctx.set_option("schedule", 0)
    assert got == theorem1_pairs(1 << 32)
    assert st["passes"] == -(-(1 << 32) // ((1 << 27) - 1))  # 33 chunks of 2^27 - 1 new values
    say(f"  {st['total_ms']:.0f} ms")


@pytest.mark.parametrize("N,prune", [(1 << 16, 1), (1 << 20, 1), ((1 << 20) + 12345, 1), (1 << 20, 0), (4374, 1)])
def test_whole_range_sort_matches_oracle(ctx, N, prune):
    """Algorithm 2: the whole range's list sorted by key, every run of equal keys reported."""
    say(f"Algorithm 2 at N={N}, member test {prune}")
    ctx.set_option("schedule", 2)
    ctx.set_option("prune", prune)
    try:
        got = ctx.search(N)
        st = ctx.stats()
        rng = ctx.search_range(35, 4375)
    finally:
        ctx.set_option("schedule", 0)
        ctx.set_option("prune", 1)
    assert got == oracle.search(N)
    assert rng == oracle.search_range(35, 4375)
    assert st["passes"] == 7  # 8-bit digits over the 53-bit fingerprint
    if not prune:
        assert st["entries"] == N


def test_whole_range_sort_candidates_exact(ctx):
    """Every pair of equal (masked) fingerprints in the sorted list is a candidate: with
    11 + 13 fingerprint bits kept the count is known exactly from the oracle's radicals."""
    N, fp_bits = 1 << 24, 13
    ctx.set_option("schedule", 2)
    ctx.set_option("fp_bits", fp_bits)
    try:
        got = ctx.search(N)
        st = ctx.stats()
    finally:
        ctx.set_option("schedule", 0)
        ctx.set_option("fp_bits", 0)
    assert got == oracle.search(N)
    keys, n_kept = join_model.group_keys(oracle.radicals(1, N + 2), 1, N + 1, 0, 0, 1, fp_bits)
    want = join_model.candidates(keys)
    assert st["entries"] == n_kept
    assert 10**4 < want < 10**6
    assert st["candidates"] == want
    assert st["candidates"] == st["pairs"] + st["false_candidates"]


def test_whole_range_sort_2_32_theorem1(ctx):
    say("Algorithm 2 up to 2^32")
    ctx.set_option("schedule", 2)
    try:
        got = ctx.search(1 << 32)
        st = ctx.stats()
    finally:
        ctx.set_option("schedule", 0)
    assert got == theorem1_pairs(1 << 32)
    say(f"  {st['total_ms']:.0f} ms, {st['entries']} entries")


def test_sort_join_chunks_collisions_and_batch(ctx):
    """Partitions of several LDS chunks (one first- and one second-level bit), colliding
    fingerprints and a batch, all through the sort join."""
    from paper_2506_01099_amd.inputs import planted_queries

    ctx.set_option("join", 1)
    try:
        ctx.set_option("b1_bits", 1)
        ctx.set_option("b2_bits", 1)
        try:
            chunked = ctx.search(1 << 18)
        finally:
            ctx.set_option("b1_bits", 0)
            ctx.set_option("b2_bits", 0)
        ctx.set_option("fp_bits", 12)
        try:
            colliding = ctx.search(1 << 22)
            st = ctx.stats()
        finally:
            ctx.set_option("fp_bits", 0)
        a, b = planted_queries()
        batch = ctx.search_batch(a, b)
        full = ctx.search(1 << 28)
    finally:
        ctx.set_option("join", 0)
    assert chunked == oracle.search(1 << 18)
    assert colliding == oracle.search(1 << 22) and st["candidates"] > st["pairs"]
    assert batch == [oracle.search_range(int(x), int(y)) for x, y in zip(a, b)]
    assert full == theorem1_pairs(1 << 28)


def test_member_test_off_same_pairs(ctx):
    """Without the member test every x becomes an entry; the pairs are the same."""
    N = 1 << 22
    ctx.set_option("prune", 0)
    try:
        got = ctx.search(N)
        st = ctx.stats()
        batch = ctx.search_batch(np.array([1, 1000, 30, 4000000], dtype=np.uint64),
                                 np.array([N + 1, 5000, 1300, N + 1], dtype=np.uint64))
    finally:
        ctx.set_option("prune", 1)
    assert got == oracle.search(N)
    assert st["entries"] == N and st["integers"] == N
    assert batch == ctx.search_batch(np.array([1, 1000, 30, 4000000], dtype=np.uint64),
                                     np.array([N + 1, 5000, 1300, N + 1], dtype=np.uint64))
    assert batch[0] == oracle.search(N) and batch[2] == oracle.search_range(30, 1300)


@pytest.mark.parametrize("a,b", [(1, 9), (2, 9), (3, 9), (35, 4375), (36, 4375), (35, 4374), (126, 16129),
                                 (127, 16129), (1000, (1 << 20) + 1), (70, 1300), ((1 << 20) - 5, (1 << 20) + 5)])
def test_search_range_matches_oracle(ctx, a, b):
    assert ctx.search_range(a, b) == oracle.search_range(a, b)


@pytest.mark.parametrize("kinds", [1, 2, 3])
def test_kinds_filter(ctx, kinds):
    assert ctx.search(1 << 20, kinds) == oracle.search(1 << 20, kinds)


def test_third_condition(ctx):
    """Erdős's third condition rad(m+2) = rad(n+2): no pair up to 2^28 meets it (none is
    known), so the lists with the bit equal the oracle's and the bit alone gives nothing.
    The branch that marks a pair (kind 5) has no known input: parity unpinned."""
    N = 1 << 28
    assert ctx.search(N, 7) == ctx.search(N, 3) == theorem1_pairs(N)
    assert ctx.search(N, 4) == []
    assert ctx.search(1 << 20, 5) == oracle.search(1 << 20, 1)
    got = ctx.search_batch(np.array([1, 70], dtype=np.uint64), np.array([1 << 20, 1300], dtype=np.uint64), 7)
    assert got == [oracle.search_range(1, 1 << 20), oracle.search_range(70, 1300)]


def _serve(ctx, reqs):
    import time

    from paper_2506_01099_amd import Server

    srv = Server(ctx, budget_bytes=8 << 30, max_inflight=2)
    try:
        tickets = [srv.submit(a, b, k) for a, b, k in reqs]
        deadline = time.time() + 60
        results = {}
        while len(results) < len(tickets) and time.time() < deadline:
            for t in tickets:
                if t not in results and srv.poll(t):
                    results[t] = srv.take(t)[0]
            time.sleep(0.001)
    finally:
        srv.stop()
    assert len(results) == len(tickets)
    return [results[t] for t in tickets]


@pytest.mark.parametrize("d", [1, 4, 6])
def test_third_condition_marks_pairs(ctx, d):
    """The marking branch of the third condition, made reachable by moving its offset:
    with rad(m + d) = rad(n + d) in place of d = 2, d = 1 marks every first-kind pair
    (it repeats the second condition), d = 4 marks only (2, 8) and d = 6 only (6, 48).
    Plain, batched and served results equal the oracle run with the same offset."""
    from paper_2506_01099_amd.inputs import planted_queries

    N = 1 << 20
    a, b = planted_queries()
    ctx.set_option("third_offset", d)
    try:
        plain = {k: ctx.search(N, k) for k in (4, 5, 7)}
        batch = ctx.search_batch(a, b, 7)
        served = _serve(ctx, [(1, N + 1, 4), (1, N + 1, 7), (30, 100000, 5), (2, 9, 6)])
    finally:
        ctx.set_option("third_offset", 2)
    for k in (4, 5, 7):
        assert plain[k] == oracle.search(N, k, third_offset=d), k
    marked = [p for p in plain[7] if p[2] == 5]
    assert marked and marked == oracle.search(N, 4, third_offset=d)
    if d == 1:
        assert [(m, n) for m, n, _ in marked] == [(m, n) for m, n, _ in oracle.search(N, 1)]
    assert batch == [oracle.search_range(int(x), int(y), 7, third_offset=d) for x, y in zip(a, b)]
    assert served == [oracle.search_range(1, N + 1, 4, third_offset=d), oracle.search_range(1, N + 1, 7, third_offset=d),
                      oracle.search_range(30, 100000, 5, third_offset=d), oracle.search_range(2, 9, 6, third_offset=d)]


def _expected_candidates(rad, a, b, grp, st, passes, fp_bits):
    keys, n_kept = join_model.group_keys(rad, a, b, grp, st["b1_bits"], passes, fp_bits)
    return join_model.candidates(keys), n_kept


@pytest.mark.parametrize("join", [0, 1])
@pytest.mark.parametrize("passes", [0, 3])
def test_join_candidates_exact_2_24(ctx, join, passes):
    """Join completeness, counted exactly: with 13 + 11 fingerprint bits kept, about 1e5
    different sets share fingerprints, and the join must report every pair of equal
    (pass, bucket, fingerprint) among the entries that pass the member test -- the
    insert/probe steps of Algorithm 3 report every earlier equal key on a chain.  The
    expected count comes from the oracle's radicals and the hash restated in numpy."""
    N, fp_bits = 1 << 24, 13
    ctx.set_option("fp_bits", fp_bits)
    ctx.set_option("passes", passes)
    ctx.set_option("join", join)
    try:
        got = ctx.search(N)
        st = ctx.stats()
    finally:
        ctx.set_option("fp_bits", 0)
        ctx.set_option("passes", 0)
        ctx.set_option("join", 0)
    assert got == oracle.search(N)
    assert st["retries"] == 0
    rad = oracle.radicals(1, N + 2)
    want, n_kept = _expected_candidates(rad, 1, N + 1, 0, st, max(1, passes), fp_bits)
    assert st["entries"] == st["joined"] == n_kept
    assert 10**4 < want < 10**6
    assert st["candidates"] == want
    assert st["candidates"] == st["pairs"] + st["false_candidates"]


@pytest.fixture(scope="module")
def rad_2_28(ctx):
    """rad(x) for x in [1, 2^28 + 1] from the library (pinned element by element and in
    aggregate by other tests), on the host."""
    import torch

    N = 1 << 28
    t = torch.empty(N + 1, dtype=torch.int64, device="cuda")
    ctx.radical_segment_dev(1, N + 2, t)
    torch.cuda.synchronize()
    rad = t.cpu().numpy()
    del t
    torch.cuda.empty_cache()
    return rad


@pytest.mark.parametrize("join,passes", [(0, 0), (0, 2), (1, 0)])
def test_join_candidates_exact_2_28(ctx, rad_2_28, join, passes):
    """The same exact candidate count at 2^28 (four first-level buckets, forced: the plan
    takes one bucket once a pass holds fewer than about 1.5e7 entries), from the
    library's radicals."""
    N, fp_bits = 1 << 28, 19
    rad = rad_2_28
    say(f"exact candidates at 2^28, join={join}, passes={passes}")
    ctx.set_option("fp_bits", fp_bits)
    ctx.set_option("passes", passes)
    ctx.set_option("join", join)
    ctx.set_option("b1_bits", 2)
    try:
        got = ctx.search(N)
        st = ctx.stats()
    finally:
        ctx.set_option("fp_bits", 0)
        ctx.set_option("passes", 0)
        ctx.set_option("join", 0)
        ctx.set_option("b1_bits", 0)
    assert got == theorem1_pairs(N)
    assert st["retries"] == 0 and st["b1_bits"] == 2
    want, n_kept = _expected_candidates(rad, 1, N + 1, 0, st, max(1, passes), fp_bits)
    assert st["entries"] == st["joined"] == n_kept
    assert 10**4 < want < 10**6
    assert st["candidates"] == want


def test_join_candidates_exact_batched(ctx):
    """Batched calls join each query with itself only: the expected count groups by query too."""
    qs = [(1, 1 << 22), (1 << 22, 3 << 21), (5 << 30, (5 << 30) + (1 << 22))]
    fp_bits = 12
    ctx.set_option("fp_bits", fp_bits)
    try:
        got = ctx.search_batch(np.array([q[0] for q in qs], dtype=np.uint64),
                               np.array([q[1] for q in qs], dtype=np.uint64))
        st = ctx.stats()
    finally:
        ctx.set_option("fp_bits", 0)
    want = 0
    for i, (a, b) in enumerate(qs):
        assert got[i] == oracle.search_range(a, b)
        keys, _ = join_model.group_keys(oracle.radicals(a, b + 1), a, b, i, st["b1_bits"], 1, fp_bits)
        want += join_model.candidates(keys)
    assert st["retries"] == 0 and want > 10**3
    assert st["candidates"] == want


def test_compact_words_match_oracle(ctx):
    """The second partition level as 8-byte words (first-level index, low fingerprint
    bits) and as 12-byte entries give the oracle's lists."""
    from paper_2506_01099_amd.inputs import planted_queries

    a, b = planted_queries()
    for compact, nbytes, nbytes_batch in ((1, 8, 8), (0, 12, 12)):
        ctx.set_option("compact", compact)
        try:
            for N in (1 << 20, (1 << 24) + 77):
                assert ctx.search(N) == oracle.search(N), (compact, N)
                assert ctx.stats()["l2_entry_bytes"] == nbytes
            got = ctx.search_batch(a, b)
            assert ctx.stats()["l2_entry_bytes"] == nbytes_batch
        finally:
            ctx.set_option("compact", 1)
        for i in range(a.size):
            assert got[i] == oracle.search_range(int(a[i]), int(b[i]))


@pytest.mark.parametrize("keep", [14, 16])
def test_compact_candidates_exact_2_24(ctx, keep):
    """Join completeness on compact words, counted exactly: with only `keep` low
    fingerprint bits in a word, different sets meet, and every pair of equal (bucket,
    partition, kept bits) must be found and read back; only equal whole fingerprints
    become candidates."""
    N = 1 << 24
    ctx.set_option("compact", 1)
    ctx.set_option("compact_fp_bits", keep)
    try:
        got = ctx.search(N)
        st = ctx.stats()
    finally:
        ctx.set_option("compact_fp_bits", 0)
        ctx.set_option("compact", 1)
    assert got == oracle.search(N)
    assert st["l2_entry_bytes"] == 8 and st["retries"] == 0
    keys, n_kept = join_model.compact_keys(oracle.radicals(1, N + 2), 1, N + 1, 0, st["b1_bits"], st["b2_bits"], keep)
    want = join_model.candidates(keys)
    assert st["entries"] == st["joined"] == n_kept
    assert 10**3 < want < 10**6
    assert st["word_matches"] == want
    assert st["candidates"] == st["pairs"] and st["false_candidates"] == 0


def test_compact_candidates_exact_2_28(ctx, rad_2_28):
    """The same at 2^28 (four first-level buckets, forced), from the library's radicals."""
    N, keep = 1 << 28, 18
    ctx.set_option("compact", 1)
    ctx.set_option("compact_fp_bits", keep)
    ctx.set_option("b1_bits", 2)
    try:
        got = ctx.search(N)
        st = ctx.stats()
    finally:
        ctx.set_option("b1_bits", 0)
        ctx.set_option("compact_fp_bits", 0)
        ctx.set_option("compact", 1)
    assert got == theorem1_pairs(N)
    assert st["l2_entry_bytes"] == 8 and st["b1_bits"] == 2
    keys, n_kept = join_model.compact_keys(rad_2_28, 1, N + 1, 0, st["b1_bits"], st["b2_bits"], keep)
    want = join_model.candidates(keys)
    assert st["entries"] == st["joined"] == n_kept
    assert 10**3 < want < 10**6
    assert st["word_matches"] == want
    assert st["candidates"] == st["pairs"] and st["false_candidates"] == 0


def test_compact_candidates_exact_batched(ctx):
    """Batched compact words: the words do not hold the query, so kept bits also meet
    across queries; the join reads such matches back and drops them."""
    qs = [(1, 1 << 22), (1 << 22, 3 << 21), (5 << 30, (5 << 30) + (1 << 22))]
    keep = 14
    ctx.set_option("compact", 1)
    ctx.set_option("compact_fp_bits", keep)
    try:
        got = ctx.search_batch(np.array([q[0] for q in qs], dtype=np.uint64),
                               np.array([q[1] for q in qs], dtype=np.uint64))
        st = ctx.stats()
    finally:
        ctx.set_option("compact_fp_bits", 0)
        ctx.set_option("compact", 1)
    allkeys = []
    for i, (a, b) in enumerate(qs):
        assert got[i] == oracle.search_range(a, b)
        keys, _ = join_model.compact_keys(oracle.radicals(a, b + 1), a, b, i, st["b1_bits"], st["b2_bits"], keep)
        allkeys.append(keys)
    want = join_model.candidates(np.concatenate(allkeys))
    assert st["l2_entry_bytes"] == 8 and st["retries"] == 0 and want > 10**3
    assert st["word_matches"] == want
    assert st["candidates"] == st["pairs"] and st["false_candidates"] == 0


@pytest.mark.parametrize("passes", [1, 2, 3, 5, 7, 16, 64])
def test_pass_count_invariance(ctx, passes):
    ctx.set_option("passes", passes)
    try:
        got = ctx.search(1 << 20)
        st = ctx.stats()
    finally:
        ctx.set_option("passes", 0)
    assert got == oracle.search(1 << 20)
    assert st["passes"] >= passes and st["entries"] == st["joined"] == member_count(1 << 20)


@pytest.mark.parametrize("b1,b2", [(1, 1), (2, 3), (10, 1), (3, 11), (0, 0)])
def test_partition_shape_invariance(ctx, b1, b2):
    """Large partitions take the chunked LDS join; many small ones the single-chunk path."""
    ctx.set_option("b1_bits", b1)
    ctx.set_option("b2_bits", b2)
    try:
        got = ctx.search(1 << 18)
    finally:
        ctx.set_option("b1_bits", 0)
        ctx.set_option("b2_bits", 0)
    assert got == oracle.search(1 << 18)


@pytest.mark.parametrize("group", [1, 2, 4, 8])
def test_group_invariance(ctx, group):
    """Eight first-level buckets, partitioned G at a time by XCD-aware workgroups."""
    ctx.set_option("group", group)
    ctx.set_option("b1_bits", 3)
    try:
        got = ctx.search(1 << 22)
        st = ctx.stats()
    finally:
        ctx.set_option("group", 0)
        ctx.set_option("b1_bits", 0)
    assert st["b1_bits"] == 3 and st["launches"]["partition"] == 8 // group
    assert got == theorem1_pairs(1 << 22)
    assert st["entries"] == st["joined"]


@pytest.mark.parametrize("seg", [8192, 16384, 1 << 17, 1 << 20])
def test_segment_length_invariance(ctx, seg):
    ctx.set_option("seg_len", seg)
    try:
        got = ctx.search(1 << 20)
        rad = ctx.radical_segment((1 << 36) - 9000, (1 << 36) + 9000)
    finally:
        ctx.set_option("seg_len", 0)
    assert got == oracle.search(1 << 20)
    assert np.array_equal(rad, oracle.radicals((1 << 36) - 9000, (1 << 36) + 9000))


def test_repeat_determinism(ctx):
    a = ctx.search(1 << 22)
    b = ctx.search(1 << 22)
    assert a == b == theorem1_pairs(1 << 22)


def test_invariant_larger_member_non_squarefree(ctx):
    for m, n, _ in ctx.search(1 << 26):
        if (m, n) == (2, 3):
            continue
        r = ctx.radical_segment(n, n + 2)
        assert int(r[0]) < n and int(r[1]) < n + 1


# --- full sizes -----------------------------------------------------------------------

def test_search_2_28_theorem1(ctx):
    got = ctx.search(1 << 28)
    assert got == theorem1_pairs(1 << 28)
    assert len(got) == 29


def test_search_2_32_theorem1(ctx):
    say("search N=2^32 (one pass)")
    got = ctx.search(1 << 32)
    st = ctx.stats()
    assert got == theorem1_pairs(1 << 32)
    assert len(got) == 33
    assert st["integers"] == 1 << 32 and 0.106 * (1 << 32) < st["entries"] < 0.108 * (1 << 32)
    assert st["joined"] == st["entries"]
    assert st["retries"] == 0


def test_search_2_36_theorem1(ctx):
    say("search N=2^36 (hash-partitioned passes)")
    got = ctx.search(1 << 36)
    st = ctx.stats()
    assert got == theorem1_pairs(1 << 36)
    assert len(got) == 37
    assert st["integers"] == 1 << 36 and 0.106 * (1 << 36) < st["entries"] < 0.108 * (1 << 36)
    assert st["joined"] == st["entries"]
    assert st["retries"] == 0


def test_search_to_1_4e12_theorem1(ctx):
    """Theorem 1's whole range, n < 1.4e12: 42 pairs, nothing else (about a minute, 12 passes)."""
    N = 1400000000000 - 1
    say("search N=1.4e12 - 1 (hash-partitioned passes)")
    got = ctx.search(N)
    st = ctx.stats()
    assert got == theorem1_pairs(N)
    assert len(got) == 42
    assert st["integers"] == N and st["retries"] == 0


# --- batched --------------------------------------------------------------------------

def test_batch_planted_matches_oracle(ctx):
    from paper_2506_01099_amd.inputs import planted_queries

    a, b = planted_queries()
    got = ctx.search_batch(a, b)
    for i in range(a.size):
        assert got[i] == oracle.search_range(int(a[i]), int(b[i])), (int(a[i]), int(b[i]))


def test_batch_random_matches_oracle_and_sequential(ctx):
    from paper_2506_01099_amd.inputs import batched_queries

    a, b = batched_queries(n=48, seed=7, log2_min=8, log2_max=12, a_bits=34)
    got = ctx.search_batch(a, b)
    for i in range(a.size):
        want = oracle.search_range(int(a[i]), int(b[i]))
        assert got[i] == want
        assert ctx.search_range(int(a[i]), int(b[i])) == want


def test_batch_overlapping_and_degenerate_queries(ctx):
    a = np.array([1, 1, 2, 5, 5, 100, 0, 3], dtype=np.uint64)
    b = np.array([5000, 5000, 9, 5, 6, 100, 10, 2], dtype=np.uint64)
    got = ctx.search_batch(a, b)
    for i in range(a.size):
        assert got[i] == oracle.search_range(int(a[i]), int(b[i]) if b[i] >= a[i] else int(a[i]))


def test_batch_config_queries_sampled(ctx):
    """The 4096 seeded queries of the batched workload; a sample is re-run one by one."""
    from paper_2506_01099_amd.inputs import batched_queries

    a, b = batched_queries()
    got = ctx.search_batch(a, b)
    for i in range(0, 4096, 256):
        assert got[i] == ctx.search_range(int(a[i]), int(b[i]))
    small = [i for i in range(4096) if int(b[i] - a[i]) <= 2048][:8]
    for i in small:
        assert got[i] == oracle.search_range(int(a[i]), int(b[i]))
    # Past the small-query class: queries of 2^13 .. 2^16 integers against the oracle.
    mid = [i for i in range(4096) if 8192 < int(b[i] - a[i]) <= 1 << 16][:6]
    assert len(mid) == 6
    for i in mid:
        say(f"  query {i}: [{int(a[i])}, {int(b[i])})")
        assert got[i] == oracle.search_range(int(a[i]), int(b[i]))
    # Every reported pair of every query is a pair of that query, by trial division.
    for i, pairs in enumerate(got):
        for m, n, kind in pairs:
            assert int(a[i]) <= m < n < int(b[i])
            rm, rm1, rn, rn1 = (oracle.rad(v) for v in (m, m + 1, n, n + 1))
            assert (kind == 1 and rm == rn and rm1 == rn1) or (kind == 2 and rm == rn1 and rm1 == rn)


# --- small-query class ------------------------------------------------------------------

def _small_queries(n, seed):
    """Ranges of 2 .. 8192 integers (lengths log-uniform, plus the class edges) at
    magnitudes from 2^4 to 2^41, and a few just past the class's largest length."""
    from paper_2506_01099_amd.inputs import SplitMix64

    g = SplitMix64(seed)
    qs = [(1, 3), (1, 9), (2, 9), (1, 8193), (1, 2049), (35, 4375), (126, 8190), ((1 << 41) - 8192, 1 << 41),
          ((1 << 42) - 8194, (1 << 42) - 2), (5 << 30, (5 << 30) + 2), (5 << 30, (5 << 30) + 2048),
          (5 << 30, (5 << 30) + 2049), (7 << 33, (7 << 33) + 8193), (3 << 20, (3 << 20) + 4096)]
    for _ in range(n):
        L = int(2.0 ** (1 + 12 * g.unit()))
        bits = 4 + int(37 * g.unit())
        a = 1 + (g.next() >> (64 - bits))
        qs.append((a, a + max(2, L)))
    a = np.array([q[0] for q in qs], dtype=np.uint64)
    b = np.array([q[1] for q in qs], dtype=np.uint64)
    return a, b


@pytest.mark.parametrize("small_max,block", [(8192, 1024), (8192, 512), (8192, 256), (2048, 1024), (2048, 256),
                                             (1024, 512)])
def test_small_class_matches_oracle(ctx, small_max, block):
    """Queries sieved, member-tested and joined inside one workgroup (each cutoff and
    workgroup size) against the oracle, batched and one by one, graph and eager."""
    a, b = _small_queries(120, seed=small_max + block)
    want = [oracle.search_range(int(x), int(y)) for x, y in zip(a, b)]
    ctx.set_option("small_max", small_max)
    ctx.set_option("small_block", block)
    try:
        got = ctx.search_batch(a, b)
        st = ctx.stats()
        ctx.set_option("graph", 0)
        eager = ctx.search_batch(a, b)
        ctx.set_option("graph", 1)
        one = [ctx.search_range(int(x), int(y)) for x, y in zip(a[:24], b[:24])]
        st_one = ctx.stats()
    finally:
        ctx.set_option("small_max", 8192)
        ctx.set_option("small_block", 0)
        ctx.set_option("graph", 1)
    n_small = int(np.count_nonzero((b - a) <= small_max))
    assert st["launches"]["small"] == 1 and n_small > 50
    assert got == eager == want
    assert one == want[:24]
    assert st_one["launches"]["small"] == (1 if int(b[23] - a[23]) <= small_max else 0)
    assert any(want), "some query holds a pair"


def test_small_class_prune_off_and_kinds(ctx):
    a, b = _small_queries(40, seed=5)
    ctx.set_option("prune", 0)
    try:
        got = ctx.search_batch(a, b, kinds=1)
        st = ctx.stats()
    finally:
        ctx.set_option("prune", 1)
    assert got == [oracle.search_range(int(x), int(y), 1) for x, y in zip(a, b)]
    small = (b - a) <= 8192
    assert st["entries"] >= int((b - a)[small].sum())


def test_small_class_candidates_exact(ctx):
    """Join completeness inside the class, counted exactly: with 12 + 11 fingerprint bits
    kept and every integer joined (member test off), the kept sets of a query collide
    (about 4 per query of 8192), and the workgroup's hash table must report every pair of
    equal (query, fingerprint) -- one table per query, no bucket or pass."""
    from paper_2506_01099_amd.inputs import SplitMix64

    g = SplitMix64(77)
    qs = [(1, 8193), (1 << 20, (1 << 20) + 8192), (5 << 30, (5 << 30) + 5000), (1 << 12, 1 << 13)]
    for _ in range(44):
        a = 1 + (g.next() >> (64 - 4 - int(36 * g.unit())))
        qs.append((a, a + 8192))
    ctx.set_option("fp_bits", 12)
    ctx.set_option("prune", 0)
    try:
        got = ctx.search_batch(np.array([q[0] for q in qs], dtype=np.uint64),
                               np.array([q[1] for q in qs], dtype=np.uint64))
        st = ctx.stats()
    finally:
        ctx.set_option("fp_bits", 0)
        ctx.set_option("prune", 1)
    want, kept = 0, 0
    for i, (a, b) in enumerate(qs):
        assert got[i] == oracle.search_range(a, b)
        keys, n_kept = join_model.group_keys(oracle.radicals(a, b + 1), a, b, i, 0, 1, 12, prune=False)
        want += join_model.candidates(keys)
        kept += n_kept
    assert st["launches"]["small"] == 1 and st["launches"]["sieve"] == 0
    assert st["entries"] == st["joined"] == kept == sum(b - a for a, b in qs)
    assert want > 100
    assert st["candidates"] == want
    assert st["candidates"] == st["pairs"] + st["false_candidates"]


def test_small_class_on_off_same_results(ctx):
    """The 4096-query batched workload and a low-magnitude mix: identical pair lists with
    the class off, at 2048 and at 8192."""
    from paper_2506_01099_amd.inputs import batched_queries

    for a, b in (batched_queries(), batched_queries(n=512, seed=3, log2_min=1, log2_max=16, a_bits=24)):
        res = []
        for small_max in (0, 2048, 8192):
            ctx.set_option("small_max", small_max)
            try:
                res.append(ctx.search_batch(a, b))
                st = ctx.stats()
            finally:
                ctx.set_option("small_max", 8192)
            assert st["launches"]["small"] == (1 if small_max else 0)
        assert res[0] == res[1] == res[2]


# --- served ---------------------------------------------------------------------------

def test_served_alone_equals_in_mix(ctx):
    import time

    from paper_2506_01099_amd import Server

    reqs = [(1, 1 << 20), (2, 9), (70, 1300), (1 << 30, (1 << 30) + (1 << 22)), (30, 100000), (1, 1 << 16)]
    alone = [ctx.search_range(a, b) for a, b in reqs]
    srv = Server(ctx, budget_bytes=8 << 30, max_inflight=2)
    try:
        tickets = [srv.submit(a, b) for a, b in reqs]
        deadline = time.time() + 60
        results = {}
        while len(results) < len(tickets) and time.time() < deadline:
            for t in tickets:
                if t not in results and srv.poll(t):
                    results[t] = srv.take(t)
            time.sleep(0.001)
    finally:
        srv.stop()
    assert len(results) == len(tickets)
    for t, want in zip(tickets, alone):
        pairs, ts, td = results[t]
        assert pairs == want
        assert td >= ts


def test_served_budget_binds(ctx):
    """A budget that holds the workspace of about two of these requests: admission holds
    the others back, the lanes' workspaces never sum past the budget, and every result
    equals the request run alone."""
    import time

    from paper_2506_01099_amd import Server

    base = 1 << 40
    reqs = [(base + i * (1 << 25), base + (i + 1) * (1 << 25)) for i in range(6)]
    reqs += [(1, 1 << 22), (70, 1300), (1 << 30, (1 << 30) + (1 << 24))]
    alone = [ctx.search_range(a, b) for a, b in reqs]
    budget = 400 << 20
    srv = Server(ctx, budget_bytes=budget, max_inflight=3)
    try:
        tickets = [srv.submit(a, b) for a, b in reqs]
        deadline = time.time() + 120
        results = {}
        while len(results) < len(tickets) and time.time() < deadline:
            for t in tickets:
                if t not in results and srv.poll(t):
                    results[t] = srv.take(t)[0]
            time.sleep(0.001)
        info = srv.info()
    finally:
        srv.stop()
    say(f"served under a {budget >> 20} MiB budget: {info}")
    assert len(results) == len(tickets)
    for t, want in zip(tickets, alone):
        assert results[t] == want
    assert info["budget_bytes"] == budget and info["admitted"] == len(reqs)
    assert 0 < info["peak_bytes"] <= budget
    assert info["memory_waits"] > 0 and info["batches"] >= 2


def test_served_request_beyond_budget_is_refused(ctx):
    """A request whose workspace cannot be planned within the budget (even split into
    passes) is refused at submission, without blocking."""
    from paper_2506_01099_amd import BxError, Server

    srv = Server(ctx, budget_bytes=96 << 20, max_inflight=1)
    try:
        with pytest.raises(BxError) as ei:
            srv.submit(1 << 40, (1 << 40) + (1 << 24))
        assert ei.value.code == -5  # BX_EBUSY
        assert srv.info()["admitted"] == 0
    finally:
        srv.stop()


def test_served_submit_without_waiting(ctx):
    """With option submit_wait = 0 a request is admitted at once or refused with BX_EBUSY,
    queueing nothing: an idle server admits it; while the one lane runs a burst, it is
    refused.  Admitted requests return Theorem 1's lists, through bx_take (no times)."""
    import time

    from paper_2506_01099_amd import BxError, Server

    srv = Server(ctx, max_inflight=1)
    ctx.set_option("submit_wait", 0)
    try:
        t = srv.submit(1, 1 << 16)  # idle lane, empty queue: admitted
        while not srv.poll(t):
            time.sleep(0.001)
        assert srv.take_pairs(t) == oracle.search_range(1, 1 << 16)
        ctx.set_option("submit_wait", 1)
        burst = [srv.submit(1, 1 << 27) for _ in range(6)]
        ctx.set_option("submit_wait", 0)
        refused, extra = 0, []
        for _ in range(50):
            try:
                extra.append(srv.submit(1, 1 << 20))
            except BxError as e:
                assert e.code == -5  # BX_EBUSY
                refused += 1
        assert refused > 0
        for t in burst:
            while not srv.poll(t):
                time.sleep(0.001)
            assert srv.take_pairs(t) == theorem1_pairs((1 << 27) - 1)
        for t in extra:
            while not srv.poll(t):
                time.sleep(0.001)
            assert srv.take_pairs(t) == theorem1_pairs((1 << 20) - 1)
        with pytest.raises(BxError) as ei:
            srv.take_pairs(burst[0])  # already taken
        assert ei.value.code == -1
    finally:
        ctx.set_option("submit_wait", 1)
        srv.stop()


def test_served_kinds_and_lane_options(ctx):
    """Requests with different kinds masks share batches; the lanes run with the owner's
    options at serve start (here the sort join)."""
    import time

    from paper_2506_01099_amd import Server

    reqs = [(1, 1 << 20, 1), (1, 1 << 20, 2), (1, 1 << 20, 4), (30, 100000, 7), (2, 9, 3)]
    ctx.set_option("join", 1)
    try:
        srv = Server(ctx, budget_bytes=8 << 30, max_inflight=2)
    finally:
        ctx.set_option("join", 0)
    try:
        tickets = [srv.submit(a, b, k) for a, b, k in reqs]
        deadline = time.time() + 60
        results = {}
        while len(results) < len(tickets) and time.time() < deadline:
            for t in tickets:
                if t not in results and srv.poll(t):
                    results[t] = srv.take(t)[0]
            time.sleep(0.001)
    finally:
        srv.stop()
    assert len(results) == len(tickets)
    for t, (a, b, k) in zip(tickets, reqs):
        want = oracle.search_range(a, b, k & 3) if k & 3 else []  # no pair meets the third condition
        assert results[t] == want, (a, b, k)


# --- graph capture, tiles, autotuner -----------------------------------------------------

def test_batch_graph_follows_options(ctx):
    """The cached batch graph is captured again when an option it bakes in changes."""
    from paper_2506_01099_amd.inputs import planted_queries

    a, b = planted_queries()
    want = [oracle.search_range(int(x), int(y)) for x, y in zip(a, b)]
    assert ctx.search_batch(a, b) == want
    for name, val, default in (("join", 1, 0), ("prune", 0, 1), ("fp_bits", 12, 0)):
        ctx.set_option(name, val)
        try:
            got = ctx.search_batch(a, b)
            again = ctx.search_batch(a, b)
        finally:
            ctx.set_option(name, default)
        assert got == again == want, name
    assert ctx.search_batch(a, b) == want


def test_batch_graph_replays_match_eager(ctx):
    """The captured batch graph, replayed with eager work and syncs in between, equals the eager path."""
    import torch

    from paper_2506_01099_amd.inputs import batched_queries, planted_queries

    a1, b1 = planted_queries()
    a2, b2 = batched_queries(n=64, seed=11, log2_min=10, log2_max=16, a_bits=36)
    a = np.concatenate([a1, a2])
    b = np.concatenate([b1, b2])
    ctx.set_option("graph", 0)
    try:
        eager = ctx.search_batch(a, b)
    finally:
        ctx.set_option("graph", 1)
    for rep in range(4):
        got = ctx.search_batch(a, b)
        st = ctx.stats()
        assert got == eager, rep
        assert st["graph_ms"] > 0
        # eager work between replays
        assert ctx.search(1 << 16) == oracle.search(1 << 16)
        torch.cuda.synchronize()
    for i in range(a1.size):
        assert eager[i] == oracle.search_range(int(a1[i]), int(b1[i]))


@pytest.mark.parametrize("tile", [2048, 8192])
def test_tile_invariance(ctx, tile):
    ctx.set_option("tile", tile)
    try:
        got = ctx.search(1 << 22)
        rad = ctx.radical_segment((1 << 40) - 70000, (1 << 40) + 70000)
        st = ctx.stats()
    finally:
        ctx.set_option("tile", 0)
    assert got == theorem1_pairs(1 << 22)
    assert np.array_equal(rad, oracle.radicals((1 << 40) - 70000, (1 << 40) + 70000))


def test_autotune_and_load(ctx, tmp_path):
    from paper_2506_01099_amd import Benelux
    from paper_2506_01099_amd.inputs import planted_queries

    a, b = planted_queries()
    path = tmp_path / "tune.json"
    with Benelux(device=0) as t:
        t.autotune(a, b, reps=1, path=path)
        text = path.read_text()
        assert '"tile"' in text and '"seg_len"' in text and '"group"' in text
        got = t.search_batch(a, b)
    for i in range(a.size):
        assert got[i] == oracle.search_range(int(a[i]), int(b[i]))
    ctx.load_tuning(path)
    try:
        assert ctx.search(1 << 20) == oracle.search(1 << 20)
    finally:
        ctx.set_option("tile", 0)
        ctx.set_option("seg_len", 0)
        ctx.set_option("group", 0)
