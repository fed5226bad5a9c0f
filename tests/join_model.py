"""Which entries the join must bring together, restated in numpy for the tests.

The GPU join reports a candidate for every two entries whose fingerprints (and,
in batched calls, query ids) are equal inside one first-level bucket of one
hash pass: the insert and probe steps of Algorithm 3 report every earlier equal
key on the probe chain, so a group of k equal keys yields k(k-1)/2 candidates.
This module recomputes, from radicals that do not come from the join, the
entries that pass the member test, their 64-bit key hash, first-level bucket,
pass and (possibly truncated) fingerprint, and from them the exact number of
candidates a complete join must emit.  The hash functions are the library's
design choices (the paper leaves the hash open), restated here from their
definitions: SplitMix64's output mix (Steele, Lea & Flood 2014) over
(lo | q << 43) * K xor hi, and the 24-bit-multiply pass hash.
"""
import numpy as np

K_MUL = np.uint64(0x9E3779B97F4A7C15)
FP_BITS = 53


def mix64(z):
    z = z.copy()
    z ^= z >> np.uint64(30)
    z *= np.uint64(0xBF58476D1CE4E5B9)
    z ^= z >> np.uint64(27)
    z *= np.uint64(0x94D049BB133111EB)
    z ^= z >> np.uint64(31)
    return z


def key64(lo, hi, grp):
    """64-bit hash of the canonical pair lo < hi and the query id (uint64 arrays)."""
    with np.errstate(over="ignore"):
        return mix64(((lo | (grp.astype(np.uint64) << np.uint64(43))) * K_MUL) ^ hi)


def pass_hash(lo, hi, grp):
    """The 32-bit hash that picks an entry's pass when a search runs several passes."""
    m24 = np.uint64(0xFFFFFF)
    m32 = np.uint64(0xFFFFFFFF)

    def mul24(a, c):
        return ((a & m24) * np.uint64(c)) & m32

    l0, l1 = lo & np.uint64(0x1FFFFF), lo >> np.uint64(21)
    h0, h1 = hi & np.uint64(0x1FFFFF), hi >> np.uint64(21)
    g = grp.astype(np.uint64)
    s = (mul24(l0, 0x9E3779) + mul24(l1, 0x7F4A7D) + mul24(h0, 0xC2B2AF) + mul24(h1, 0x85EBCB)
         + mul24(g, 0x27D4EB)) & m32
    s ^= s >> np.uint64(15)
    s = (s * np.uint64(0x2C1B3C6D)) & m32
    s ^= s >> np.uint64(12)
    return s


def fp_mask(fp_bits):
    """The fingerprint bits a search keeps under the test option fp_bits (0 = all 53)."""
    full = (1 << FP_BITS) - 1
    if fp_bits == 0 or fp_bits >= 42:
        return full
    return (full & ~((1 << 42) - 1)) | ((1 << fp_bits) - 1)


def kept(x, r0, r1, b):
    """Member test: x (with r0 = rad(x), r1 = rad(x + 1)) can belong to a pair m < n < b.
    int64 arrays.  y * M > b is taken as M > floor(b / y) (y >= 1), which is exact and
    cannot overflow: the product itself passes 2^63 once y and M are near 2^32."""
    drop0 = (r0 == x) & (np.maximum(2, r1 - 1) > b // x)
    drop1 = (r1 == x + 1) & (np.maximum(2, r0 - 1) > b // (x + 1))
    return (x <= 3) | ~(drop0 | drop1)


def group_keys(rad, a, b, grp, b1_bits, passes, fp_bits, prune=True):
    """For the query [a, b) with rad[i] = rad(a + i), i in [0, b - a], the join group of
    every entry that passes the member test: one uint64 per entry holding its pass,
    first-level bucket, query and kept fingerprint bits.  Entries meet exactly when
    their group keys are equal."""
    n = b - a
    x = np.arange(a, b, dtype=np.int64)
    r = rad.astype(np.int64)
    r0, r1 = r[:n], r[1:n + 1]
    keep = kept(x, r0, r1, b) if prune else np.ones(n, dtype=bool)
    u0, u1 = r0[keep].astype(np.uint64), r1[keep].astype(np.uint64)
    lo, hi = np.minimum(u0, u1), np.maximum(u0, u1)
    g = np.full(lo.shape, grp, dtype=np.uint64)
    h = key64(lo, hi, g)
    bucket = h & np.uint64((1 << b1_bits) - 1)
    fp = (h >> np.uint64(11)) & np.uint64(fp_mask(fp_bits))
    if passes > 1:
        bounds = np.array([(p << 32) // passes for p in range(1, passes)], dtype=np.uint64)
        pidx = np.searchsorted(bounds, pass_hash(lo, hi, g), side="right").astype(np.uint64)
    else:
        pidx = np.zeros(lo.shape, dtype=np.uint64)
    # The fingerprint keeps its top 11 bits and its low fp_bits bits (< 42): 11 + fp_bits
    # bits of information, packed next to the pass (6 bits), bucket (10) and query (15).
    assert 0 < fp_bits <= 21
    top, low = fp >> np.uint64(42), fp & np.uint64((1 << fp_bits) - 1)
    fpc = (top << np.uint64(fp_bits)) | low
    return (((pidx << np.uint64(10) | bucket) << np.uint64(15) | g) << np.uint64(32)) | fpc, int(keep.sum())


def compact_keys(rad, a, b, grp, b1_bits, b2_bits, keep_bits):
    """For the query [a, b), the group of every kept entry under the compact second
    level (one pass): entries meet when their first-level bucket (low b1_bits of the
    key hash), their partition (top b2_bits of the 53-bit fingerprint) and the low
    keep_bits of the fingerprint agree -- the query itself is not compared (the join
    reads such matches back from the first level and drops those across queries)."""
    n = b - a
    x = np.arange(a, b, dtype=np.int64)
    r = rad.astype(np.int64)
    r0, r1 = r[:n], r[1:n + 1]
    keep = kept(x, r0, r1, b)
    u0, u1 = r0[keep].astype(np.uint64), r1[keep].astype(np.uint64)
    lo, hi = np.minimum(u0, u1), np.maximum(u0, u1)
    h = key64(lo, hi, np.full(lo.shape, grp, dtype=np.uint64))
    bucket = h & np.uint64((1 << b1_bits) - 1)
    fp = h >> np.uint64(11)
    part = fp >> np.uint64(53 - b2_bits) if b2_bits else np.zeros_like(fp)
    low = fp & np.uint64((1 << keep_bits) - 1)
    assert b1_bits + b2_bits + keep_bits <= 64
    return (((bucket << np.uint64(b2_bits)) | part) << np.uint64(keep_bits)) | low, int(keep.sum())


def candidates(keys):
    """Pairs inside groups of equal keys: sum of k(k-1)/2."""
    if keys.size == 0:
        return 0
    _, cnt = np.unique(keys, return_counts=True)
    cnt = cnt.astype(np.int64)
    return int((cnt * (cnt - 1) // 2).sum())
