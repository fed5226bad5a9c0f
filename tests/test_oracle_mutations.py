"""The oracle's pins catch plausible mistakes.

Each case copies the oracle's source to a temporary directory, plants one mistake
(a dropped term, an off-by-one, a swapped classification, a lost group member, a
missing overlap value), builds it with the host compiler and checks that at least one
pin rejects it.  The real oracle is never modified.
"""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_facts import theorem1_pairs
from test_oracle import _bruteforce_third, spf_radicals, squarefree_count

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "benelux_oracle.cpp")

MUTATIONS = {
    "drop_large_prime_cofactor": ("  if (x > 1) r *= x;\n", "\n"),
    "trial_bound_off_by_one": ("for (uint64_t d = 3; d <= x / d; d += 2)", "for (uint64_t d = 3; d < x / d; d += 2)"),
    "adjacent_pairs_only": ("for (size_t j = i + 1; j < xs.size(); ++j)",
                            "for (size_t j = i + 1; j < xs.size() && j == i + 1; ++j)"),
    "kinds_swapped": ("(r[m - a] == r[n - a]) ? 1u : 2u", "(r[m - a] == r[n - a]) ? 2u : 1u"),
    "missing_overlap_value": ("radicals_mt(a, b + 1, r.data(), threads);", "radicals_mt(a, b, r.data(), threads);"),
    "two_kept_twice": ("    while ((x & 1) == 0) x >>= 1;\n", "    x >>= 1;\n"),
    "third_offset_off_by_one": ("rad_trial(n + third_offset)", "rad_trial(n + third_offset + 1)"),
    "third_fixed_offset": ("rad_trial(m + third_offset)", "rad_trial(m + 2)"),
    "third_marks_without_kind_bit": ("pairs.push_back({m, n, kind | 4u, 0u});", "pairs.push_back({m, n, kind, 0u});"),
}


class Mutant:
    def __init__(self, path):
        self.lib = ctypes.CDLL(path)
        self.lib.orc_rad.argtypes = [ctypes.c_uint64]
        self.lib.orc_rad.restype = ctypes.c_uint64
        self.lib.orc_radicals.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64), ctypes.c_int]
        self.lib.orc_search_range.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int,
                                              ctypes.POINTER(ctypes.POINTER(oracle.oracle._Pair)),
                                              ctypes.POINTER(ctypes.c_size_t), ctypes.c_void_p, ctypes.c_void_p]
        self.lib.orc_search_range_ex.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                                 ctypes.c_int, ctypes.POINTER(ctypes.POINTER(oracle.oracle._Pair)),
                                                 ctypes.POINTER(ctypes.c_size_t), ctypes.c_void_p, ctypes.c_void_p]
        self.lib.orc_free.argtypes = [ctypes.c_void_p]

    def radicals(self, lo, hi):
        out = np.zeros(hi - lo, dtype=np.uint64)
        self.lib.orc_radicals(lo, hi, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), 2)
        return out

    def search_range(self, a, b, kinds=3, third_offset=2):
        p = ctypes.POINTER(oracle.oracle._Pair)()
        c = ctypes.c_size_t(0)
        assert self.lib.orc_search_range_ex(a, b, kinds, third_offset, 2, ctypes.byref(p), ctypes.byref(c),
                                            None, None) == 0
        res = [(int(p[i].m), int(p[i].n), int(p[i].kind)) for i in range(c.value)]
        if c.value:
            self.lib.orc_free(p)
        return res


def pins_pass(m):
    """True when every pin accepts the (possibly mutated) oracle."""
    r = spf_radicals(4097)
    if not np.array_equal(m.radicals(1, 4098).astype(np.int64), r[1:]):
        return False
    if m.search_range(1, 4097) != theorem1_pairs(4096):
        return False
    if m.search_range(1, (1 << 20) + 1) != theorem1_pairs(1 << 20):
        return False
    for a, b in [(35, 4375), (2, 9), (126, 16129)]:
        if m.search_range(a, b) != [p for p in theorem1_pairs(1 << 20) if p[0] >= a and p[1] < b]:
            return False
    x = np.arange(1, (1 << 16) + 1, dtype=np.uint64)
    if int(np.count_nonzero(m.radicals(1, (1 << 16) + 1) == x)) != squarefree_count(1 << 16):
        return False
    # Third condition: brute force by the definition for the offsets 1, 2, 4.
    rr = spf_radicals(4097 + 8)
    for d in (1, 2, 4):
        want = [(a, b, 5) for a, b in _bruteforce_third(4096, d, rr)]
        if m.search_range(1, 4097, kinds=4, third_offset=d) != want:
            return False
        marked = {(a, b) for a, b, _ in want}
        full = [(a, b, 5 if (a, b) in marked else k) for a, b, k in theorem1_pairs(4096)]
        if m.search_range(1, 4097, kinds=7, third_offset=d) != full:
            return False
    return True


def build_variant(tmp_path, name, old, new):
    src = open(SRC).read()
    assert old in src, f"mutation {name} no longer applies to the oracle source"
    d = tmp_path / name
    d.mkdir()
    path = d / "benelux_oracle.cpp"
    path.write_text(src.replace(old, new, 1))
    lib = d / "liboracle_mut.so"
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-pthread", "-o", str(lib), str(path)])
    return str(lib)


def test_unmutated_oracle_passes_pins(tmp_path):
    lib = tmp_path / "liboracle_copy.so"
    shutil.copy(oracle.lib_path(), lib)
    assert pins_pass(Mutant(str(lib)))


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(tmp_path, name):
    old, new = MUTATIONS[name]
    m = Mutant(build_variant(tmp_path, name, old, new))
    assert not pins_pass(m), f"the pins did not catch the planted mistake {name}"
