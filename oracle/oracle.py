"""ctypes wrapper over liboracle.so (test infrastructure only)."""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "benelux_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


class _Pair(ctypes.Structure):
    _fields_ = [("m", ctypes.c_uint64), ("n", ctypes.c_uint64),
                ("kind", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


def lib_path():
    return _LIB


def build(force=True):
    """Compile the oracle with the host compiler (g++), in-tree."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-pthread",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        lib.orc_rad.argtypes = [ctypes.c_uint64]
        lib.orc_rad.restype = ctypes.c_uint64
        lib.orc_radicals.argtypes = [ctypes.c_uint64, ctypes.c_uint64,
                                     ctypes.POINTER(ctypes.c_uint64), ctypes.c_int]
        lib.orc_radicals.restype = ctypes.c_int
        lib.orc_search_range.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int,
                                         ctypes.POINTER(ctypes.POINTER(_Pair)),
                                         ctypes.POINTER(ctypes.c_size_t),
                                         ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        lib.orc_search_range.restype = ctypes.c_int
        lib.orc_search_range_ex.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                            ctypes.c_int, ctypes.POINTER(ctypes.POINTER(_Pair)),
                                            ctypes.POINTER(ctypes.c_size_t),
                                            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        lib.orc_search_range_ex.restype = ctypes.c_int
        lib.orc_free.argtypes = [ctypes.c_void_p]
        lib.orc_free.restype = None
        _lib = lib
    return _lib


def rad(x):
    """rad(x) by trial division (x >= 1)."""
    if x < 1:
        raise ValueError("rad is defined for positive integers")
    return int(_load().orc_rad(int(x)))


def radicals(lo, hi, threads=0):
    """numpy uint64 array of rad(x) for x in [lo, hi)."""
    if lo < 1 or hi < lo:
        raise ValueError("need 1 <= lo <= hi")
    out = np.empty(hi - lo, dtype=np.uint64)
    rc = _load().orc_radicals(int(lo), int(hi),
                              out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), int(threads))
    if rc != 0:
        raise RuntimeError(f"orc_radicals failed ({rc})")
    return out


def search_range_timed(a, b, kinds=3, threads=0, third_offset=2):
    """(pairs, t_radicals_s, t_join_s); pairs sorted list of (m, n, kind), max(a,1) <= m < n < b.

    kinds is a mask in 1..7: 1 first kind, 2 second kind, 4 a first-kind pair that
    also has rad(m + third_offset) = rad(n + third_offset), reported as kind 5
    (third_offset = 2 is Erdos's third condition)."""
    if kinds not in range(1, 8):
        raise ValueError("kinds must be a mask in 1..7")
    if third_offset < 0:
        raise ValueError("third_offset must be >= 0")
    p = ctypes.POINTER(_Pair)()
    cnt = ctypes.c_size_t(0)
    tr, tj = ctypes.c_double(0.0), ctypes.c_double(0.0)
    lib = _load()
    rc = lib.orc_search_range_ex(int(a), int(b), int(kinds), int(third_offset), int(threads), ctypes.byref(p),
                                 ctypes.byref(cnt), ctypes.byref(tr), ctypes.byref(tj))
    if rc != 0:
        raise RuntimeError(f"orc_search_range_ex failed ({rc})")
    try:
        pairs = [(int(p[i].m), int(p[i].n), int(p[i].kind)) for i in range(cnt.value)]
    finally:
        if cnt.value:
            lib.orc_free(p)
    return pairs, tr.value, tj.value


def search_range(a, b, kinds=3, threads=0, third_offset=2):
    return search_range_timed(a, b, kinds, threads, third_offset)[0]


def search(N, kinds=3, threads=0, third_offset=2):
    """All pairs 1 <= m < n <= N (radicals over [1, N+1])."""
    return search_range(1, N + 1, kinds, threads, third_offset)
