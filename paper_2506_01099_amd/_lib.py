"""ctypes binding of libbenelux.so: argument marshalling only.

Every step of the search runs in the library's HIP kernels; there is no Python
or CPU fallback.  Loading fails loudly when the library has not been built.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbenelux.so")

BX_OK, BX_EINVAL, BX_ERANGE, BX_ENOMEM, BX_EDEVICE, BX_EBUSY, BX_EINTERNAL = 0, -1, -2, -3, -4, -5, -6
_NAMES = {BX_EINVAL: "BX_EINVAL", BX_ERANGE: "BX_ERANGE", BX_ENOMEM: "BX_ENOMEM", BX_EDEVICE: "BX_EDEVICE",
          BX_EBUSY: "BX_EBUSY", BX_EINTERNAL: "BX_EINTERNAL"}

# Every symbol declared in include/benelux.h.
EXPORTS = [
    "bx_create", "bx_destroy", "bx_set_stream", "bx_radical_segment", "bx_radical_segment_dev",
    "bx_radical_segment_dev_noalloc", "bx_benelux_search", "bx_search_range", "bx_search_batch", "bx_serve_start", "bx_serve_stop",
    "bx_submit", "bx_poll", "bx_take", "bx_take_timed", "bx_serve_get_info", "bx_now", "bx_get_stats", "bx_set_option", "bx_free",
    "bx_autotune", "bx_load_tuning",
    "bx_last_error", "benelux_search", "radical_segment",
]


class BxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class Pair(ctypes.Structure):
    _fields_ = [("m", ctypes.c_uint64), ("n", ctypes.c_uint64),
                ("kind", ctypes.c_uint32), ("query", ctypes.c_uint32)]


class ServeInfo(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_uint64), ("peak_bytes", ctypes.c_uint64), ("held_bytes", ctypes.c_uint64),
                ("admitted", ctypes.c_uint64), ("batches", ctypes.c_uint64), ("max_batch", ctypes.c_uint32),
                ("lanes", ctypes.c_uint32), ("memory_waits", ctypes.c_uint64), ("releases", ctypes.c_uint64)]


class Stats(ctypes.Structure):
    _fields_ = [("passes", ctypes.c_uint32), ("retries", ctypes.c_uint32),
                ("integers", ctypes.c_uint64), ("entries", ctypes.c_uint64),
                ("candidates", ctypes.c_uint64), ("pairs", ctypes.c_uint64),
                ("launches", ctypes.c_uint32 * 6), ("kernel_ms", ctypes.c_double * 6),
                ("total_ms", ctypes.c_double), ("b1_bits", ctypes.c_uint32), ("b2_bits", ctypes.c_uint32),
                ("seg_len", ctypes.c_uint32), ("tile", ctypes.c_uint32), ("graph_ms", ctypes.c_double),
                ("joined", ctypes.c_uint64), ("false_candidates", ctypes.c_uint64),
                ("l2_entry_bytes", ctypes.c_uint32), ("word_matches", ctypes.c_uint32)]


_lib = None


def load():
    """The CDLL of the built library (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    # Share one HIP runtime with PyTorch: torch bundles its own libamdhip64 /
    # libhsa-runtime64 (same sonames).  Loading torch first makes the dynamic
    # linker bind this library to those copies, so torch's device buffers and
    # streams are valid handles for the library (two runtimes in one process
    # cannot share a device).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2506_01099_amd.build.build() "
                          "(the HIP library is required; there is no fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, u64, u32, sz = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_size_t
    P64 = ctypes.POINTER(ctypes.c_uint64)
    PP = ctypes.POINTER(ctypes.POINTER(Pair))
    sig = {
        "bx_create": ([ctypes.POINTER(vp), ctypes.c_int, u64, u64], ctypes.c_int),
        "bx_destroy": ([vp], None),
        "bx_set_stream": ([vp, vp], ctypes.c_int),
        "bx_radical_segment": ([vp, u64, u64, P64], ctypes.c_int),
        "bx_radical_segment_dev": ([vp, u64, u64, vp, vp], ctypes.c_int),
        "bx_radical_segment_dev_noalloc": ([vp, u64, u64, vp, vp], ctypes.c_int),
        "bx_benelux_search": ([vp, u64, u32, PP, ctypes.POINTER(sz)], ctypes.c_int),
        "bx_search_range": ([vp, u64, u64, u32, PP, ctypes.POINTER(sz)], ctypes.c_int),
        "bx_search_batch": ([vp, P64, P64, sz, u32, PP, ctypes.POINTER(sz)], ctypes.c_int),
        "bx_serve_start": ([vp, u64, ctypes.c_int], ctypes.c_int),
        "bx_serve_stop": ([vp], ctypes.c_int),
        "bx_submit": ([vp, u64, u64, u32, P64], ctypes.c_int),
        "bx_poll": ([vp, u64, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
        "bx_take": ([vp, u64, PP, ctypes.POINTER(sz)], ctypes.c_int),
        "bx_take_timed": ([vp, u64, PP, ctypes.POINTER(sz), ctypes.POINTER(ctypes.c_double),
                           ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
        "bx_serve_get_info": ([vp, ctypes.POINTER(ServeInfo)], ctypes.c_int),
        "bx_now": ([], ctypes.c_double),
        "bx_autotune": ([vp, P64, P64, sz, ctypes.c_int, ctypes.c_char_p], ctypes.c_int),
        "bx_load_tuning": ([vp, ctypes.c_char_p], ctypes.c_int),
        "bx_get_stats": ([vp, ctypes.POINTER(Stats)], ctypes.c_int),
        "bx_set_option": ([vp, ctypes.c_char_p, ctypes.c_int64], ctypes.c_int),
        "bx_free": ([vp], None),
        "bx_last_error": ([], ctypes.c_char_p),
        "benelux_search": ([u64, u32, PP, ctypes.POINTER(sz)], ctypes.c_int),
        "radical_segment": ([u64, u64, P64], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def check(rc):
    if rc != BX_OK:
        msg = load().bx_last_error()
        raise BxError(rc, msg.decode() if msg else "")
    return rc
