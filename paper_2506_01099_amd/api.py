"""Thin Python binding over the C-ABI in include/benelux.h (argument marshalling only).

Radicals (Algorithm 1 of arXiv:2506.01099) and the join over the sets
{rad(x), rad(x+1)} (Section 2) run in the library's HIP kernels.  PyTorch is used
only for device buffers and streams (radical_segment_dev).
"""
import ctypes

import numpy as np

from ._lib import Pair, ServeInfo, Stats, check, load

FIRST, SECOND, BOTH, THIRD = 1, 2, 3, 4  # THIRD: also rad(m+2) = rad(n+2) (kind 5)
VALUE_LIMIT = 1 << 42


def _split_by_offsets(flat, offs, q):
    """Per-query slices of a flat pair list, offs holding the q + 1 running offsets (a
    ctypes size_t array): one bulk conversion of the offsets instead of q * 2 ctypes reads."""
    if not flat:
        return [[] for _ in range(q)]
    b = np.frombuffer(offs, dtype=np.uintp, count=q + 1).tolist()
    return [flat[b[i]:b[i + 1]] for i in range(q)]


def _pairs_from(ptr, count):
    lib = load()
    try:
        return [(int(ptr[i].m), int(ptr[i].n), int(ptr[i].kind)) for i in range(count)]
    finally:
        if count:
            lib.bx_free(ptr)


class Benelux:
    """A library context: resident prime tables, workspace and a HIP stream on one device."""

    def __init__(self, device=0, hi_max=VALUE_LIMIT - 1, hbm_budget=0):
        lib = load()
        self._lib = lib
        self._h = ctypes.c_void_p()
        check(lib.bx_create(ctypes.byref(self._h), int(device), int(hi_max), int(hbm_budget)))
        self.device = device
        self.hi_max = hi_max

    def close(self):
        if self._h:
            self._lib.bx_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- configuration ---------------------------------------------------------------
    def set_option(self, name, value):
        check(self._lib.bx_set_option(self._h, name.encode(), int(value)))

    def set_stream(self, stream):
        """Run on a torch.cuda.Stream (or a raw hipStream_t int); None = own stream."""
        handle = None if stream is None else int(getattr(stream, "cuda_stream", stream))
        check(self._lib.bx_set_stream(self._h, ctypes.c_void_p(handle)))

    def stats(self):
        st = Stats()
        check(self._lib.bx_get_stats(self._h, ctypes.byref(st)))
        names = ["sieve", "partition", "join", "verify", "radicals", "small"]
        return {
            "passes": st.passes, "retries": st.retries, "integers": st.integers, "entries": st.entries,
            "candidates": st.candidates, "pairs": st.pairs,
            "launches": dict(zip(names, list(st.launches))), "kernel_ms": dict(zip(names, list(st.kernel_ms))),
            "total_ms": st.total_ms, "b1_bits": st.b1_bits, "b2_bits": st.b2_bits,
            "seg_len": st.seg_len, "tile": st.tile, "graph_ms": st.graph_ms,
            "joined": st.joined, "false_candidates": st.false_candidates, "l2_entry_bytes": st.l2_entry_bytes,
            "word_matches": st.word_matches,
        }

    def autotune(self, a, b, reps=1, path=None):
        """Sweep tile / segment length / group on the queries [a[i], b[i]); keep the fastest."""
        a = np.ascontiguousarray(a, dtype=np.uint64)
        b = np.ascontiguousarray(b, dtype=np.uint64)
        P64 = ctypes.POINTER(ctypes.c_uint64)
        check(self._lib.bx_autotune(self._h, a.ctypes.data_as(P64), b.ctypes.data_as(P64), a.size, int(reps),
                                    None if path is None else str(path).encode()))

    def load_tuning(self, path):
        check(self._lib.bx_load_tuning(self._h, str(path).encode()))

    # -- radicals ----------------------------------------------------------------------
    def radical_segment(self, lo, hi, out=None):
        """numpy uint64 array of rad(x), x in [lo, hi)."""
        n = max(0, int(hi) - int(lo))
        if out is None:
            out = np.empty(n, dtype=np.uint64)
        if out.dtype != np.uint64 or out.size < n or not out.flags.c_contiguous:
            raise ValueError("out must be a contiguous uint64 array of hi - lo elements")
        check(self._lib.bx_radical_segment(self._h, int(lo), int(hi),
                                           out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))))
        return out[:n]

    def radical_segment_dev(self, lo, hi, out_tensor, stream=None):
        """Write rad(x), x in [lo, hi), into a torch uint64/int64 CUDA tensor on `stream`
        (torch's current stream by default; its handle is 0 for the default stream, which
        the library takes as HIP's null stream)."""
        import torch

        n = max(0, int(hi) - int(lo))
        if not out_tensor.is_cuda or out_tensor.element_size() != 8 or out_tensor.numel() < n \
                or not out_tensor.is_contiguous():
            raise ValueError("out_tensor must be a contiguous 8-byte CUDA tensor with hi - lo elements")
        s = stream if stream is not None else torch.cuda.current_stream(out_tensor.device)
        check(self._lib.bx_radical_segment_dev(self._h, int(lo), int(hi), ctypes.c_void_p(out_tensor.data_ptr()),
                                               ctypes.c_void_p(int(s.cuda_stream))))
        return out_tensor

    # -- searches ------------------------------------------------------------------------
    def search(self, N, kinds=BOTH):
        """Sorted [(m, n, kind)] with 1 <= m < n <= N."""
        p, c = ctypes.POINTER(Pair)(), ctypes.c_size_t(0)
        check(self._lib.bx_benelux_search(self._h, int(N), int(kinds), ctypes.byref(p), ctypes.byref(c)))
        return _pairs_from(p, c.value)

    def search_range(self, a, b, kinds=BOTH):
        """Sorted [(m, n, kind)] with max(a,1) <= m < n < b."""
        p, c = ctypes.POINTER(Pair)(), ctypes.c_size_t(0)
        check(self._lib.bx_search_range(self._h, int(a), int(b), int(kinds), ctypes.byref(p), ctypes.byref(c)))
        return _pairs_from(p, c.value)

    def search_batch(self, a, b, kinds=BOTH):
        """List (one per query) of sorted [(m, n, kind)] inside [a[i], b[i])."""
        a = np.ascontiguousarray(a, dtype=np.uint64)
        b = np.ascontiguousarray(b, dtype=np.uint64)
        if a.shape != b.shape or a.ndim != 1:
            raise ValueError("a and b must be 1-D arrays of equal length")
        q = a.size
        offs = (ctypes.c_size_t * (q + 1))()
        p = ctypes.POINTER(Pair)()
        P64 = ctypes.POINTER(ctypes.c_uint64)
        check(self._lib.bx_search_batch(self._h, a.ctypes.data_as(P64), b.ctypes.data_as(P64), q, int(kinds),
                                        ctypes.byref(p), offs))
        return _split_by_offsets(_pairs_from(p, offs[q]), offs, q)


class Server:
    """Continuous-batching request loop of the library (bx_serve_*)."""

    def __init__(self, ctx, budget_bytes=0, max_inflight=2):
        self.ctx = ctx
        self._lib = ctx._lib
        check(self._lib.bx_serve_start(ctx._h, int(budget_bytes), int(max_inflight)))

    def submit(self, a, b, kinds=BOTH):
        t = ctypes.c_uint64(0)
        check(self._lib.bx_submit(self.ctx._h, int(a), int(b), int(kinds), ctypes.byref(t)))
        return t.value

    def poll(self, ticket):
        d = ctypes.c_int(0)
        check(self._lib.bx_poll(self.ctx._h, int(ticket), ctypes.byref(d)))
        return bool(d.value)

    def take(self, ticket):
        """(pairs, t_submit, t_done) of a finished request."""
        p, c = ctypes.POINTER(Pair)(), ctypes.c_size_t(0)
        ts, td = ctypes.c_double(0), ctypes.c_double(0)
        check(self._lib.bx_take_timed(self.ctx._h, int(ticket), ctypes.byref(p), ctypes.byref(c), ctypes.byref(ts),
                                      ctypes.byref(td)))
        return _pairs_from(p, c.value), ts.value, td.value

    def take_pairs(self, ticket):
        """The pair list of a finished request (bx_take)."""
        p, c = ctypes.POINTER(Pair)(), ctypes.c_size_t(0)
        check(self._lib.bx_take(self.ctx._h, int(ticket), ctypes.byref(p), ctypes.byref(c)))
        return _pairs_from(p, c.value)

    def info(self):
        """Admission record: budget, peak and current workspace bytes, batches, waits."""
        v = ServeInfo()
        check(self._lib.bx_serve_get_info(self.ctx._h, ctypes.byref(v)))
        return {name: int(getattr(v, name)) for name, _ in ServeInfo._fields_}

    def now(self):
        return self._lib.bx_now()

    def stop(self):
        check(self._lib.bx_serve_stop(self.ctx._h))


def benelux_search(N, kinds=BOTH):
    """The library's default-context search: sorted [(m, n, kind)], 1 <= m < n <= N."""
    lib = load()
    p, c = ctypes.POINTER(Pair)(), ctypes.c_size_t(0)
    check(lib.benelux_search(int(N), int(kinds), ctypes.byref(p), ctypes.byref(c)))
    return _pairs_from(p, c.value)


def radical_segment(lo, hi, out=None):
    """The library's default-context radicals: numpy uint64 rad(x), x in [lo, hi)."""
    lib = load()
    n = max(0, int(hi) - int(lo))
    if out is None:
        out = np.empty(n, dtype=np.uint64)
    check(lib.radical_segment(int(lo), int(hi), out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))))
    return out[:n]
