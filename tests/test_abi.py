"""CPU checks of the boundary: the library builds, loads and exports every
declared symbol, and fails cleanly (no crash) without a GPU."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_2506_01099_amd as bx
from paper_2506_01099_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "benelux.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_parses():
    names = header_functions()
    assert "bx_benelux_search" in names and "radical_segment" in names and "benelux_search" in names
    assert sorted(_lib.EXPORTS) == names


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    for name in header_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    for name in header_functions():
        assert name in exported, name


def test_library_is_gfx950_code_object():
    out = subprocess.run(["strings", _lib.LIB_PATH], capture_output=True, text=True).stdout
    assert "gfx950" in out


def test_errors_without_device_or_bad_args():
    lib = _lib.load()
    h = ctypes.c_void_p()
    assert lib.bx_create(None, 0, 2**20, 0) == _lib.BX_EINVAL
    rc = lib.bx_create(ctypes.byref(h), 0, 2**43, 0)
    assert rc == _lib.BX_ERANGE
    assert b"hi_max" in lib.bx_last_error()
    assert lib.bx_search_range(None, 1, 10, 3, None, None) == _lib.BX_EINVAL
    assert lib.bx_radical_segment(None, 1, 10, None) == _lib.BX_EINVAL


@pytest.mark.skipif(os.path.exists("/dev/kfd") and os.access("/dev/kfd", os.R_OK), reason="a GPU is present")
def test_create_without_gpu_reports_device_error():
    with pytest.raises(bx.BxError) as ei:
        bx.Benelux(device=0, hi_max=2**20)
    assert ei.value.code == _lib.BX_EDEVICE


def test_batch_result_split_by_offsets():
    """The binding's per-query split of a batched call's flat pair list (argument
    marshalling only) against slicing with each offset read one by one."""
    import ctypes

    from paper_2506_01099_amd.api import _split_by_offsets

    for counts in ([], [0], [0, 0, 0], [2, 0, 1, 0, 3], [0] * 4096):
        q = len(counts)
        offs = (ctypes.c_size_t * (q + 1))()
        for i, c in enumerate(counts):
            offs[i + 1] = offs[i] + c
        flat = [(i, i + 1, 1) for i in range(offs[q])]
        want = [flat[offs[i]:offs[i + 1]] for i in range(q)]
        assert _split_by_offsets(flat, offs, q) == want
