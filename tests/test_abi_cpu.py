"""Host-side checks of the C-ABI library (no GPU work is launched)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tl.h")
LIB = os.path.join(ROOT, "paper_2203_04774_amd", "libtl.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(tl_[a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libtl.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["tl_orient", "tl_cost", "tl_list", "tl_list_range", "tl_csr_free", "tl_strerror"]:
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_strerror_and_host_only_errors(lib):
    lib.tl_strerror.restype = ctypes.c_char_p
    lib.tl_last_error.restype = ctypes.c_char_p
    texts = {lib.tl_strerror(c).decode() for c in range(6)}
    assert len(texts) == 6
    assert lib.tl_strerror(99).decode() == "unknown error code"
    lib.tl_set_chunk_triangles.argtypes = [ctypes.c_uint64]
    assert lib.tl_set_chunk_triangles(0) == 1          # TL_EINVAL
    assert b"chunk" in lib.tl_last_error()
    lib.tl_csr_free.argtypes = [ctypes.c_void_p]
    lib.tl_csr_free(None)                               # no-op


def test_null_arguments_rejected_without_device_work(lib):
    vp = ctypes.c_void_p
    lib.tl_cost.argtypes = [vp, ctypes.c_int, vp, vp]
    out = ctypes.c_uint64()
    assert lib.tl_cost(None, 0, None, ctypes.byref(out)) == 1
    lib.tl_csr_size.argtypes = [vp, vp, vp]
    assert lib.tl_csr_size(None, None, None) == 1


def test_python_binding_imports():
    import paper_2203_04774_amd as tl
    assert set(tl.ALGOS) == {"A++", "A+-", "A--"}


def test_tuning_keys_and_ranges(lib):
    """Tuning is host state: known keys take values in range, others are
    refused (plan_full stays below one long window of 256 items, which the
    heavy walk's unchecked bitmap reads rely on)."""
    lib.tl_set_tuning.argtypes = [ctypes.c_char_p, ctypes.c_uint64]
    lib.tl_get_tuning.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_uint64)]
    v = ctypes.c_uint64()
    assert lib.tl_get_tuning(b"plan_full", ctypes.byref(v)) == 0
    old = v.value
    assert lib.tl_set_tuning(b"plan_full", 255) == 0
    assert lib.tl_set_tuning(b"plan_full", 256) != 0
    assert lib.tl_get_tuning(b"plan_full", ctypes.byref(v)) == 0 and v.value == 255
    assert lib.tl_set_tuning(b"plan_full", old) == 0
    assert lib.tl_set_tuning(b"no_such_key", 1) != 0
    for key, bad in ((b"chunk_growth", 0), (b"chunk_growth", 65), (b"chunk_margin", 99), (b"chunk_task_div", 0),
                     (b"task_div", 1025), (b"light_wave_items", 63)):
        assert lib.tl_set_tuning(key, bad) != 0
    for key in (b"chunk_growth", b"chunk_margin", b"chunk_task_div", b"task_div", b"light_wave_items"):
        assert lib.tl_get_tuning(key, ctypes.byref(v)) == 0
        assert lib.tl_set_tuning(key, v.value) == 0
    assert lib.tl_set_tuning(b"batch_plan_full", 8) == 0
