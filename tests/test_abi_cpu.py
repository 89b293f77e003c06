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


# ctypes mirrors in the binding and the C structs they stand for
MIRRORS = {
    "Summary": "tl_summary",
    "NeighResult": "tl_neigh_result",
    "ServerConfig": "tl_server_config",
    "Job": "tl_job",
    "JobResult": "tl_job_result",
    "ServerStats": "tl_server_stats",
    "ListStats": "tl_list_stats",
}


def c_layouts(tmp_path):
    """sizeof and offsetof of every mirrored struct, from a C program compiled
    against include/tl.h with the host compiler."""
    import shutil
    import subprocess
    import sys
    sys.path.insert(0, ROOT)
    import paper_2203_04774_amd.tl as b
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "tl.h"', "int main(void) {"]
    for py, c in MIRRORS.items():
        lines.append(f'printf("{py} size %zu\\n", sizeof({c}));')
        # offsets of the C fields named like the mirror's (arrays are flattened
        # in the mirrors: mode_items[7] -> items_bitmap ... items_split)
        for name, _ in getattr(b, py)._fields_:
            if not name.startswith("items_"):
                lines.append(f'printf("{py} {name} %zu\\n", offsetof({c}, {name}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    return b, [line.split() for line in out.splitlines()]


def test_binding_structs_match_the_header(tmp_path):
    """Every ctypes struct of the binding has the C struct's size and field
    offsets (a mirror that drifts would read or write the wrong bytes)."""
    b, rows = c_layouts(tmp_path)
    for py, what, val in rows:
        cls = getattr(b, py)
        if what == "size":
            assert ctypes.sizeof(cls) == int(val), (py, ctypes.sizeof(cls), val)
        else:
            assert getattr(cls, what).offset == int(val), (py, what)
