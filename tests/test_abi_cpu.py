"""CPU checks of the C-ABI boundary: the library loads, exports every entry
point the header declares, the header is valid C99, and the binding's
structure layouts match the header's."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "thapi_tally.h")


def declared_functions():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(thapi_tally_\w+)\s*\(", txt, re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2504_03683_amd import tally
    if not os.path.exists(tally.LIB_PATH):
        from paper_2504_03683_amd import build
        build.build()
    return tally.load()


def test_header_declares_the_boundary():
    from paper_2504_03683_amd import tally
    assert declared_functions() == sorted(tally.ENTRY_POINTS)


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", lib._name], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (thapi_tally_\w+)", out))
    for f in declared_functions():
        assert f in exported, f
        assert hasattr(lib, f)


def test_header_is_c99_and_layouts_match(tmp_path):
    src = tmp_path / "probe.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "thapi_tally.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(thapi_tally_config), sizeof(thapi_tally_row),
         sizeof(thapi_tally_stats), sizeof(thapi_stream_key), offsetof(thapi_tally_row, count),
         offsetof(thapi_tally_config, fn_has_size), offsetof(thapi_tally_config, hip_stream));
  return 0;
}
""")
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Werror", "-pedantic", "-I", os.path.join(ROOT, "include"),
                           str(src), "-o", str(exe)])
    vals = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    from paper_2504_03683_amd import tally
    assert vals[0] == ctypes.sizeof(tally.Config)
    assert vals[1] == tally.ROW_DTYPE.itemsize == 88
    assert vals[2] == ctypes.sizeof(tally.Stats)
    assert vals[3] == ctypes.sizeof(tally.StreamKey)
    assert vals[4] == tally.ROW_DTYPE.fields["count"][1]
    assert vals[5] == tally.Config.fn_has_size.offset
    assert vals[6] == tally.Config.hip_stream.offset


def test_strerror_and_argument_errors_without_gpu(lib):
    from paper_2504_03683_amd import tally
    for code in range(-9, 1):
        assert lib.thapi_tally_strerror(code)
    assert lib.thapi_tally_strerror(-99) == b"unknown status"
    # null config / bad ABI version are rejected before any device call
    h = ctypes.c_void_p()
    assert lib.thapi_tally_open(None, ctypes.byref(h)) == tally.E_INVAL
    c = tally.Config()
    c.abi_version = 999
    assert lib.thapi_tally_open(ctypes.byref(c), ctypes.byref(h)) == tally.E_INVAL
    # version 1 passed the stream key to submit by pointer; it is refused
    c.abi_version = 1
    c.format = 1
    c.n_fns = 10
    assert lib.thapi_tally_open(ctypes.byref(c), ctypes.byref(h)) == tally.E_INVAL
    c.abi_version = tally.ABI_VERSION
    c.format = 9
    assert lib.thapi_tally_open(ctypes.byref(c), ctypes.byref(h)) == tally.E_INVAL
    c.format = 1
    c.n_fns = 10
    c.max_depth = 65
    assert lib.thapi_tally_open(ctypes.byref(c), ctypes.byref(h)) == tally.E_INVAL
    assert lib.thapi_tally_flush(None, 0, 0) == tally.E_INVAL
    assert lib.thapi_tally_flush_noalloc(None, 0, 0) == tally.E_INVAL
    assert lib.thapi_tally_last_shape(None, None) == tally.E_INVAL
    assert lib.thapi_tally_close(None) == tally.E_INVAL


def test_package_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2504_03683_amd import tally
    monkeypatch.setattr(tally, "_lib", None)
    monkeypatch.setattr(tally, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        tally.load()


def test_service_with_graph_is_rejected_without_gpu(lib):
    """The streaming form cannot be combined with graph capture: open refuses
    it before touching the device."""
    from paper_2504_03683_amd import tally
    h = ctypes.c_void_p()
    c = tally.Config()
    c.abi_version = tally.ABI_VERSION
    c.format = 1
    c.n_fns = 4
    c.flags = tally.SERVICE | tally.GRAPH
    assert lib.thapi_tally_open(ctypes.byref(c), ctypes.byref(h)) == tally.E_INVAL
    assert not h.value
