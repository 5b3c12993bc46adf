"""The C-ABI library loads and exports every function include/*.h declares;
argument errors come back synchronously before any launch (no GPU needed)."""
import ctypes
import glob
import os
import re

import pytest

import paper_1905_13415_amd as pp
from datagen import dialects as D

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(pp_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_function():
    names = _declared_functions()
    assert {"pp_parse", "pp_workspace_size", "pp_status_str"} <= names
    lib = pp.lib()
    for name in sorted(names):
        assert hasattr(lib, name), name


def test_no_oracle_in_product_library():
    out = os.popen(f"nm -D --defined-only {pp.LIB_PATH}").read()
    assert "orc_" not in out


def test_workspace_size_and_status_text():
    head = 256 + 4096  # ticket counter, byte tables
    head += 64 * 32  # column descriptors
    assert pp.workspace_size(0) == head
    assert pp.workspace_size(32768) == head + 8 * 8          # default: 512 threads x 64 B
    assert pp.workspace_size(32769) == head + 2 * 8 * 8
    assert pp.workspace_size(1 << 20, pp.options(16, 256)) == head + 256 * 8 * 8
    assert pp.workspace_size(1 << 20, pp.options(48, 256)) == 0
    assert pp.lib().pp_status_str(0) == b"ok"
    assert pp.lib().pp_status_str(-2) == b"invalid DFA"


def _call(dfa_struct, n=16, ncols=1, types=(0,), ws=1 << 20, in_ptr=0x1000, opts=None):
    L = pp.lib()
    t = (ctypes.c_int32 * max(ncols, 1))(*types)
    sch = pp.PpSchema(ncols, ctypes.cast(t, ctypes.c_void_p))
    fake = ctypes.c_void_p(0x2000)
    ptrs = (ctypes.c_void_p * 64)(*([0x3000] * 64))
    out = pp.PpOutputs(4, 4, 0x4000, 0x5000, 0x6000, ctypes.cast(ptrs, ctypes.c_void_p),
                       ctypes.cast(ptrs, ctypes.c_void_p), ctypes.cast(ptrs, ctypes.c_void_p), 0x7000)
    return L.pp_parse(in_ptr, n, ctypes.byref(dfa_struct), ctypes.byref(sch), ctypes.byref(out),
                      fake, ws, ctypes.byref(opts) if opts else None, None)


def test_argument_errors_are_synchronous():
    good = pp.dfa_struct(D.csv4())
    bad = pp.dfa_struct(D.csv4())
    bad.start_state = 4
    assert _call(bad) == -2
    bad = pp.dfa_struct(D.csv4())
    bad.next[1][2] = 7  # next state out of range
    assert _call(bad) == -2
    bad = pp.dfa_struct(D.paper6())
    bad.next[0][5] = 0  # invalid state must absorb
    assert _call(bad) == -2
    bad = pp.dfa_struct(D.csv4())
    bad.group_of[65] = 9  # group out of range
    assert _call(bad) == -2
    assert _call(good, ncols=65, types=[0] * 65) == -3
    assert _call(good, types=(9,)) == -3
    assert _call(good, ws=8) == -4
    assert _call(good, n=-1) == -1
    assert _call(good, in_ptr=None) == -1
    assert _call(good, opts=pp.options(48, 256)) == -1
    assert _call(good, opts=pp.options(32, 128)) == -1
    assert _call(good, opts=pp.options(64, 1024)) == -1
