"""The C ABI library: it loads without a GPU and exports every function that
include/sv.h declares; the Python binding names the same set; the op record
layout matches between the IR and the header.  No compute calls here."""
import ctypes
import os
import re
import subprocess

import numpy as np

from paper_2606_12770_amd import sv
from paper_2606_12770_amd.circuits.ir import OP_DTYPE

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sv.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sv_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = sv.load_library()
    names = declared_functions()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), f"{name} declared in sv.h but not exported"
    out = subprocess.run(["nm", "-D", "--defined-only", sv.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (sv_[a-z_0-9]+)$", out, flags=re.M))
    assert set(names) <= exported
    # nothing exported under the sv_ prefix that the header does not declare
    assert exported <= set(names), exported - set(names)


def test_binding_covers_header():
    assert sorted(sv.EXPORTED) == declared_functions()


def test_op_record_layout_matches_header():
    text = open(HEADER).read()
    fields = re.search(r"typedef struct \{(.*?)\} sv_op;", text, flags=re.S).group(1)
    names = re.findall(r"(uint32_t|uint64_t)\s+(\w+);", fields)
    assert [n for _t, n in names] == list(OP_DTYPE.names)
    sizes = {"uint32_t": 4, "uint64_t": 8}
    assert sum(sizes[t] for t, _n in names) == OP_DTYPE.itemsize == 40
    # kind codes agree
    codes = dict(re.findall(r"#define (SV_OP_[A-Z]+)\s+(\d+)", text))
    from paper_2606_12770_amd.circuits import ir
    for name, val in codes.items():
        assert getattr(ir, name[len("SV_OP_"):]) == int(val)


def test_error_strings_without_device():
    lib = sv.load_library()
    assert lib.sv_strerror(0).decode() == "ok"
    assert "zero-probability" in lib.sv_strerror(-3).decode()
    assert lib.sv_strerror(-99).decode() == "unknown error"
