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


def _comment_blocks():
    """Each declared function with the comment block written right above it
    (a declaration that directly follows another shares its block)."""
    text = open(HEADER).read()
    out = {}
    pending = ""
    for m in re.finditer(r"/\*(.*?)\*/|\b(sv_[a-z_0-9]+)\s*\(", text, flags=re.S):
        if m.group(1) is not None:
            pending = m.group(1)
        elif m.group(2) not in out:
            out[m.group(2)] = pending
    return out


def test_every_entry_point_cites_the_passage_that_defines_it():
    """Every exported computation names the section of the paper it follows;
    only the two diagnostics calls are library-defined, and say so."""
    blocks = _comment_blocks()
    names = declared_functions()
    assert set(blocks) >= set(names)
    for name in names:
        block = blocks[name]
        if name in ("sv_strerror", "sv_last_error"):
            assert "no passage of the paper" in block, name
            continue
        if name.endswith("_noalloc"):
            # the variant for callers that cannot allocate names those callers
            assert "cannot allocate" in block, name
            continue
        assert re.search(r"Sec\. (II|III|IV)(\.[A-F](\.\d)?)?", block), f"{name}: no section cited"
        assert name in block, f"{name}: its comment block does not name it"


def _plan_create_rc(n, ops, params):
    """sv_plan_create on host-validated input: argument checks run before any
    HIP call, so invalid ops are refused here without a device."""
    lib = sv.load_library()
    ops = np.ascontiguousarray(ops, dtype=OP_DTYPE)
    params = np.ascontiguousarray(params, dtype=np.float64)
    out = ctypes.c_void_p()
    return lib.sv_plan_create(n, sv.SV_C64, ops.ctypes.data, len(ops),
                              params.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(params), None,
                              ctypes.byref(out))


def test_out_of_range_ops_are_refused_before_any_launch():
    from paper_2606_12770_amd.circuits import ir
    n = 10
    params = np.zeros(8)

    def op(kind, target=0, width=0, mask=0, val=0, param=0):
        r = np.zeros(1, dtype=OP_DTYPE)
        r["kind"], r["target"], r["width"] = kind, target, width
        r["ctrl_mask"], r["ctrl_val"], r["param"] = mask, val, param
        return r

    bad = [
        op(ir.X, target=0xFFFFFFFF),                       # wraps to -1 as a signed int
        op(ir.X, target=1 << 31),
        op(ir.U, target=1 << 31),
        op(ir.PHASE, target=3, param=0xFFFFFFFFFFFFFFFF),  # param + count wraps around
        op(ir.U, target=3, param=(1 << 64) - 4),
        op(ir.U, target=3, param=1),                       # needs params[1..9): one past the pool
        op(ir.INC, target=0xFFFFFFFE, width=4),            # target + width wraps around
        op(ir.INC, target=8, width=3),                     # register past the last qubit
        op(ir.SWAP, target=2, width=0xFFFFFFFF),
        op(ir.SWAP, target=1 << 31, width=2),
        op(ir.X, target=2, mask=1 << 10),                  # control qubit >= n
        op(ir.X, target=2, mask=1, val=2),                 # value outside the mask
    ]
    for rec in bad:
        assert _plan_create_rc(n, rec, params) == sv.SV_EINVAL, rec
        assert sv.sv_last_error()
    assert _plan_create_rc(n, op(ir.U, target=3, param=0), params) != sv.SV_EINVAL


def test_unknown_option_values_are_refused_on_the_host():
    from paper_2606_12770_amd.circuits import ir
    lib = sv.load_library()
    r = np.zeros(1, dtype=OP_DTYPE)
    r["kind"], r["target"] = ir.X, 1
    params = np.zeros(1)
    for field, value in (("split_real", 3), ("split_real", -1), ("peephole", 5), ("compile", 7)):
        o = sv._opts()
        setattr(o, field, value)
        out = ctypes.c_void_p()
        rc = lib.sv_plan_create(4, sv.SV_C64, r.ctypes.data, 1, params.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                1, ctypes.byref(o), ctypes.byref(out))
        assert rc == sv.SV_EINVAL, (field, value)
        assert field.split("_")[0] in sv.sv_last_error(), sv.sv_last_error()


def test_sequence_entries_are_checked_against_the_plan_count():
    lib = sv.load_library()
    plans = (ctypes.c_void_p * 1)(None)
    for bad in ([1], [-1], [0, 5]):
        seq = np.asarray(bad, dtype=np.int32)
        rc = lib.sv_plan_execute_seq(plans, 1, seq.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), len(seq), None)
        assert rc == sv.SV_EINVAL
        assert "outside the plan array" in sv.sv_last_error()


def test_binding_structs_match_header(tmp_path):
    """sv_apply_opts and sv_plan_info: the ctypes mirrors have the header's
    size and every field at the header's offset (a C probe compiled here)."""
    structs = {"sv_apply_opts": sv.sv_apply_opts, "sv_plan_info": sv.sv_plan_info}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "sv.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines.append("return 0; }")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for name, cls in structs.items():
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert got[(name, field)] == getattr(cls, field).offset, (name, field)
