"""Specialised tile-pass sources, checked on the host.

The planner's passes for circuits that reach every op kind (controlled
single-qubit matrices, real rotations, X on register and thread bits, phases,
projector phases with the signal on tile, register or thread bits,
increments, decrements, swaps and X flips on exchanges), both precisions,
register widths 4 and 5, tile sizes 10 to 13, gate runs of the Carleman
value encodings (from 21 qubits) and the benchmark circuit at 28 qubits are
turned into kernel sources and compiled for gfx950 with hiprtc.  No device
is needed; running them is the GPU tests' job (tests/test_gpu_compiled.py).
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from paper_2606_12770_amd.circuits.random_circuit import random_layered_circuit, random_mixed_circuit

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2606_12770_amd", "csrc")
OUT = os.path.join(ROOT, "_build", "libjit_check.so")


@pytest.fixture(scope="module")
def jit():
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-fPIC", "-shared", "-D__HIP_PLATFORM_AMD__",
                           "-I/opt/rocm/include", "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", OUT,
                           os.path.join(CSRC, "planner.cpp"), os.path.join(CSRC, "tile_codegen.cpp"),
                           os.path.join(ROOT, "tests", "csrc", "jit_check.cpp"),
                           "-L/opt/rocm/lib", "-lhiprtc", "-Wl,-rpath,/opt/rocm/lib"])
    L = ctypes.CDLL(OUT)
    L.jit_check.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t,
                            ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                            ctypes.c_char_p, ctypes.c_char_p]
    L.jit_check.restype = ctypes.c_int
    return L


def compile_circuit(L, circ, dtype, b=12, rb=4, persistent=0):
    ops, params = circ.arrays()
    params = np.ascontiguousarray(params, dtype=np.float64)
    rc = L.jit_check(circ.n, dtype, ops.ctypes.data, len(ops), params.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                     b, rb, persistent, None, None)
    assert rc > 0, f"generated source did not compile (code {rc})"
    return rc


@pytest.mark.parametrize("n,b,rb", [(14, 12, 4), (15, 12, 5), (13, 10, 4), (16, 13, 5), (12, 11, 5), (15, 13, 4)])
@pytest.mark.parametrize("dtype", [0, 1])
def test_mixed_circuits_compile(jit, n, b, rb, dtype):
    if dtype == 1 and b == 13:
        b = 12
    compile_circuit(jit, random_mixed_circuit(n, 250, seed=n + b + rb, max_ctrl=5), dtype, b, rb)


@pytest.mark.parametrize("dtype", [0, 1])
def test_carleman_ladder_with_gate_runs_compiles(jit, dtype):
    from paper_2606_12770_amd.circuits import carleman_circuit as cc
    cfg = cc.CarlemanConfig(nx=8, tau=1.0, nk=2, nt=2, dt=0.1, amp=0.05)
    enc = cc.build_ul(cfg)
    circ = cc.build_qsvt(enc, np.random.default_rng(3).uniform(-np.pi, np.pi, 4))
    k = compile_circuit(jit, circ, dtype)
    # the ladder repeats U_L and U_L^dagger: far fewer distinct kernels than passes
    assert k < 60


@pytest.mark.parametrize("persistent", [0, 1])
@pytest.mark.parametrize("b,rb", [(12, 4), (13, 4)])
def test_benchmark_circuit_compiles(jit, persistent, b, rb):
    compile_circuit(jit, random_layered_circuit(28, 3, seed=0), 0, b, rb, persistent=persistent)


@pytest.mark.parametrize("dtype", [0, 1])
def test_persistent_form_compiles(jit, dtype):
    compile_circuit(jit, random_mixed_circuit(16, 250, seed=9, max_ctrl=5), dtype, 12, 4, persistent=1)


@pytest.mark.parametrize("b,rb", [(12, 4), (13, 4)])
def test_split_real_gates_compile(jit, tmp_path, b, rb):
    """Complex64 plans with SV_SPLIT_REAL_ON emit their real 2x2 gates as
    hi + lo calls (gur2) and compile; with SV_SPLIT_REAL_OFF the same circuit
    emits none."""
    c = random_mixed_circuit(15, 250, seed=31, max_ctrl=5)
    ops, params = c.arrays()
    params = np.ascontiguousarray(params, dtype=np.float64)
    jit.jit_check_set_split_real.argtypes = [ctypes.c_int]
    jit.jit_check_set_split_real.restype = None
    counts = {}
    for split in (1, 2):
        src = tmp_path / f"split{split}.hip"
        jit.jit_check_set_split_real(split)
        try:
            rc = jit.jit_check(c.n, 0, ops.ctypes.data, len(ops), params.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               b, rb, 0, str(src).encode(), None)
        finally:
            jit.jit_check_set_split_real(0)
        assert rc > 0, f"generated source did not compile (code {rc})"
        counts[split] = src.read_text().count("gur2(x[")
    assert counts[1] == 0 and counts[2] > 0, counts


def test_sources_compile_with_the_hip_compiler_command(jit, tmp_path):
    """The library compiles generated units with the ROCm HIP compiler in child
    processes (device code only, one code object); the same command line on a
    unit of the benchmark circuit's passes gives an AMD GPU ELF code object."""
    clang = "/opt/rocm/lib/llvm/bin/clang++"
    if not os.access(clang, os.X_OK):
        pytest.skip("no ROCm HIP compiler here")
    c = random_layered_circuit(28, 2, seed=0)
    ops, params = c.arrays()
    params = np.ascontiguousarray(params, dtype=np.float64)
    src = tmp_path / "unit_src.hip"
    rc = jit.jit_check(c.n, 0, ops.ctypes.data, len(ops), params.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                       12, 4, 0, str(src).encode(), None)
    assert rc > 0
    unit = tmp_path / "unit.hip"
    unit.write_text("#include <hip/hip_runtime.h>\n" + src.read_text())
    out = tmp_path / "unit.co"
    subprocess.check_call([clang, "-x", "hip", "--offload-arch=gfx950", "--offload-device-only",
                           "--no-gpu-bundle-output", "-O3", "-Xclang", "-target-feature", "-Xclang",
                           "-packed-fp32-ops", "-I/opt/rocm/include", "-c", str(unit), "-o", str(out)])
    head = out.read_bytes()[:20]
    assert head[:4] == b"\x7fELF"
    assert int.from_bytes(head[18:20], "little") == 224  # EM_AMDGPU
