"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer.

The planner (with the CPU emulation of the launch steps) and the FP64
reference simulator are each built into a command-line driver with
-fsanitize=address,undefined (host compilers only; no GPU code is involved)
and run on circuits that reach every op kind, both plan modes, both
precisions' plans, dense blocks, gate runs and wide registers.  Any
out-of-bounds access, use after free, signed overflow or bad shift aborts the
driver; the states it writes must also match the unsanitized oracle.
"""
import os
import subprocess
import tempfile

import numpy as np
import pytest

from oracle import statevector as osv
from paper_2606_12770_amd.circuits.random_circuit import (random_dense_block_circuit, random_layered_circuit,
                                                          random_mixed_circuit, random_state)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2606_12770_amd", "csrc")
BUILD = os.path.join(ROOT, "_build", "sanitize")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
           OMP_NUM_THREADS="2")


@pytest.fixture(scope="module")
def drivers():
    os.makedirs(BUILD, exist_ok=True)
    plan = os.path.join(BUILD, "plan_driver")
    orc = os.path.join(BUILD, "oracle_driver")
    subprocess.check_call(["g++", "-std=c++17"] + SAN + ["-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", plan,
                           os.path.join(CSRC, "planner.cpp"), os.path.join(ROOT, "tests", "csrc", "plan_emu.cpp"),
                           os.path.join(ROOT, "tests", "csrc", "sanitize_driver.cpp")])
    subprocess.check_call(["gcc", "-std=c99", "-fopenmp"] + SAN + ["-o", orc,
                           os.path.join(ROOT, "oracle", "sv_oracle.c"),
                           os.path.join(ROOT, "tests", "csrc", "oracle_sanitize_driver.c"), "-lm"])
    return plan, orc


def run_case(exe, circ, psi0, dtype=0, mode=1, b=12, rb=4, dense_min_ops=0, env=None):
    ops, params = circ.arrays()
    with tempfile.TemporaryDirectory() as td:
        case, out = os.path.join(td, "case.bin"), os.path.join(td, "out.bin")
        with open(case, "wb") as f:
            np.asarray([circ.n, dtype, mode, b, rb, dense_min_ops], dtype=np.int32).tofile(f)
            np.asarray([len(ops), len(params)], dtype=np.uint64).tofile(f)
            np.ascontiguousarray(ops).tofile(f)
            np.ascontiguousarray(params, dtype=np.float64).tofile(f)
            np.ascontiguousarray(psi0, dtype=np.complex128).tofile(f)
        r = subprocess.run([exe, case, out], capture_output=True, text=True, env=dict(ENV, **(env or {})))
        assert r.returncode == 0, f"{os.path.basename(exe)} exited {r.returncode}\n{r.stderr[-4000:]}"
        assert "runtime error" not in r.stderr, r.stderr[-4000:]
        return np.fromfile(out, dtype=np.complex128)


CASES = [
    ("mixed-14q-fused-c64", lambda: random_mixed_circuit(14, 300, seed=1, max_ctrl=5), dict(dtype=0, b=12, rb=4)),
    ("mixed-13q-fused-c128-rb5", lambda: random_mixed_circuit(13, 300, seed=2, max_ctrl=5),
     dict(dtype=1, b=12, rb=5)),
    ("mixed-10q-plain", lambda: random_mixed_circuit(10, 200, seed=3, max_ctrl=5), dict(dtype=0, mode=0)),
    ("layered-16q", lambda: random_layered_circuit(16, 4, seed=4), dict(dtype=0, b=12, rb=4)),
    ("dense-14q", lambda: random_dense_block_circuit(14, 3, 5, 5), dict(dtype=1, b=12, rb=4, dense_min_ops=16)),
]


@pytest.mark.parametrize("name,make,kw", CASES, ids=[c[0] for c in CASES])
def test_planner_and_oracle_clean_under_sanitizers(drivers, name, make, kw):
    plan_exe, orc_exe = drivers
    circ = make()
    psi0 = random_state(circ.n, 17)
    want = osv.run(circ, psi0)
    got_orc = run_case(orc_exe, circ, psi0, **kw)
    assert np.max(np.abs(got_orc - want)) < 1e-13
    got_plan = run_case(plan_exe, circ, psi0, **kw)
    assert np.max(np.abs(got_plan - want)) < 1e-12


def test_carleman_gate_runs_clean_under_sanitizers(drivers):
    """A 22-qubit Carleman ladder (d = 3): its value encodings form the gate
    runs that the planner sorts from 21 qubits up (the run path of the planner)."""
    from paper_2606_12770_amd.circuits import carleman_circuit as cc
    cfg = cc.CarlemanConfig(nx=8, tau=1.0, nk=2, nt=2, dt=0.1, amp=0.05)
    enc = cc.build_ul(cfg)
    circ = cc.build_qsvt(enc, np.random.default_rng(5).uniform(-np.pi, np.pi, 4))
    assert circ.n >= 21, circ.n
    psi0 = random_state(circ.n, 3)
    want = osv.run(circ, psi0)
    got = run_case(drivers[0], circ, psi0, dtype=0, b=12, rb=4)
    assert np.max(np.abs(got - want)) < 1e-12


def test_complex64_parameter_rounding_clean_under_sanitizers(drivers):
    """The complex64 parameter conversion (projector phases rounded to a
    balanced product, real gates split into hi + lo) on a circuit with both,
    in the sanitized planner: the emulated state, computed in FP64 from the
    rounded parameters, stays within FP32 parameter error of the oracle."""
    from paper_2606_12770_amd.circuits.ir import Circuit
    rng = np.random.default_rng(8)
    n = 13
    c = random_mixed_circuit(n, 200, seed=9, max_ctrl=4)
    for k in range(300):
        sig = int(rng.integers(n))
        mask = int(rng.integers(1 << n)) & ~(1 << sig)
        c.projphase(sig, mask, int(rng.integers(1 << n)) & mask, float(rng.uniform(-np.pi, np.pi)))
        t = int(rng.integers(n))
        c.ry(t, float(rng.uniform(-np.pi, np.pi)), {(t + 1) % n: 1})
    psi0 = random_state(n, 4)
    want = osv.run(c, psi0)
    for split in ("1", "2"):
        got = run_case(drivers[0], c, psi0, dtype=0, b=12, rb=4,
                       env={"SAN_ROUND_PARAMS": "1", "SAN_SPLIT_REAL": split})
        err = np.max(np.abs(got - want))
        print(f"split_real {split}: max error {err:.2e}")
        assert err < 1e-5
