"""Host-side tests of the fused planner.

The planner's tile programs are executed by a CPU emulation of the tile kernel
(tests/csrc/plan_emu.cpp, built here with g++ together with the planner
source) and compared with the FP64 reference simulator.  The emulation also
checks every global/LDS index for range and every exchange for collisions, so
a planner bug shows up here before any GPU run.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from oracle import statevector as osv
from paper_2606_12770_amd.circuits.random_circuit import (random_circuit_with_inverse_pairs, random_layered_circuit,
                                                          random_mixed_circuit, random_state)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2606_12770_amd", "csrc")
OUT = os.path.join(ROOT, "_build", "libplan_emu.so")


@pytest.fixture(scope="module")
def emu():
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    srcs = [os.path.join(CSRC, "planner.cpp"), os.path.join(ROOT, "tests", "csrc", "plan_emu.cpp")]
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-I", os.path.join(ROOT, "include"),
                           "-I", CSRC, "-o", OUT] + srcs)
    L = ctypes.CDLL(OUT)
    L.emu_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t,
                          ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                          ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_uint64), ctypes.c_int]
    L.emu_run.restype = ctypes.c_int
    return L


def run_emu(L, circ, psi0, mode=1, b=0, rb=0, dtype=0, dense_min_ops=0):
    ops, params = circ.arrays()
    psi = np.array(psi0, dtype=np.complex128, copy=True)
    stats = (ctypes.c_uint64 * 7)()
    dp = ctypes.POINTER(ctypes.c_double)
    rc = L.emu_run(circ.n, dtype, ops.ctypes.data, len(ops), params.ctypes.data_as(dp), mode, b, rb,
                   psi.ctypes.data_as(dp), stats, dense_min_ops)
    assert rc == 0, f"emulation check failed with code {rc}"
    return psi, list(stats)


@pytest.mark.parametrize("n,b,rb,seed", [(10, 10, 4, 0), (11, 10, 4, 1), (12, 12, 4, 2), (13, 12, 4, 3),
                                         (14, 12, 5, 4), (14, 11, 5, 5), (15, 12, 4, 6), (12, 11, 5, 7),
                                         (15, 13, 4, 8), (14, 13, 4, 9)])
def test_fused_plan_matches_oracle_mixed(emu, n, b, rb, seed):
    c = random_mixed_circuit(n, 400, seed=seed, max_ctrl=5)
    psi0 = random_state(n, seed)
    want = osv.run(c, psi0)
    got, stats = run_emu(emu, c, psi0, 1, b, rb)
    assert np.max(np.abs(got - want)) < 1e-12
    assert stats[1] >= 1


@pytest.mark.parametrize("n,b,rb", [(14, 12, 4), (16, 12, 4), (16, 13, 5), (17, 13, 4)])
def test_fused_plan_matches_oracle_layered(emu, n, b, rb):
    c = random_layered_circuit(n, 6, seed=n, n_mcx=10, max_ctrl=8, inc_width=6)
    want = osv.run(c)
    got, stats = run_emu(emu, c, osv.zero_state(n), 1, b, rb)
    assert np.max(np.abs(got - want)) < 1e-12
    # fusion must beat one launch per op by a wide margin
    assert stats[0] * 4 < len(c)


@pytest.mark.parametrize("dtype", [0, 1])
def test_fused_plan_matches_oracle_24q(emu, dtype):
    """At 24 qubits the planner widens resident sets with lookahead; the op
    order, register choice and plain split are those of the large states."""
    n = 24
    c = random_layered_circuit(n, 3, seed=5, n_mcx=10, max_ctrl=8, inc_width=6)
    psi0 = random_state(n, 6)
    want = osv.run(c, psi0)
    got, stats = run_emu(emu, c, psi0, 1, 12, 4, dtype)
    assert np.max(np.abs(got - want)) < 1e-12
    assert stats[1] * 4 < len(c)


def test_gate_runs_carleman_22q(emu):
    """From 21 qubits the planner sorts runs of ops that share a tile mask by
    tile value (the kernel then bisects for a tile's ops); the Carleman value
    encodings form such runs.  The 22-qubit ladder at d = 3 through the fused
    planner against the reference simulator, complex64 plan."""
    from paper_2606_12770_amd.circuits import carleman_circuit as cc
    cfg = cc.CarlemanConfig(nx=8, tau=1.0, nk=2, nt=2, dt=0.1, amp=0.05)
    enc = cc.build_ul(cfg)
    circ = cc.build_qsvt(enc, np.random.default_rng(3).uniform(-np.pi, np.pi, 4))
    psi0 = random_state(circ.n, 9)
    want = osv.run(circ, psi0)
    got, stats = run_emu(emu, circ, psi0, 1, 12, 4, 0)
    assert np.max(np.abs(got - want)) < 1e-12
    assert stats[5] > 0  # the plan holds gate runs


def test_plain_plan_matches_oracle(emu):
    n = 9
    c = random_mixed_circuit(n, 300, seed=11)
    psi0 = random_state(n, 12)
    got, stats = run_emu(emu, c, psi0, 0)
    assert np.max(np.abs(got - osv.run(c, psi0))) < 1e-12
    assert stats[0] == len(c) and stats[1] == 0


def test_wide_register_falls_back_to_plain_launch(emu):
    n = 14
    from paper_2606_12770_amd.circuits.ir import Circuit
    c = Circuit(n).h(0).inc(0, 13).h(3).dec(1, 12, {0: 1})
    psi0 = random_state(n, 3)
    got, stats = run_emu(emu, c, psi0, 1, 10, 4)
    assert np.max(np.abs(got - osv.run(c, psi0))) < 1e-12


@pytest.mark.parametrize("b,rb", [(10, 4), (12, 4), (13, 5)])
@pytest.mark.parametrize("elementary", [False, True])
def test_fused_plan_carleman_ladder(emu, b, rb, elementary):
    """The QSVT ladder of a small Carleman-LBM instance through the fused planner."""
    from paper_2606_12770_amd.circuits import carleman_circuit as cc
    cfg = cc.CarlemanConfig(nx=2, tau=0.9, nk=2, nt=2, dt=0.1, amp=0.1)
    enc = cc.build_ul(cfg)
    rng = np.random.default_rng(b)
    circ = cc.build_qsvt(enc, rng.uniform(-np.pi, np.pi, 4))
    if elementary:
        circ = cc.lower_to_elementary(circ)
    psi0 = random_state(circ.n, b + rb)
    want = osv.run(circ, psi0)
    got, stats = run_emu(emu, circ, psi0, 1, b, rb)
    assert np.max(np.abs(got - want)) < 1e-12
    assert stats[0] * 3 < len(circ)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_plain_split_matches_oracle(emu, seed):
    """A group of ops that is cheaper as plain launches (each sweeping only its
    controlled subspace) than as one tile pass goes to plain launches: here
    controlled increments of two 7-qubit registers that do not commute, so each
    would fill a pass of its own.  Uncontrolled layers stay in tile passes.
    The mixed plan must equal the reference simulator."""
    from paper_2606_12770_amd.circuits.ir import Circuit
    n = 20
    rng = np.random.default_rng(seed)
    c = Circuit(n)
    for layer in range(3):
        for q in range(n):
            c.ry(q, rng.uniform(-np.pi, np.pi))
        for _ in range(4):
            c.inc(13, 7, {int(q): int(rng.integers(2)) for q in (6, 8, 10, 12)})
            c.dec(6, 7, {int(q): int(rng.integers(2)) for q in (13, 15, 17, 19)})
        qs = rng.permutation(n)
        c.x(int(qs[0]), {int(q): int(rng.integers(2)) for q in qs[1:9]})
    psi0 = random_state(n, seed)
    want = osv.run(c, psi0)
    got, stats = run_emu(emu, c, psi0, 1, 12, 4)
    assert np.max(np.abs(got - want)) < 1e-12
    assert stats[4] > 0 and stats[1] > 0  # some ops went to plain launches, some stayed in tile passes


@pytest.mark.parametrize("dtype,b,rb", [(0, 12, 4), (0, 12, 5), (0, 13, 5), (0, 13, 4), (1, 12, 4), (1, 11, 5),
                                        (1, 13, 4)])
def test_precomputed_pass_fields_at_benchmark_size(emu, dtype, b, rb):
    """Run maps, swizzle tables and LDS addressing of every pass of the
    28-qubit benchmark circuit (first 20 layers), checked without emulation."""
    c = random_layered_circuit(28, 20, seed=0)
    ops, params = c.arrays()
    emu.emu_check_fields.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t,
                                     ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_int]
    emu.emu_check_fields.restype = ctypes.c_int
    rc = emu.emu_check_fields(28, dtype, ops.ctypes.data, len(ops),
                              params.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), b, rb)
    assert rc == 0


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("n,seed", [(12, 0), (14, 1), (16, 2)])
def test_dense_blocks_match_oracle(emu, n, seed, dtype):
    from paper_2606_12770_amd.circuits.random_circuit import random_dense_block_circuit
    c = random_dense_block_circuit(n, 4, 5, seed)
    psi0 = random_state(n, seed)
    want = osv.run(c, psi0)
    got, stats = run_emu(emu, c, psi0, 1, 12, 4, dtype, dense_min_ops=16)
    assert np.max(np.abs(got - want)) < 1e-12
    assert stats[0] >= stats[1] + 4  # the four deep runs became dense passes
    # without dense blocks the same plan path agrees too
    got2, _ = run_emu(emu, c, psi0, 1, 12, 4, dtype, dense_min_ops=0)
    assert np.max(np.abs(got2 - want)) < 1e-12


@pytest.mark.parametrize("n,seed", [(12, 0), (14, 1), (17, 2)])
def test_six_qubit_dense_blocks_match_oracle(emu, n, seed):
    """dense_qubits = 6: runs confined to six qubits become 64 x 64 blocks
    (64 groups of 64 amplitudes per tile); the emulated plan matches the oracle,
    and complex128 plans refuse six-qubit blocks."""
    from paper_2606_12770_amd.circuits.random_circuit import random_dense_block_circuit
    c = random_dense_block_circuit(n, 4, 5, seed, width=6)
    psi0 = random_state(n, seed)
    want = osv.run(c, psi0)
    emu.emu_set_dense_qubits(6)
    try:
        got, stats = run_emu(emu, c, psi0, 1, 12, 4, 0, dense_min_ops=16)
        assert np.max(np.abs(got - want)) < 1e-12
        assert stats[0] >= stats[1] + 4  # the four deep runs became dense passes
        ops, params = c.arrays()
        buf = np.array(psi0, dtype=np.complex128)
        dp = ctypes.POINTER(ctypes.c_double)
        rc = emu.emu_run(c.n, 1, ops.ctypes.data, len(ops), params.ctypes.data_as(dp), 1, 12, 4,
                         buf.ctypes.data_as(dp), None, 16)
        assert rc == -5  # SV_EUNSUPPORTED
    finally:
        emu.emu_set_dense_qubits(0)
    # the same circuit with five-qubit blocks
    got, stats = run_emu(emu, c, psi0, 1, 12, 4, 0, dense_min_ops=16)
    assert np.max(np.abs(got - want)) < 1e-12


def _rotation_ladder(count, seed=3):
    """Controlled rotations of five repeated angles (a value-load pattern),
    with an X now and then; returns the circuit and the bound the planner's
    SV_SPLIT_REAL_AUTO compares with 1e-4 (per gate, the largest change of a
    column's squared norm under nearest FP32 rounding)."""
    from paper_2606_12770_amd.circuits.ir import Circuit
    n = 10
    angles = [0.483873, -0.240160, 0.159892, 1.047198, -0.0468790]
    rng = np.random.default_rng(seed)
    c = Circuit(n)
    bound = 0.0
    for k in range(count):
        th = angles[k % len(angles)]
        t = int(rng.integers(n))
        ctl = {(t + 1 + j) % n: int(rng.integers(2)) for j in range(int(rng.integers(0, 4)))}
        c.ry(t, th, ctl)
        cs, sn = np.float32(np.cos(th / 2)), np.float32(np.sin(th / 2))
        bound += abs(float(cs) ** 2 + float(sn) ** 2 - 1.0)
        if k % 5 == 4:
            xt = int(rng.integers(n))
            c.x(xt, {(xt + 1 + int(rng.integers(n - 1))) % n: 1} if k % 2 else None)
    return c, bound


def _run_rounded(emu, c, psi0, mode, split):
    emu.emu_set_param_rounding.argtypes = [ctypes.c_int]
    emu.emu_set_param_rounding.restype = None
    emu.emu_set_split_real.argtypes = [ctypes.c_int]
    emu.emu_set_split_real.restype = None
    emu.emu_set_param_rounding(1)
    emu.emu_set_split_real(split)
    try:
        got, _ = run_emu(emu, c, psi0, mode, 10, 4, 0)
    finally:
        emu.emu_set_param_rounding(0)
        emu.emu_set_split_real(0)
    return got


def test_complex64_real_gates_carry_their_remainder(emu):
    """A block-encoding call applies the same value-load rotations to the same
    controlled subspaces every time, so a rotation whose FP32 (cos, sin) has
    c^2 + s^2 != 1 drains or inflates its subspace by the same fraction in each
    call.  With the parameters rounded as the library uploads them, 6,000
    controlled rotations of five repeated angles: tile passes with
    SV_SPLIT_REAL_ON (hi + lo entries, each to about 2^-48, 3.6e-15, a gate)
    and plain launches (always hi + lo) keep the norm to 2e-11 and match the
    FP64 result to 1e-12; with SV_SPLIT_REAL_OFF the nearest FP32 entries move
    the norm by more than 1e-6."""
    c, bound = _rotation_ladder(6000)
    psi0 = random_state(c.n, 9)
    want = osv.run(c, psi0)
    for mode, split, exact in ((1, 2, True), (0, 0, True), (1, 1, False)):
        got = _run_rounded(emu, c, psi0, mode, split)
        drift = abs(np.vdot(got, got).real - 1.0)
        err = np.max(np.abs(got - want))
        print(f"mode {mode} split_real {split}: norm drift {drift:.2e}, max error {err:.2e}")
        if exact:
            assert drift < 2e-11
            assert err < 1e-12
        else:
            assert drift > 1e-6


@pytest.mark.parametrize("n,b,rb", [(14, 12, 4), (15, 13, 4), (14, 12, 5), (13, 10, 4)])
def test_split_real_plans_match_oracle(emu, n, b, rb):
    """Plans with SV_SPLIT_REAL_ON at several geometries (512-thread tiles
    included): in FP64 emulation (parameters unrounded) the state matches the
    oracle to 1e-12, the same as without the split."""
    c = random_mixed_circuit(n, 400, seed=3 * n + b, max_ctrl=5)
    psi0 = random_state(n, n)
    want = osv.run(c, psi0)
    emu.emu_set_split_real.argtypes = [ctypes.c_int]
    emu.emu_set_split_real.restype = None
    emu.emu_set_split_real(2)
    try:
        got, _ = run_emu(emu, c, psi0, 1, b, rb, 0)
    finally:
        emu.emu_set_split_real(0)
    assert np.max(np.abs(got - want)) < 1e-12


def test_split_real_auto_follows_the_norm_bound(emu):
    """SV_SPLIT_REAL_AUTO splits the real gates of a complex64 plan exactly when
    the summed FP32 column-norm errors of its real gates exceed 1e-4: the
    emulated state is then bit for bit that of SV_SPLIT_REAL_ON, else that of
    SV_SPLIT_REAL_OFF."""
    for count in (300, 12000):
        c, bound = _rotation_ladder(count, seed=4)
        psi0 = random_state(c.n, 10)
        auto = _run_rounded(emu, c, psi0, 1, 0)
        on = _run_rounded(emu, c, psi0, 1, 2)
        off = _run_rounded(emu, c, psi0, 1, 1)
        assert not np.array_equal(on, off)
        print(f"{count} rotations: bound {bound:.2e}")
        assert np.array_equal(auto, on if bound > 1e-4 else off)
        assert (bound > 1e-4) == (count == 12000)


def test_complex64_projector_phases_keep_the_norm(emu):
    """A QSVT sequence applies one projector phase per step, each with its own
    angle, and every such gate multiplies the whole state by c^2 + s^2 once
    (cos, sin) are rounded to FP32.  Rounded to nearest, the factors of 20,000
    random phases multiply to more than 1e-6 away from 1 (checked below).
    Complex64 plans round each pair within one ulp of the nearest so that the
    running product stays next to 1: with the plan's parameters rounded as the
    library uploads them the norm holds to 1e-7, and no amplitude moves further
    from the FP64 result than the angle bound allows (half an ulp of each
    entry, summed over the phases)."""
    from paper_2606_12770_amd.circuits.ir import Circuit
    n, count = 10, 20000
    rng = np.random.default_rng(11)
    c = Circuit(n)
    thetas = rng.uniform(-np.pi, np.pi, count)
    for k, th in enumerate(thetas):
        sig = int(rng.integers(n))
        mask = int(rng.integers(1 << n)) & ~(1 << sig)
        val = int(rng.integers(1 << n)) & mask
        c.projphase(sig, mask, val, float(th))
        if k % 7 == 0:
            t = int(rng.integers(n))
            c.x(t, {(t + 1) % n: 1})
    cn = np.cos(thetas).astype(np.float32).astype(np.float64)
    sn = np.sin(thetas).astype(np.float32).astype(np.float64)
    nearest_drift = abs(np.prod(cn * cn + sn * sn) - 1.0)
    assert nearest_drift > 1e-6
    ulp_c = np.spacing(np.abs(cn).astype(np.float32)).astype(np.float64)
    ulp_s = np.spacing(np.abs(sn).astype(np.float32)).astype(np.float64)
    angle_bound = np.sum(np.maximum(0.5 * (np.abs(np.sin(thetas)) * ulp_c + np.abs(np.cos(thetas)) * ulp_s),
                                    np.abs(np.cos(thetas) * (sn - np.sin(thetas))
                                           - np.sin(thetas) * (cn - np.cos(thetas)))))
    psi0 = random_state(n, 5)
    want = osv.run(c, psi0)
    emu.emu_set_param_rounding.argtypes = [ctypes.c_int]
    emu.emu_set_param_rounding.restype = None
    emu.emu_set_param_rounding(1)
    try:
        got, stats = run_emu(emu, c, psi0, 1, 10, 4, 0)
    finally:
        emu.emu_set_param_rounding(0)
    drift = abs(np.vdot(got, got).real - 1.0)
    err = np.max(np.abs(got - want))
    print(f"norm drift {drift:.2e} (nearest rounding {nearest_drift:.2e}); max error {err:.2e}, "
          f"angle bound {angle_bound:.2e}")
    assert stats[1] >= 1
    assert drift < 1e-7
    assert err < angle_bound + 1e-7


@pytest.mark.parametrize("mode", [0, 1])
def test_complex64_hadamards_keep_the_norm(emu, mode):
    """Uncontrolled Hadamards stored as fp32(1/sqrt 2) would each shrink the
    state by 1.7e-8 (the rounding of 1/sqrt 2, always downward); complex64
    plans store them in exact pairs (sqrt 2 H, H / sqrt 2).  With the plan's
    parameters rounded to float as the library uploads them, 4,000 Hadamards
    (interleaved with CNOTs so that none fold together) keep the norm to
    1e-12, where the rounded matrix alone would lose 1.4e-4; with an odd
    count, the one left over costs its single 3.4e-8 in a tile pass (a plain
    launch carries its matrix as hi + lo and loses nothing)."""
    from paper_2606_12770_amd.circuits.ir import Circuit
    n = 12
    emu.emu_set_param_rounding.argtypes = [ctypes.c_int]
    emu.emu_set_param_rounding.restype = None
    for extra in (0, 1):
        c = Circuit(n)
        for layer in range(4000 // n):
            for q in range(n):
                c.h(q)
            for q in range(n):
                c.x((q + 1 + layer) % n, {q: 1})
        for q in range(4000 - (4000 // n) * n + extra):
            c.h(q)
        n_h = sum(1 for r in c.arrays()[0] if r["kind"] == 0)
        assert n_h == 4000 + extra
        psi0 = random_state(n, 2)
        want = osv.run(c, psi0)
        emu.emu_set_param_rounding(1)
        try:
            got, _ = run_emu(emu, c, psi0, mode, 12, 4, 0)
        finally:
            emu.emu_set_param_rounding(0)
        drift = abs(np.vdot(got, got).real - 1.0)
        print(f"mode {mode}: {n_h} Hadamards, norm drift {drift:.2e}")
        assert drift < (1e-12 if extra == 0 else 1e-7)
        assert np.max(np.abs(got - want)) < 1e-12 + extra * 1e-7
        # without the pairing the rounded Hadamard loses this much per gate
        h32 = np.float32(1 / np.sqrt(2))
        assert 1.0 - 2 * float(h32) ** 2 > 3e-8



def test_dense_blocks_chosen_by_cost(emu):
    """With a negative dense_min_ops the planner's cost model sets the run
    length that makes a dense block: at 20 qubits the deep five-qubit runs of
    the dense-block circuit qualify, the random layered circuit's short runs
    do not; both plans still match the oracle."""
    from paper_2606_12770_amd.circuits.random_circuit import random_dense_block_circuit
    n = 20
    c = random_dense_block_circuit(n, 3, 12, 2)
    psi0 = random_state(n, 5)
    got, stats = run_emu(emu, c, psi0, 1, 12, 4, 0, dense_min_ops=-1)
    assert np.max(np.abs(got - osv.run(c, psi0))) < 1e-12
    assert stats[0] > stats[1]  # dense passes among the launches
    layered = random_layered_circuit(n, 3, seed=2)
    got, stats = run_emu(emu, layered, osv.zero_state(n), 1, 12, 4, 0, dense_min_ops=-1)
    assert np.max(np.abs(got - osv.run(layered))) < 1e-12
    assert stats[0] == stats[1] + stats[4]  # tile passes and split plain launches only


@pytest.mark.parametrize("mode,n,seed", [(1, 13, 0), (1, 14, 1), (0, 10, 2), (0, 12, 3)])
def test_peephole_cancels_inverse_pairs(emu, mode, n, seed):
    """Sec. III.F.2's peephole pass: adjacent inverse pairs are dropped (their
    count exactly as spliced in), the decoys stay, and the planned circuit still
    matches the oracle's run of the full op list."""
    c, expect = random_circuit_with_inverse_pairs(n, seed)
    psi0 = random_state(n, seed + 7)
    want = osv.run(c, psi0)
    emu.emu_set_peephole(2)
    try:
        got, stats = run_emu(emu, c, psi0, mode, 12 if mode else 0, 4 if mode else 0)
    finally:
        emu.emu_set_peephole(0)
    assert np.max(np.abs(got - want)) < 1e-12
    assert stats[6] == expect
    if mode == 0:
        assert stats[0] == len(c) - expect  # one launch per remaining op
    emu.emu_set_peephole(1)
    try:
        got, stats = run_emu(emu, c, psi0, mode, 12 if mode else 0, 4 if mode else 0)
    finally:
        emu.emu_set_peephole(0)
    assert np.max(np.abs(got - want)) < 1e-12
    assert stats[6] == 0


def test_peephole_default_follows_mode(emu):
    """SV_PEEPHOLE_AUTO: on in fused plans, off in plain ones."""
    c, expect = random_circuit_with_inverse_pairs(12, 4)
    psi0 = random_state(12, 3)
    _, fused = run_emu(emu, c, psi0, 1, 12, 4)
    _, plain = run_emu(emu, c, psi0, 0)
    assert fused[6] == expect and plain[6] == 0 and plain[0] == len(c)


def test_peephole_on_first_order_ladder(emu):
    """On a first-order QSVT ladder the X pairs where one U_L call meets the
    next are dropped, and the result is unchanged."""
    from paper_2606_12770_amd.circuits import carleman_circuit as cc
    cfg = cc.CarlemanConfig(nx=8, order=1, nk=1)
    enc = cc.build_ul(cfg)
    c = cc.build_qsvt(enc, np.linspace(0.1, 0.5, 6))
    psi0 = random_state(c.n, 11)
    want = osv.run(c, psi0)
    got, stats = run_emu(emu, c, psi0, 1, 12, 4)
    assert np.max(np.abs(got - want)) < 1e-12
    assert stats[6] > 0


@pytest.mark.parametrize("coalesce", [1, 3, 4, 6, 8])
@pytest.mark.parametrize("dtype", [0, 1])
def test_coalesce_width_matches_oracle(emu, coalesce, dtype):
    """sv_apply_opts.coalesce_qubits: plans keeping 1 to 8 lowest qubits
    resident in every pass match the oracle (the emulation also checks every
    pass's load mapping and LDS addressing)."""
    n = 16
    c = random_layered_circuit(n, 6, seed=n, n_mcx=10, max_ctrl=8, inc_width=6)
    want = osv.run(c)
    emu.emu_set_coalesce_qubits(coalesce)
    try:
        got, stats = run_emu(emu, c, osv.zero_state(n), 1, 12, 4, dtype)
    finally:
        emu.emu_set_coalesce_qubits(0)
    assert np.max(np.abs(got - want)) < 1e-12
    assert stats[1] >= 1
