"""Compiled tile passes (sv_apply_opts.compile) on the GPU.

A compiled plan runs every tile pass as a kernel generated for that pass
(its op list written out as straight-line code) instead of the generic tile
kernel that reads the op records at run time.  The plan, and the arithmetic of
every op, are the same, so:
* compiled and generic runs of the same plan give bit-identical states
  (random circuits with every op kind, both precisions, register widths 4 and
  5, tile sizes 10 to 13; the 22-qubit Carleman ladder with its gate runs and
  projector phases; the first layers of the 28-qubit benchmark circuit);
* both agree with the FP64 reference simulator to the usual bars
  (complex128 1e-12; complex64 element-wise, 1e-5 of the largest amplitude
  per 1,000 gates); permutation-only circuits are bit-exact;
* automatic selection compiles plans of 21 qubits and more.
"""
import numpy as np
import pytest

from oracle import statevector as osv
from paper_2606_12770_amd.circuits.ir import Circuit
from paper_2606_12770_amd.circuits.random_circuit import random_layered_circuit, random_mixed_circuit, random_state
from tests.gpu_util import assert_c64_close, require_gpu

pytestmark = pytest.mark.gpu


def run(sv, circ, psi0, dtype, compile_mode, b=0, rb=0, split_real=0):
    ops, params = circ.arrays()
    plan = sv.sv_plan_create(circ.n, dtype, ops, params, sv.SV_MODE_FUSED, b, rb, compile=compile_mode,
                             split_real=split_real)
    info = sv.sv_plan_get_info(plan)
    st = sv.State(circ.n, dtype, psi0)
    sv.sv_plan_execute(plan, st.h, 1)
    out = st.amplitudes()
    st.close()
    sv.sv_plan_free(plan)
    return out, info


@pytest.mark.parametrize("n,b,rb", [(10, 10, 4), (13, 12, 4), (14, 12, 5), (16, 13, 5), (17, 11, 4), (19, 12, 4)])
@pytest.mark.parametrize("dtype", [0, 1])
def test_compiled_equals_generic_and_oracle(n, b, rb, dtype):
    sv = require_gpu()
    if dtype == 1 and b == 13:
        b = 12
    c = random_mixed_circuit(n, 400, seed=7 * n + b + rb + dtype, max_ctrl=6)
    psi0 = random_state(n, n + dtype)
    want = osv.run(c, psi0)
    got, info = run(sv, c, psi0, dtype, sv.SV_COMPILE_ON, b, rb)
    gen, info_g = run(sv, c, psi0, dtype, sv.SV_COMPILE_OFF, b, rb)
    print(f"n={n} b={b} rb={rb} dtype={dtype}: {info['n_tile_passes']} passes, {info['n_compiled_kernels']} "
          f"compiled kernels, max |compiled - generic| {np.max(np.abs(got - gen)):.1e}", flush=True)
    assert info["n_compiled_kernels"] > 0 and info_g["n_compiled_kernels"] == 0
    assert np.array_equal(got.view(np.uint64), gen.view(np.uint64))
    if dtype == 1:
        assert np.max(np.abs(got - want)) < 1e-12
    else:
        assert_c64_close(got, want, len(c), what=f"compiled n={n}")


@pytest.mark.parametrize("n,b,rb", [(13, 12, 4), (16, 13, 5), (19, 12, 4)])
def test_split_real_gates_compiled_equal_generic(n, b, rb):
    """SV_SPLIT_REAL_ON (complex64 real 2x2 gates as hi + lo FP32 entries):
    compiled passes and the generic kernel give bit-identical states, both
    within the complex64 bar of the oracle."""
    sv = require_gpu()
    c = random_mixed_circuit(n, 400, seed=5 * n + b, max_ctrl=6)
    psi0 = random_state(n, n + 3)
    want = osv.run(c, psi0)
    got, info = run(sv, c, psi0, 0, sv.SV_COMPILE_ON, b, rb, sv.SV_SPLIT_REAL_ON)
    gen, _ = run(sv, c, psi0, 0, sv.SV_COMPILE_OFF, b, rb, sv.SV_SPLIT_REAL_ON)
    assert info["n_compiled_kernels"] > 0
    assert np.array_equal(got.view(np.uint64), gen.view(np.uint64))
    assert_c64_close(got, want, len(c), what=f"split real n={n}")


def test_split_real_gates_keep_the_norm_of_a_rotation_ladder():
    """20,000 controlled rotations of five repeated angles (a value-load
    pattern) on 14 qubits in complex64.  With nearest FP32 entries
    (SV_SPLIT_REAL_OFF) each rotation scales its subspace by the same
    c^2 + s^2 every time and the norm drifts systematically; with hi + lo
    entries (SV_SPLIT_REAL_ON) only the FP32 arithmetic's drift is left, less
    than a fifth of it, and the amplitudes match the oracle at least as well."""
    sv = require_gpu()
    n = 14
    angles = [0.483873, -0.240160, 0.159892, 1.047198, -0.0468790]
    rng = np.random.default_rng(21)
    c = Circuit(n)
    for k in range(20000):
        t = int(rng.integers(n))
        ctl = {(t + 1 + j) % n: int(rng.integers(2)) for j in range(int(rng.integers(0, 3)))}
        c.ry(t, angles[k % len(angles)], ctl)
        if k % 5 == 4:
            xt = int(rng.integers(n))
            c.x(xt, {(xt + 1 + int(rng.integers(n - 1))) % n: 1})
    psi0 = random_state(n, 22)
    want = osv.run(c, psi0)
    res = {}
    for split in (sv.SV_SPLIT_REAL_OFF, sv.SV_SPLIT_REAL_ON):
        got, _ = run(sv, c, psi0, 0, sv.SV_COMPILE_AUTO, 12, 4, split)
        res[split] = (abs(np.vdot(got, got).real - 1.0), np.max(np.abs(got - want)))
        print(f"split_real {split}: norm drift {res[split][0]:.2e}, max error {res[split][1]:.2e}", flush=True)
    assert res[sv.SV_SPLIT_REAL_OFF][0] > 1e-5
    assert res[sv.SV_SPLIT_REAL_ON][0] < 0.2 * res[sv.SV_SPLIT_REAL_OFF][0]
    assert res[sv.SV_SPLIT_REAL_ON][1] <= res[sv.SV_SPLIT_REAL_OFF][1]


@pytest.mark.parametrize("dtype", [0, 1])
def test_compiled_permutations_bit_exact(dtype):
    sv = require_gpu()
    n = 16
    rng = np.random.default_rng(11)
    c = Circuit(n)
    for _ in range(200):
        k = int(rng.integers(0, 4))
        qs = [int(v) for v in rng.permutation(n)]
        ctrl = {q: int(rng.integers(0, 2)) for q in qs[2:2 + int(rng.integers(0, 4))]}
        if k == 0:
            c.x(qs[0], ctrl)
        elif k == 1:
            c.swap(qs[0], qs[1], ctrl)
        else:
            w = int(rng.integers(1, 9))
            base = int(rng.integers(0, n - w + 1))
            ctrl = {q: v for q, v in ctrl.items() if not base <= q < base + w}
            (c.inc if k == 2 else c.dec)(base, w, ctrl)
    psi0 = random_state(n, 12)
    if dtype == 0:
        psi0 = psi0.astype(np.complex64).astype(np.complex128)
    want = osv.run(c, psi0)
    got, info = run(sv, c, psi0, dtype, sv.SV_COMPILE_ON)
    assert info["n_compiled_kernels"] > 0
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))


@pytest.mark.parametrize("dtype", [0, 1])
def test_compiled_carleman_ladder_22q(dtype):
    """The C1 ladder at d = 13 (22 qubits): value-encoding gate runs become
    switches on the tile value, projector phases with the signal qubit on
    every kind of bit; automatic selection compiles it."""
    from paper_2606_12770_amd.circuits import carleman_circuit as cc
    from paper_2606_12770_amd.circuits import qsp
    sv = require_gpu()
    cfg = cc.CarlemanConfig(nx=8, tau=1.0, nk=2, nt=2, dt=0.1, amp=0.05)
    enc = cc.build_ul(cfg)
    circ = cc.build_qsvt(enc, qsp.inversion_phases(1.2, 13)[0])
    psi0 = np.zeros(1 << circ.n, dtype=np.complex128)
    psi0[: 1 << enc.layout.n_x] = cc.rhs_x_block(cfg, enc.layout)
    want = osv.run(circ, psi0)
    got, info = run(sv, circ, psi0, dtype, sv.SV_COMPILE_AUTO)
    gen, _ = run(sv, circ, psi0, dtype, sv.SV_COMPILE_OFF)
    print(f"C1 ladder dtype={dtype}: {info['n_tile_passes']} passes, {info['n_compiled_kernels']} compiled kernels",
          flush=True)
    assert info["n_compiled_kernels"] > 0
    assert info["n_compiled_kernels"] < info["n_tile_passes"]
    assert np.array_equal(got.view(np.uint64), gen.view(np.uint64))
    if dtype == 1:
        assert np.max(np.abs(got - want)) < 1e-12
    else:
        assert_c64_close(got, want, len(circ), what="compiled C1 ladder")


@pytest.mark.parametrize("dtype", [0, 1])
def test_compiled_benchmark_prefix_28q(dtype):
    """Two layers of the 28-qubit benchmark circuit, the benchmark's launch
    configuration: compiled equals generic bit for bit, and both the oracle."""
    sv = require_gpu()
    c = random_layered_circuit(28, 2, seed=0)
    want = osv.run(c)
    got, info = run(sv, c, osv.zero_state(28), dtype, sv.SV_COMPILE_AUTO)
    gen, _ = run(sv, c, osv.zero_state(28), dtype, sv.SV_COMPILE_OFF)
    assert info["n_compiled_kernels"] > 0
    assert np.array_equal(got.view(np.uint64), gen.view(np.uint64))
    if dtype == 1:
        assert np.max(np.abs(got - want)) < 1e-12
    else:
        assert_c64_close(got, want, len(c), what="compiled 28q prefix")


@pytest.mark.parametrize("n,b,rb", [(12, 12, 4), (18, 12, 4), (20, 11, 5), (26, 12, 4)])
@pytest.mark.parametrize("dtype", [0, 1])
def test_persistent_compiled_equals_grid_compiled(n, b, rb, dtype):
    """The persistent compiled form (resident workgroups walking the tiles, the
    next tile's loads in flight) gives the grid form's state bit for bit; at
    26 qubits each workgroup handles several tiles."""
    sv = require_gpu()
    c = random_mixed_circuit(n, 300, seed=3 * n + rb + dtype, max_ctrl=6)
    psi0 = random_state(n, 40 + n) if n <= 20 else osv.zero_state(n)
    ops, params = c.arrays()
    outs = []
    for form in (sv.SV_TILE_LAUNCH_PERSISTENT, sv.SV_TILE_LAUNCH_GRID):
        plan = sv.sv_plan_create(n, dtype, ops, params, sv.SV_MODE_FUSED, b, rb, tile_launch=form,
                                 compile=sv.SV_COMPILE_ON)
        assert sv.sv_plan_get_info(plan)["n_compiled_kernels"] > 0
        st = sv.State(n, dtype, psi0)
        sv.sv_plan_execute(plan, st.h, 1)
        outs.append(st.amplitudes())
        st.close()
        sv.sv_plan_free(plan)
    assert np.array_equal(outs[0].view(np.uint64), outs[1].view(np.uint64))
    if n <= 20:
        want = osv.run(c, psi0)
        if dtype == 1:
            assert np.max(np.abs(outs[0] - want)) < 1e-12
        else:
            assert_c64_close(outs[0], want, len(c), what=f"persistent compiled n={n}")


def test_invalid_compile_mode_is_refused():
    sv = require_gpu()
    c = random_mixed_circuit(14, 50, seed=1)
    ops, params = c.arrays()
    with pytest.raises(sv.SVError) as e:
        sv.sv_plan_create(14, 0, ops, params, sv.SV_MODE_FUSED, compile=7)
    assert e.value.code == sv.SV_EINVAL


@pytest.mark.parametrize("n,persistent", [(14, 0), (17, 0), (20, 0), (22, 1)])
@pytest.mark.parametrize("dtype", [0, 1])
def test_512_thread_tiles_match_oracle(n, persistent, dtype):
    """Geometry (13,4): 2^13 amplitudes per workgroup of 512 threads, 16 per
    thread, which only compiled passes run.  Every op kind against the
    oracle (complex128 to 1e-12, complex64 element-wise), in the grid and the
    persistent launch forms; the same plan without compilation is refused."""
    sv = require_gpu()
    c = random_mixed_circuit(n, 400, seed=11 * n + dtype, max_ctrl=6)
    psi0 = random_state(n, 70 + n)
    want = osv.run(c, psi0)
    ops, params = c.arrays()
    form = sv.SV_TILE_LAUNCH_PERSISTENT if persistent else sv.SV_TILE_LAUNCH_GRID
    plan = sv.sv_plan_create(n, dtype, ops, params, sv.SV_MODE_FUSED, 13, 4, tile_launch=form,
                             compile=sv.SV_COMPILE_ON)
    info = sv.sv_plan_get_info(plan)
    st = sv.State(n, dtype, psi0)
    sv.sv_plan_execute(plan, st.h, 1)
    got = st.amplitudes()
    st.close()
    sv.sv_plan_free(plan)
    print(f"(13,4) n={n} dtype={dtype} persistent={persistent}: {info['n_tile_passes']} passes, "
          f"max abs err {np.max(np.abs(got - want)):.2e}", flush=True)
    assert info["tile_qubits"] == 13 and info["reg_qubits"] == 4 and info["n_compiled_kernels"] > 0
    if dtype == 1:
        assert np.max(np.abs(got - want)) < 1e-12
    else:
        assert_c64_close(got, want, len(c), what=f"(13,4) n={n}")
    with pytest.raises(sv.SVError):
        sv.sv_plan_create(n, dtype, ops, params, sv.SV_MODE_FUSED, 13, 4, compile=sv.SV_COMPILE_OFF)


@pytest.mark.parametrize("dtype", [0, 1])
def test_512_thread_tiles_benchmark_prefix_28q(dtype):
    """Two layers of the 28-qubit benchmark circuit at geometry (13,4) against
    the oracle."""
    sv = require_gpu()
    c = random_layered_circuit(28, 2, seed=0)
    want = osv.run(c)
    got, info = run(sv, c, osv.zero_state(28), dtype, sv.SV_COMPILE_ON, 13, 4)
    assert info["n_compiled_kernels"] > 0
    if dtype == 1:
        assert np.max(np.abs(got - want)) < 1e-12
    else:
        assert_c64_close(got, want, len(c), what="(13,4) 28q prefix")


def test_512_thread_tiles_compile_automatically():
    """Automatic mode compiles a 512-thread plan at any size (below 21 qubits
    too), since no generic kernel runs it."""
    sv = require_gpu()
    c = random_mixed_circuit(16, 200, seed=21, max_ctrl=5)
    psi0 = random_state(16, 22)
    got, info = run(sv, c, psi0, 0, sv.SV_COMPILE_AUTO, 13, 4)
    assert info["n_compiled_kernels"] > 0
    assert_c64_close(got, osv.run(c, psi0), len(c), what="(13,4) automatic")
