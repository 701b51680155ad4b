"""GPU parity of the HIP path against the FP64 reference simulator.

Bars: complex128 runs agree with the oracle to 1e-12 (max abs amplitude
difference on normalised states) and infidelity <= 1e-12; complex64 runs to
infidelity <= 1e-6 and, amplitude by amplitude, within 1e-5 of the largest
amplitude per 1,000 gates (at least 1e-5); permutation-only circuits are
bit-exact.  Sizes span
several tiles and both tile geometries; the 28-qubit case is the benchmark's
launch configuration on a prefix of its circuit.
"""
import numpy as np
import pytest

from oracle import statevector as osv
from paper_2606_12770_amd.circuits.ir import Circuit
from paper_2606_12770_amd.circuits.random_circuit import (random_circuit_with_inverse_pairs, random_layered_circuit,
                                                          random_mixed_circuit, random_state)
from tests.gpu_util import assert_c64_close, require_gpu

pytestmark = pytest.mark.gpu


def infid(a, b):
    return 1.0 - abs(np.vdot(a, b)) ** 2 / (np.vdot(a, a).real * np.vdot(b, b).real)


def run_gpu(sv, circ, psi0, dtype, mode, b=0, rb=0):
    st = sv.State(circ.n, dtype, psi0)
    st.apply(circ, mode, b, rb)
    out = st.amplitudes()
    st.close()
    return out


@pytest.mark.parametrize("n", [6, 10, 14])
@pytest.mark.parametrize("dtype", [0, 1])
def test_plain_every_kind(n, dtype):
    sv = require_gpu()
    c = random_mixed_circuit(n, 300, seed=n + 10 * dtype, max_ctrl=min(5, n - 2))
    psi0 = random_state(n, 1)
    want = osv.run(c, psi0)
    got = run_gpu(sv, c, psi0, dtype, sv.SV_MODE_PLAIN)
    print(f"plain n={n} dtype={dtype} maxabs={np.max(np.abs(got - want)):.2e} infid={infid(want, got):.2e}", flush=True)
    if dtype == 1:
        assert np.max(np.abs(got - want)) < 1e-12
        assert infid(want, got) < 1e-12
    else:
        assert infid(want, got) < 1e-6
        assert_c64_close(got, want, len(c), what=f"plain n={n}")


@pytest.mark.parametrize("n,b,rb", [(10, 10, 4), (12, 12, 4), (14, 12, 4), (16, 12, 4), (16, 13, 5),
                                    (18, 12, 4), (20, 11, 5)])
@pytest.mark.parametrize("dtype", [0, 1])
def test_fused_mixed(n, b, rb, dtype):
    sv = require_gpu()
    if dtype == 1 and b == 13:
        b = 12
    c = random_mixed_circuit(n, 400, seed=3 * n + b + dtype, max_ctrl=6)
    psi0 = random_state(n, 2)
    want = osv.run(c, psi0)
    got = run_gpu(sv, c, psi0, dtype, sv.SV_MODE_FUSED, b, rb)
    print(f"fused n={n} b={b} rb={rb} dtype={dtype} infid={infid(want, got):.2e}", flush=True)
    if dtype == 1:
        assert np.max(np.abs(got - want)) < 1e-12
        assert infid(want, got) < 1e-12
    else:
        assert infid(want, got) < 1e-6
        assert_c64_close(got, want, len(c), what=f"fused n={n} b={b} rb={rb}")


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("mode", [0, 1])
def test_layered_20q(dtype, mode):
    sv = require_gpu()
    n = 20
    c = random_layered_circuit(n, 40, seed=5)
    want = osv.run(c)
    got = run_gpu(sv, c, osv.zero_state(n), dtype, mode)
    f = infid(want, got)
    print(f"layered n=20 dtype={dtype} mode={mode} infid={f:.2e}", flush=True)
    assert f < (1e-12 if dtype == 1 else 1e-6)
    if dtype == 1:
        assert np.max(np.abs(got - want)) < 1e-12
    else:
        assert_c64_close(got, want, len(c), what="layered n=20")


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("mode", [0, 1])
def test_permutations_bit_exact(dtype, mode):
    sv = require_gpu()
    n = 16
    rng = np.random.default_rng(7)
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
            w = int(rng.integers(1, 11))  # widths up to 8 shift in one workgroup, wider ones serially
            base = int(rng.integers(0, n - w + 1))
            ctrl = {q: v for q, v in ctrl.items() if not base <= q < base + w}
            (c.inc if k == 2 else c.dec)(base, w, ctrl)
    psi0 = random_state(n, 8)
    if dtype == 0:  # the state holds float values; permuting them must not change a bit
        psi0 = psi0.astype(np.complex64).astype(np.complex128)
    want = osv.run(c, psi0)
    got = run_gpu(sv, c, psi0, dtype, mode)
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))


@pytest.mark.parametrize("dtype", [0, 1])
def test_plain_split_matches_oracle(dtype):
    """Fused plans in which the cost model sends some op groups to plain launches
    (controlled increments of two 7-qubit registers that do not commute, each of
    which would fill a tile pass of its own) against the reference simulator,
    and against the same plan with tile passes only."""
    sv = require_gpu()
    n = 20
    rng = np.random.default_rng(3)
    c = Circuit(n)
    for layer in range(3):
        for q in range(n):
            c.ry(q, rng.uniform(-np.pi, np.pi))
        for _ in range(4):
            c.inc(13, 7, {int(q): int(rng.integers(2)) for q in (6, 8, 10, 12)})
            c.dec(6, 7, {int(q): int(rng.integers(2)) for q in (13, 15, 17, 19)})
        qs = rng.permutation(n)
        c.x(int(qs[0]), {int(q): int(rng.integers(2)) for q in qs[1:9]})
    psi0 = random_state(n, 4)
    want = osv.run(c, psi0)
    ops, params = c.arrays()
    outs = {}
    for split in (sv.SV_PLAIN_SPLIT_AUTO, sv.SV_PLAIN_SPLIT_OFF):
        plan = sv.sv_plan_create(n, dtype, ops, params, sv.SV_MODE_FUSED, 12, 4, plain_split=split)
        info = sv.sv_plan_get_info(plan)
        st = sv.sv_alloc(n, dtype, psi0)
        sv.sv_plan_execute(plan, st, 1)
        outs[split] = sv.sv_amplitudes(st)
        sv.sv_free(st)
        sv.sv_plan_free(plan)
        print(f"split={split} dtype={dtype}: {info['n_tile_passes']} tile passes, {info['n_split_ops']} ops as plain "
              f"launches, infidelity {infid(want, outs[split]):.2e}", flush=True)
        assert (info["n_split_ops"] > 0) == (split == sv.SV_PLAIN_SPLIT_AUTO)
        if dtype == 1:
            assert np.max(np.abs(outs[split] - want)) < 1e-12
        else:
            assert infid(want, outs[split]) < 1e-6
            assert_c64_close(outs[split], want, len(c), what=f"plain split {split}")


def test_reductions_postselect_inner():
    sv = require_gpu()
    n = 18
    psi = random_state(n, 4)
    for dtype in (0, 1):
        st = sv.State(n, dtype, psi)
        assert abs(st.prob() - 1.0) < (1e-6 if dtype == 0 else 1e-13)
        mask, val = 0b101000000000010001, 0b001000000000000001
        idx = np.arange(1 << n)
        keep = (idx & mask) == val
        P = float(np.sum(np.abs(psi[keep]) ** 2))
        assert abs(st.prob(mask, val) - P) < (1e-7 if dtype == 0 else 1e-14)
        got = st.postselect(mask, val)
        assert abs(got - P) < (1e-7 if dtype == 0 else 1e-14)
        amp = st.amplitudes()
        want = np.where(keep, psi / np.sqrt(P), 0)
        assert np.max(np.abs(amp - want)) < (1e-5 if dtype == 0 else 1e-13)
        other = sv.State(n, 1, random_state(n, 5))
        ip = sv.sv_inner(st.h, other.h)
        ref = np.vdot(amp, other.amplitudes())
        assert abs(ip - ref) < 1e-12
        st.close()
        other.close()


def test_errors_are_reported_before_launch():
    sv = require_gpu()
    n = 8
    st = sv.State(n, 1)
    bad = [Circuit(n).x(8), Circuit(n).x(2, [2]), Circuit(n).inc(6, 3), Circuit(n).swap(1, 1),
           Circuit(n).inc(0, 3, [1])]
    for c in bad:
        with pytest.raises(sv.SVError) as e:
            st.apply(c)
        assert e.value.code == sv.SV_EINVAL
    assert abs(st.amplitudes()[0] - 1.0) == 0.0  # untouched
    # zero-probability post-selection leaves the state unchanged
    with pytest.raises(sv.SVError) as e:
        st.postselect(1, 1)
    assert e.value.code == sv.SV_EZEROPROB
    assert st.amplitudes()[0] == 1.0
    st.close()


@pytest.mark.parametrize("dtype", [0, 1])
def test_benchmark_configuration_28q_prefix(dtype):
    """28 qubits, the benchmark's fused launch configuration (its tile geometry,
    the nontemporal-streaming instantiation of states of 256 MiB and more), on
    the first two layers of the benchmark circuit, compared amplitude by
    amplitude with the FP64 reference simulator."""
    sv = require_gpu()
    n = 28
    c = random_layered_circuit(n, 2, seed=0)
    want = osv.run(c)
    got = run_gpu(sv, c, osv.zero_state(n), dtype, sv.SV_MODE_FUSED)
    f = infid(want, got)
    print(f"28q prefix dtype={dtype} infid={f:.2e}", flush=True)
    assert f < (1e-12 if dtype == 1 else 1e-6)
    if dtype == 1:
        assert np.max(np.abs(got - want)) < 1e-12
    else:
        assert_c64_close(got, want, len(c), what="28q prefix")


def test_benchmark_circuit_20_layer_prefix_elementwise():
    """The first 20 layers (780 gates) of the 28-qubit benchmark circuit in the
    benchmark's own configuration (complex64, compiled tile passes, geometry
    (12,4), plain splits) against the FP64 reference simulator, amplitude by
    amplitude (about 30 s of host time for the reference)."""
    sv = require_gpu()
    n = 28
    c = random_layered_circuit(n, 20, seed=0)
    want = osv.run(c)
    ops, params = c.arrays()
    plan = sv.sv_plan_create(n, sv.SV_C64, ops, params, sv.SV_MODE_FUSED)
    info = sv.sv_plan_get_info(plan)
    st = sv.State(n, sv.SV_C64)
    sv.sv_plan_execute(plan, st.h, 1)
    got = st.amplitudes()
    st.close()
    sv.sv_plan_free(plan)
    print(f"28q 20-layer prefix: {info['n_tile_passes']} passes, {info['n_compiled_kernels']} compiled kernels, "
          f"infidelity {infid(want, got):.2e}", flush=True)
    assert info["n_compiled_kernels"] > 0 and info["tile_qubits"] == 12 and info["reg_qubits"] == 4
    assert infid(want, got) < 1e-6
    assert_c64_close(got, want, len(c), what="28q 20-layer prefix")


def test_layered_26q_complex64_elementwise():
    """Six layers of the benchmark's random layered circuit on 26 qubits
    (512 MiB: streamed tile passes with the resident-set lookahead and op
    ordering of large states), complex64 fused, amplitude by amplitude
    against the FP64 reference simulator."""
    sv = require_gpu()
    n = 26
    c = random_layered_circuit(n, 6, seed=3)
    want = osv.run(c)
    got = run_gpu(sv, c, osv.zero_state(n), sv.SV_C64, sv.SV_MODE_FUSED)
    print(f"26q 6 layers: infid={infid(want, got):.2e}", flush=True)
    assert infid(want, got) < 1e-6
    assert_c64_close(got, want, len(c), what="26q layered")


def _run_plan(sv, circ, psi0, dtype, tile_launch, b=0, rb=0):
    ops, params = circ.arrays()
    plan = sv.sv_plan_create(circ.n, dtype, ops, params, sv.SV_MODE_FUSED, b, rb, tile_launch=tile_launch)
    st = sv.State(circ.n, dtype, psi0)
    sv.sv_plan_execute(plan, st.h, 1)
    out = st.amplitudes()
    st.close()
    sv.sv_plan_free(plan)
    return out


@pytest.mark.parametrize("n,b,rb", [(12, 12, 4), (16, 12, 4), (18, 12, 4), (20, 11, 5)])
@pytest.mark.parametrize("dtype", [0, 1])
def test_persistent_tile_launch_matches_oracle(n, b, rb, dtype):
    """The persistent launch form (resident workgroups walking the tiles, the
    next tile's loads in flight) against the FP64 reference simulator, and bit
    for bit against one workgroup per tile (same passes, same arithmetic)."""
    sv = require_gpu()
    c = random_mixed_circuit(n, 400, seed=5 * n + b + dtype, max_ctrl=6)
    psi0 = random_state(n, 3)
    want = osv.run(c, psi0)
    got = _run_plan(sv, c, psi0, dtype, sv.SV_TILE_LAUNCH_PERSISTENT, b, rb)
    grid = _run_plan(sv, c, psi0, dtype, sv.SV_TILE_LAUNCH_GRID, b, rb)
    print(f"persistent n={n} b={b} rb={rb} dtype={dtype} infid={infid(want, got):.2e}", flush=True)
    assert np.array_equal(got.view(np.uint64), grid.view(np.uint64))
    if dtype == 1:
        assert np.max(np.abs(got - want)) < 1e-12
    else:
        assert infid(want, got) < 1e-6
        assert_c64_close(got, want, len(c), what=f"persistent n={n}")


@pytest.mark.parametrize("dtype", [0, 1])
def test_persistent_tile_launch_many_tiles_per_workgroup(dtype):
    """26 qubits (16,384 tiles: several per resident workgroup) and the
    benchmark's launch geometry: bit for bit equal to one workgroup per tile,
    and the inverse circuit returns |0...0>."""
    sv = require_gpu()
    n = 26
    c = random_mixed_circuit(n, 300, seed=11 + dtype, max_ctrl=6)
    psi0 = np.zeros(1 << n, dtype=np.complex128)
    psi0[0] = 1.0
    got = _run_plan(sv, c, psi0, dtype, sv.SV_TILE_LAUNCH_PERSISTENT)
    grid = _run_plan(sv, c, psi0, dtype, sv.SV_TILE_LAUNCH_GRID)
    assert np.array_equal(got.view(np.uint64), grid.view(np.uint64))
    back = _run_plan(sv, c.dagger(), got, dtype, sv.SV_TILE_LAUNCH_PERSISTENT)
    p0 = abs(back[0]) ** 2 / np.vdot(back, back).real
    print(f"persistent 26q dtype={dtype}: |<0|U^dagger U|0>|^2 = {p0:.15f}", flush=True)
    assert 1.0 - p0 < (1e-12 if dtype == 1 else 1e-5)


@pytest.mark.parametrize("n,mode,compile", [(14, 1, 1), (22, 1, 2), (12, 0, 0)])
@pytest.mark.parametrize("dtype", [0, 1])
def test_peephole_matches_oracle(n, mode, compile, dtype):
    """Plans with the peephole pass on (Sec. III.F.2: adjacent inverse pairs
    dropped): the count dropped is the number spliced in, and the state matches
    the oracle's run of the full op list (complex128 to 1e-12, complex64
    element-wise to the complex64 bar)."""
    sv = require_gpu()
    c, expect = random_circuit_with_inverse_pairs(n, n + dtype)
    psi0 = random_state(n, 9)
    want = osv.run(c, psi0)
    ops, params = c.arrays()
    plan = sv.sv_plan_create(n, dtype, ops, params, mode, 12 if mode else 0, 4 if mode else 0, compile=compile,
                             peephole=sv.SV_PEEPHOLE_ON)
    info = sv.sv_plan_get_info(plan)
    st = sv.sv_alloc(n, dtype, psi0)
    sv.sv_plan_execute(plan, st, 1)
    got = sv.sv_amplitudes(st)
    sv.sv_free(st)
    sv.sv_plan_free(plan)
    print(f"peephole n={n} mode={mode} dtype={dtype}: dropped {info['n_cancelled_ops']} of {len(c)} ops, "
          f"max abs err {np.max(np.abs(got - want)):.2e}", flush=True)
    assert info["n_cancelled_ops"] == expect
    if dtype == 1:
        assert np.max(np.abs(got - want)) < 1e-12
    else:
        assert_c64_close(got, want, len(c), what=f"peephole n={n} mode={mode}")


def test_touched_bytes_count_whole_lines():
    """sv_plan_info.touched_bytes: a plain launch whose control sits on a qubit
    inside a 128-byte line still moves whole lines; one controlled above the
    line moves half the state; a tile pass moves the whole state either way."""
    sv = require_gpu()
    n = 20
    c = Circuit(n)
    c.x(10, [0])   # control inside a line (complex64: 16 amplitudes per line)
    c.x(10, [15])  # control above it
    ops, params = c.arrays()
    full = 2 * (1 << n) * 8
    plan = sv.sv_plan_create(n, sv.SV_C64, ops, params, sv.SV_MODE_PLAIN)
    info = sv.sv_plan_get_info(plan)
    sv.sv_plan_free(plan)
    assert info["bytes_moved"] == full
    assert info["touched_bytes"] == full + full // 2
    plan = sv.sv_plan_create(n, sv.SV_C64, ops, params, sv.SV_MODE_FUSED, 12, 4, plain_split=sv.SV_PLAIN_SPLIT_OFF)
    info = sv.sv_plan_get_info(plan)
    sv.sv_plan_free(plan)
    assert info["touched_bytes"] == info["bytes_moved"] == info["n_tile_passes"] * full


@pytest.mark.parametrize("dtype,coalesce", [(0, 4), (1, 3), (0, 3)])
def test_coalesce_width_matches_oracle(dtype, coalesce):
    """Plans with fewer lowest qubits kept resident (sv_apply_opts.coalesce_qubits:
    runs of one 128-byte line, or half a line) against the oracle: a layered
    circuit at 22 qubits, compiled passes."""
    sv = require_gpu()
    n = 22
    c = random_layered_circuit(n, 8, seed=5)
    want = osv.run(c)
    ops, params = c.arrays()
    plan = sv.sv_plan_create(n, dtype, ops, params, sv.SV_MODE_FUSED, 12, 4, compile=sv.SV_COMPILE_ON,
                             coalesce_qubits=coalesce)
    st = sv.State(n, dtype)
    sv.sv_plan_execute(plan, st.h, 1)
    got = st.amplitudes()
    st.close()
    sv.sv_plan_free(plan)
    if dtype == 1:
        assert np.max(np.abs(got - want)) < 1e-12
    else:
        assert_c64_close(got, want, len(c), what=f"coalesce {coalesce}")
