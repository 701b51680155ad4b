"""Dense 5-qubit blocks on matrix cores against the FP64 reference simulator:
deep runs confined to five qubits become one 32 x 32 block each, applied with
FP32 MFMA for complex64 (bar: infidelity <= 1e-6, amplitudes within 1e-5) and
FP64 MFMA for complex128 (amplitudes within 1e-12 of the gate-by-gate oracle)."""
import numpy as np
import pytest

from oracle import statevector as osv
from paper_2606_12770_amd.circuits.random_circuit import random_dense_block_circuit, random_state
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu


def infid(a, b):
    return 1.0 - abs(np.vdot(a, b)) ** 2 / (np.vdot(a, a).real * np.vdot(b, b).real)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("n,blocks,depth", [(12, 3, 4), (16, 6, 5), (20, 8, 6), (23, 4, 8)])
def test_dense_blocks_match_oracle(n, blocks, depth, dtype):
    sv = require_gpu()
    c = random_dense_block_circuit(n, blocks, depth, seed=n)
    psi0 = random_state(n, n + 1)
    want = osv.run(c, psi0)
    ops, params = c.arrays()
    dt = sv.SV_C64 if dtype == "c64" else sv.SV_C128
    plan = sv.sv_plan_create(n, dt, ops, params, sv.SV_MODE_FUSED, 12, 4, 16)
    info = sv.sv_plan_get_info(plan)
    st = sv.sv_alloc(n, dt, psi0)
    sv.sv_plan_execute(plan, st, 1)
    got = sv.sv_amplitudes(st)
    sv.sv_free(st)
    sv.sv_plan_free(plan)
    f = infid(want, got)
    print(f"dense {dtype} n={n} blocks={blocks} depth={depth}: {info['n_dense_passes']} dense passes absorbing "
          f"{info['n_dense_ops']} of {len(c)} ops, infidelity {f:.2e}", flush=True)
    assert info["n_dense_passes"] == blocks
    if dtype == "c64":
        assert f < 1e-6
        assert np.max(np.abs(got - want)) < 1e-5
    else:
        assert np.max(np.abs(got - want)) < 1e-12


@pytest.mark.parametrize("n,blocks,depth", [(12, 3, 4), (16, 6, 5), (20, 8, 6), (23, 4, 8)])
def test_split_bf16_dense_blocks_match_oracle(n, blocks, depth):
    """Complex64 dense blocks on BF16 matrix cores with split operands (hi + lo
    BF16 parts, three products, FP32 accumulation): infidelity within the
    complex64 bar of 1e-6; every amplitude within 2^-14 of the largest per
    block applied (the split leaves about 2^-16 of each block product)."""
    sv = require_gpu()
    c = random_dense_block_circuit(n, blocks, depth, seed=n)
    psi0 = random_state(n, n + 1)
    want = osv.run(c, psi0)
    ops, params = c.arrays()
    outs = {}
    for bf16 in (0, 1):
        plan = sv.sv_plan_create(n, sv.SV_C64, ops, params, sv.SV_MODE_FUSED, 12, 4, 16, dense_bf16=bf16)
        info = sv.sv_plan_get_info(plan)
        st = sv.sv_alloc(n, sv.SV_C64, psi0)
        sv.sv_plan_execute(plan, st, 1)
        outs[bf16] = sv.sv_amplitudes(st)
        sv.sv_free(st)
        sv.sv_plan_free(plan)
        assert info["n_dense_passes"] == blocks
    got = outs[1]
    f = infid(want, got)
    err = np.max(np.abs(got - want)) / np.max(np.abs(want))
    err32 = np.max(np.abs(outs[0] - want)) / np.max(np.abs(want))
    print(f"split-BF16 dense n={n} blocks={blocks}: infidelity {f:.2e} (FP32 {infid(want, outs[0]):.2e}), "
          f"rel max err {err:.2e} (FP32 {err32:.2e})", flush=True)
    assert f < 1e-6
    assert err < blocks * 2.0 ** -14


@pytest.mark.parametrize("bf16", [0, 1])
@pytest.mark.parametrize("n,blocks,depth", [(12, 3, 4), (16, 6, 5), (20, 8, 6), (24, 4, 8)])
def test_six_qubit_dense_blocks_match_oracle(n, blocks, depth, bf16):
    """Six-qubit blocks (64 x 64, complex64) on FP32 matrix cores and in split
    BF16: the deep runs become dense passes; infidelity within 1e-6 and
    every amplitude within the bar of the five-qubit form (FP32: 1e-5
    absolute; split BF16: 2^-14 of the largest per block applied)."""
    sv = require_gpu()
    c = random_dense_block_circuit(n, blocks, depth, seed=n + 1, width=6)
    psi0 = random_state(n, n + 2)
    want = osv.run(c, psi0)
    ops, params = c.arrays()
    plan = sv.sv_plan_create(n, sv.SV_C64, ops, params, sv.SV_MODE_FUSED, 12, 4, 16, dense_bf16=bf16,
                             dense_qubits=6)
    info = sv.sv_plan_get_info(plan)
    st = sv.sv_alloc(n, sv.SV_C64, psi0)
    sv.sv_plan_execute(plan, st, 1)
    got = sv.sv_amplitudes(st)
    sv.sv_free(st)
    sv.sv_plan_free(plan)
    f = infid(want, got)
    err = np.max(np.abs(got - want)) / np.max(np.abs(want))
    print(f"six-qubit dense {'split-BF16' if bf16 else 'FP32'} n={n} blocks={blocks}: {info['n_dense_passes']} dense "
          f"passes absorbing {info['n_dense_ops']} of {len(c)} ops, infidelity {f:.2e}, rel max err {err:.2e}",
          flush=True)
    # every deep run is absorbed; a run may be cut where the ops between blocks
    # join it, giving one dense pass more
    assert blocks <= info["n_dense_passes"] <= 2 * blocks
    assert f < 1e-6
    if bf16:
        assert err < blocks * 2.0 ** -14
    else:
        assert np.max(np.abs(got - want)) < 1e-5


def test_six_qubit_blocks_refused_for_complex128():
    sv = require_gpu()
    c = random_dense_block_circuit(12, 2, 4, seed=3, width=6)
    ops, params = c.arrays()
    with pytest.raises(sv.SVError) as e:
        sv.sv_plan_create(12, sv.SV_C128, ops, params, sv.SV_MODE_FUSED, 12, 4, 16, dense_qubits=6)
    assert e.value.code == -5
