"""Edge cases of the C ABI and the kernels.

* Degenerate sizes: 1 to 7 qubits (fused mode falls back to per-gate launches
  when a tile would have fewer than 64 threads), one tile exactly (b = n),
  ragged tile counts, the empty circuit.
* Errors raised on the host before any launch: a state too large for the device
  (SV_ENOMEM), ranges outside the state.
* Amplitude ranges with ragged offsets and lengths, copies across precisions.
* The benchmark workload at full depth (28 qubits, 200 layers, the fused launch
  configuration bench.py times): the circuit followed by its inverse must return
  |0...0> (a property that holds at any size; the oracle checks the same launch
  configuration amplitude by amplitude on a two-layer prefix elsewhere).
"""
import numpy as np
import pytest

from oracle import statevector as osv
from paper_2606_12770_amd.circuits.ir import Circuit
from paper_2606_12770_amd.circuits.random_circuit import random_layered_circuit, random_mixed_circuit, random_state
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7])
@pytest.mark.parametrize("mode", [0, 1])
def test_tiny_states_every_kind(n, mode):
    sv = require_gpu()
    c = random_mixed_circuit(n, 60, seed=n, max_ctrl=max(0, min(3, n - 2)))
    psi0 = random_state(n, 2 * n)
    want = osv.run(c, psi0)
    for dtype, tol in ((1, 1e-13), (0, 1e-5)):
        st = sv.State(n, dtype, psi0)
        st.apply(c, mode)
        got = st.amplitudes()
        st.close()
        assert np.max(np.abs(got - want)) < tol


@pytest.mark.parametrize("n", [11, 12, 13])
def test_single_and_ragged_tile_counts(n):
    sv = require_gpu()
    c = random_mixed_circuit(n, 200, seed=100 + n, max_ctrl=4)
    psi0 = random_state(n, n)
    want = osv.run(c, psi0)
    for b in (12, 11):
        st = sv.State(n, 1, psi0)
        st.apply(c, 1, b, 4)
        assert np.max(np.abs(st.amplitudes() - want)) < 1e-12
        st.close()


def test_empty_circuit_leaves_state_bit_identical():
    sv = require_gpu()
    psi0 = random_state(14, 1)
    for dtype in (0, 1):
        st = sv.State(14, dtype, psi0)
        before = st.amplitudes()
        st.apply(Circuit(14), 1)
        st.apply(Circuit(14), 0)
        assert np.array_equal(st.amplitudes().view(np.uint64), before.view(np.uint64))
        st.close()


def test_out_of_memory_and_ranges_are_refused():
    sv = require_gpu()
    with pytest.raises(sv.SVError) as e:
        sv.sv_alloc(36, sv.SV_C128)   # 1 TiB
    assert e.value.code == sv.SV_ENOMEM
    st = sv.State(10, 1)
    with pytest.raises(sv.SVError) as e:
        sv.sv_amplitudes(st.h, 1000, 100)
    assert e.value.code == sv.SV_EINVAL
    with pytest.raises(sv.SVError) as e:
        sv.sv_set_amplitudes(st.h, np.ones(30), 1000)
    assert e.value.code == sv.SV_EINVAL
    st.close()


def test_ragged_amplitude_ranges_and_cross_precision_copy():
    sv = require_gpu()
    n = 15
    psi = random_state(n, 9)
    st = sv.State(n, 1)
    sv.sv_set_amplitudes(st.h, psi[:777], 0)
    sv.sv_set_amplitudes(st.h, psi[777:20001], 777)
    sv.sv_set_amplitudes(st.h, psi[20001:], 20001)
    assert np.array_equal(st.amplitudes(), psi)
    assert np.array_equal(sv.sv_amplitudes(st.h, 12345, 3), psi[12345:12348])
    lo = sv.State(n, 0)
    sv.sv_copy(lo.h, st.h)
    assert np.array_equal(lo.amplitudes(), psi.astype(np.complex64).astype(np.complex128))
    back = sv.State(n, 1)
    sv.sv_copy(back.h, lo.h)
    assert np.array_equal(back.amplitudes(), lo.amplitudes())
    for s in (st, lo, back):
        s.close()


@pytest.mark.parametrize("dtype", [0, 1])
def test_benchmark_workload_full_depth_inverts(dtype):
    sv = require_gpu()
    n = 28
    c = random_layered_circuit(n, 200, seed=0)
    ops, params = c.arrays()
    dops, dparams = c.dagger().arrays()
    fwd = sv.sv_plan_create(n, dtype, ops, params, sv.SV_MODE_FUSED)
    inv = sv.sv_plan_create(n, dtype, dops, dparams, sv.SV_MODE_FUSED)
    st = sv.sv_alloc(n, dtype)
    sv.sv_plan_execute(fwd, st, 1)
    mid = sv.sv_postselect(st, 0, 0, keep=False, renormalize=False)
    p0 = sv.sv_postselect(st, (1 << n) - 1, 0, keep=False, renormalize=False)
    sv.sv_plan_execute(inv, st, 1)
    back = sv.sv_postselect(st, (1 << n) - 1, 0, keep=False, renormalize=False)
    norm = sv.sv_postselect(st, 0, 0, keep=False, renormalize=False)
    sv.sv_free(st)
    sv.sv_plan_free(fwd)
    sv.sv_plan_free(inv)
    print(f"28q 200 layers dtype={dtype}: |psi|^2={mid:.12f} |<0|psi>|^2={p0:.3e} after inverse "
          f"|<0|psi>|^2={back:.12f} |psi|^2={norm:.12f}", flush=True)
    # the forward circuit spreads the state (no amplitude near 1), the inverse brings it back
    assert p0 < 1e-6
    eps = 2.0 ** -52 if dtype == 1 else 2.0 ** -23
    assert abs(norm - 1.0) < 2 * len(c) * eps
    assert 1.0 - back / norm < (1e-10 if dtype == 1 else 1e-5)
