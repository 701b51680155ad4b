"""Batched execution of independent circuits of uneven size.

* One launch per level over the tiles of every instance must give exactly the
  states that running each plan on its own gives (same tile code, same
  arithmetic: bit-identical), with and without HIP-graph capture.
* Small Carleman-LBM instances in a batch against the FP64 reference simulator.
* A batch that holds a plan with gate runs (22-qubit Carleman ladder) matches
  its plans run alone, bit for bit.
* Graph replays, with the program's own eager work between them, match the
  eager result after every replay.
* Invalid batches are refused on the host.
* Compiled plans run in the concurrent form (instances on side streams that
  fork from and join back to one stream, one graph): bit-identical to each
  plan run alone, graph and eager alike, with plain launches among the steps,
  states outside an arena, and plans freed before the batch runs.
* Complex64 plans whose real gates carry hi + lo entries (split_real) run
  in both batch forms bit-identical to each plan alone.
* The 64-instance batched workload itself (21-28 qubits, complex64, d = 3):
  every instance's system amplitudes against the oracle's singular-value
  transform of its own L, amplitude by amplitude.
"""
import numpy as np
import pytest

from oracle import statevector as osv
from paper_2606_12770_amd.circuits import carleman_circuit as cc
from paper_2606_12770_amd.circuits import qsp
from paper_2606_12770_amd.circuits.random_circuit import random_layered_circuit, random_mixed_circuit, random_state
from tests.carleman_ref import ladder_reference
from tests.gpu_util import assert_c64_close, require_gpu

pytestmark = pytest.mark.gpu


def _plans(sv, circs, dtype, b=12, rb=4, compile=0):
    out = []
    for c in circs:
        ops, params = c.arrays()
        out.append(sv.sv_plan_create(c.n, dtype, ops, params, sv.SV_MODE_FUSED, b, rb,
                                      plain_split=sv.SV_PLAIN_SPLIT_OFF, compile=compile))
    return out


def _mixed_batch(seed):
    rng = np.random.default_rng(seed)
    ns = [14, 17, 20, 15, 18, 21, 16]
    circs = [random_mixed_circuit(n, 150, seed=int(rng.integers(1 << 30)), max_ctrl=4) for n in ns]
    circs[3] = random_layered_circuit(15, 6, seed=2)
    inits = [random_state(n, 100 + i) for i, n in enumerate(ns)]
    return circs, inits


ONE_GROUP = (1 << 64) - 1


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("use_graph,group_bytes", [(False, ONE_GROUP), (True, ONE_GROUP), (True, 0), (False, 1 << 22)])
def test_batch_equals_one_at_a_time(dtype, use_graph, group_bytes):
    sv = require_gpu()
    circs, inits = _mixed_batch(dtype)
    plans = _plans(sv, circs, dtype)
    states = sv.sv_alloc_batch([c.n for c in circs], dtype)
    for st, v in zip(states, inits):
        sv.sv_set_amplitudes(st, v, 0)
    batch = sv.sv_batch_create(states, plans, use_graph, group_bytes)
    sv.sv_batch_execute(batch, 2)
    got = [sv.sv_amplitudes(st) for st in states]
    for i, (c, v, p) in enumerate(zip(circs, inits, plans)):
        ref = sv.sv_alloc(c.n, dtype, v)
        sv.sv_plan_execute(p, ref, 2)
        want = sv.sv_amplitudes(ref)
        sv.sv_free(ref)
        print(f"instance {i}: n={c.n} dtype={dtype} graph={use_graph} maxabs={np.max(np.abs(got[i] - want)):.1e}",
              flush=True)
        assert np.array_equal(got[i], want)
        if c.n <= 17:
            oracle = osv.run(c, osv.run(c, v))
            tol = 1e-12 if dtype == 1 else 1e-5
            assert np.max(np.abs(got[i] - oracle)) < tol
    launches, groups, gates = sv.sv_batch_levels(batch)
    assert gates == sum(len(c) for c in circs)
    passes = [sv.sv_plan_get_info(p)["n_launches"] for p in plans]
    if group_bytes == ONE_GROUP:
        assert groups == 1 and launches == max(passes)
    else:
        assert 1 <= groups <= len(circs) and max(passes) <= launches <= sum(passes)
    sv.sv_batch_free(batch)
    for st in states:
        sv.sv_free(st)
    for p in plans:
        sv.sv_plan_free(p)


def test_batch_of_carleman_ladders_matches_oracle():
    sv = require_gpu()
    cfgs = [cc.CarlemanConfig(nx=2, tau=0.9, nk=1, nt=1, amp=0.1),
            cc.CarlemanConfig(nx=2, tau=0.7, nk=2, nt=2, amp=0.05),
            cc.CarlemanConfig(nx=4, tau=1.1, nk=1, nt=1, amp=0.08, wavenumber=2)]
    phases = qsp.inversion_phases(2.0, 5)[0]
    circs, inits = [], []
    for cfg in cfgs:
        enc = cc.build_ul(cfg)
        circs.append(cc.build_qsvt(enc, phases))
        v = np.zeros(1 << enc.layout.n, dtype=np.complex128)
        v[: 1 << enc.layout.n_x] = cc.rhs_x_block(cfg, enc.layout)
        inits.append(v)
    plans = _plans(sv, circs, 1)
    states = sv.sv_alloc_batch([c.n for c in circs], 1)
    for st, v in zip(states, inits):
        sv.sv_set_amplitudes(st, v, 0)
    batch = sv.sv_batch_create(states, plans, True)
    sv.sv_batch_execute(batch, 1)
    for c, v, st in zip(circs, inits, states):
        got = sv.sv_amplitudes(st)
        want = osv.run(c, v)
        print(f"carleman batch n={c.n}: maxabs {np.max(np.abs(got - want)):.1e}", flush=True)
        assert np.max(np.abs(got - want)) < 1e-12
    sv.sv_batch_free(batch)
    for st in states:
        sv.sv_free(st)
    for p in plans:
        sv.sv_plan_free(p)


@pytest.mark.parametrize("dtype", [0, 1])
def test_batch_with_gate_runs(dtype):
    """A 22-qubit Carleman ladder (its value encodings become gate runs from 21
    qubits; the CPU plan emulation of the same configuration shows the runs)
    batched with smaller circuits: the level that holds runs takes the run
    kernel for all of its passes, and every instance must come out bit-identical
    to its plan run alone; the ladder also against the reference simulator."""
    sv = require_gpu()
    cfg = cc.CarlemanConfig(nx=8, tau=1.0, nk=2, nt=2, dt=0.1, amp=0.05)
    ladder = cc.build_qsvt(cc.build_ul(cfg), np.random.default_rng(3).uniform(-np.pi, np.pi, 4))
    assert ladder.n == 22
    circs = [ladder, random_mixed_circuit(16, 200, seed=5, max_ctrl=4), random_layered_circuit(21, 3, seed=6)]
    inits = [random_state(c.n, 40 + i) for i, c in enumerate(circs)]
    plans = _plans(sv, circs, dtype)
    states = sv.sv_alloc_batch([c.n for c in circs], dtype)
    for st, v in zip(states, inits):
        sv.sv_set_amplitudes(st, v, 0)
    batch = sv.sv_batch_create(states, plans, True, ONE_GROUP)
    sv.sv_batch_execute(batch, 1)
    for i, (c, v, p, st) in enumerate(zip(circs, inits, plans, states)):
        got = sv.sv_amplitudes(st)
        ref = sv.sv_alloc(c.n, dtype, v)
        sv.sv_plan_execute(p, ref, 1)
        want = sv.sv_amplitudes(ref)
        sv.sv_free(ref)
        print(f"gate-run batch instance {i}: n={c.n} dtype={dtype} maxabs={np.max(np.abs(got - want)):.1e}",
              flush=True)
        assert np.array_equal(got, want)
        if i == 0:
            oracle = osv.run(c, v)
            tol = 1e-12 if dtype == 1 else 1e-5
            assert np.max(np.abs(got - oracle)) < tol
    sv.sv_batch_free(batch)
    for st in states:
        sv.sv_free(st)
    for p in plans:
        sv.sv_plan_free(p)


def test_graph_replays_match_eager_with_work_between():
    sv = require_gpu()
    circs, inits = _mixed_batch(5)
    plans = _plans(sv, circs, 0)
    g_states = sv.sv_alloc_batch([c.n for c in circs], 0)
    e_states = sv.sv_alloc_batch([c.n for c in circs], 0)
    for a, b_, v in zip(g_states, e_states, inits):
        sv.sv_set_amplitudes(a, v, 0)
        sv.sv_set_amplitudes(b_, v, 0)
    gb = sv.sv_batch_create(g_states, plans, True)
    eb = sv.sv_batch_create(e_states, plans, False)
    for replay in range(4):
        sv.sv_batch_execute(gb, 1)
        sv.sv_batch_execute(eb, 1)
        for a, b_ in zip(g_states, e_states):
            # eager work of the program between replays: FP64 reductions, read-out
            na = sv.sv_postselect(a, 0, 0, keep=False, renormalize=False)
            nb = sv.sv_postselect(b_, 0, 0, keep=False, renormalize=False)
            assert na == nb
            assert np.array_equal(sv.sv_amplitudes(a), sv.sv_amplitudes(b_)), f"replay {replay} differs"
    sv.sv_batch_free(gb)
    sv.sv_batch_free(eb)
    for st in g_states + e_states:
        sv.sv_free(st)
    for p in plans:
        sv.sv_plan_free(p)


def test_invalid_batches_are_refused():
    sv = require_gpu()
    c1 = random_mixed_circuit(14, 50, seed=1)
    c2 = random_mixed_circuit(15, 50, seed=2)
    o1, p1 = c1.arrays()
    o2, p2 = c2.arrays()
    pa = sv.sv_plan_create(14, 0, o1, p1, sv.SV_MODE_FUSED, 12, 4, plain_split=sv.SV_PLAIN_SPLIT_OFF)
    pb = sv.sv_plan_create(15, 0, o2, p2, sv.SV_MODE_FUSED, 11, 4, plain_split=sv.SV_PLAIN_SPLIT_OFF)  # other geometry
    pc = sv.sv_plan_create(15, 0, o2, p2, sv.SV_MODE_PLAIN)           # per-gate steps
    st = sv.sv_alloc_batch([14, 15], 0)
    for plans, code in (([pa, pb], sv.SV_EINVAL), ([pa, pc], sv.SV_EINVAL)):
        with pytest.raises(sv.SVError) as e:
            sv.sv_batch_create(st, plans, False)
        assert e.value.code == code
    with pytest.raises(sv.SVError) as e:
        sv.sv_batch_create([st[0], st[0]], [pa, pa], False)
    assert e.value.code == sv.SV_EINVAL
    # states outside an arena, or from two arenas, are refused
    lone = sv.sv_alloc(15, 0)
    other = sv.sv_alloc_batch([15], 0)
    pd = sv.sv_plan_create(15, 0, o2, p2, sv.SV_MODE_FUSED, 12, 4, plain_split=sv.SV_PLAIN_SPLIT_OFF)
    for pair in ([st[0], lone], [st[0], other[0]]):
        with pytest.raises(sv.SVError) as e:
            sv.sv_batch_create(pair, [pa, pd], False)
        assert e.value.code == sv.SV_EINVAL
    sv.sv_plan_free(pd)
    sv.sv_free(lone)
    sv.sv_free(other[0])
    for s in st:
        sv.sv_free(s)
    for p in (pa, pb, pc):
        sv.sv_plan_free(p)


def test_batched_workload_matches_oracle():
    """The benchmark's batched workload as the benchmark runs it: 64 seeded
    Carleman-LBM instances (N_x, N_K, N_t, tau, amplitude and wavenumber drawn
    per seed; 21-28 qubits), the QSVT ladder at d = 3 from b, complex64 in one
    arena, graph-captured.  Every instance against the oracle's transform."""
    from paper_2606_12770_amd.circuits import batch_workload
    sv = require_gpu()
    d = 3
    cfgs = batch_workload.batch_configs(64)
    phases = qsp.inversion_phases(max(1.2, (d - 1) / 10.0), d)[0]
    encs = [cc.build_ul(cfg) for cfg in cfgs]
    circs = [cc.build_qsvt(e, phases) for e in encs]
    states = sv.sv_alloc_batch([c.n for c in circs], sv.SV_C64)
    plans = _plans(sv, circs, sv.SV_C64)
    for st, cfg, e in zip(states, cfgs, encs):
        sv.sv_set_amplitudes(st, cc.rhs_x_block(cfg, e.layout), 0)
    batch = sv.sv_batch_create(states, plans, True, 0)
    sv.sv_batch_execute(batch, 1)
    worst_f, worst_e = 0.0, 0.0
    for i, (st, cfg, e) in enumerate(zip(states, cfgs, encs)):
        L = e.layout
        want, idx = ladder_reference(cfg, L, e.lam, phases)
        got = sv.sv_amplitudes(st, 0, 1 << L.n_sys)[idx]
        f = 1.0 - abs(np.vdot(want, got)) ** 2 / (np.vdot(want, want).real * np.vdot(got, got).real)
        err = np.max(np.abs(got - want)) / np.max(np.abs(want))
        worst_f, worst_e = max(worst_f, f), max(worst_e, err)
        print(f"instance {i}: {L.n} qubits (N_x {cfg.nx}, N_K {cfg.nk}, N_t {cfg.nt}), infidelity {f:.1e}, "
              f"rel max err {err:.1e}", flush=True)
        assert f < 1e-6
        assert_c64_close(got, want, len(circs[i]), what=f"batched instance {i}")
    print(f"worst over 64 instances: infidelity {worst_f:.1e}, rel max err {worst_e:.1e}", flush=True)
    sv.sv_batch_free(batch)
    for p in plans:
        sv.sv_plan_free(p)
    for st in states:
        sv.sv_free(st)


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("use_graph", [False, True])
def test_concurrent_batch_of_compiled_plans(dtype, use_graph):
    sv = require_gpu()
    circs, inits = _mixed_batch(10 + dtype)
    # compiled plans with the automatic plain split (plain launches among the steps)
    plans = []
    for c in circs:
        ops, params = c.arrays()
        plans.append(sv.sv_plan_create(c.n, dtype, ops, params, sv.SV_MODE_FUSED, compile=sv.SV_COMPILE_ON))
    refs = []
    for c, v, p in zip(circs, inits, plans):
        ref = sv.sv_alloc(c.n, dtype, v)
        sv.sv_plan_execute(p, ref, 2)
        refs.append(sv.sv_amplitudes(ref))
        sv.sv_free(ref)
    states = [sv.sv_alloc(c.n, dtype, v) for c, v in zip(circs, inits)]   # not an arena
    batch = sv.sv_batch_create(states, plans, use_graph, 0)
    launches, groups, gates = sv.sv_batch_levels(batch)
    assert gates == sum(len(c) for c in circs)
    assert launches == sum(sv.sv_plan_get_info(p)["n_launches"] for p in plans)
    assert groups == 4
    for p in plans:  # the batch holds the plans
        sv.sv_plan_free(p)
    sv.sv_batch_execute(batch, 1)
    sv.sv_batch_execute(batch, 1)   # a replay when captured
    for i, (c, st) in enumerate(zip(circs, states)):
        got = sv.sv_amplitudes(st)
        print(f"concurrent instance {i}: n={c.n} dtype={dtype} graph={use_graph} "
              f"maxabs={np.max(np.abs(got - refs[i])):.1e}", flush=True)
        assert np.array_equal(got.view(np.uint64), refs[i].view(np.uint64))
    sv.sv_batch_free(batch)
    for st in states:
        sv.sv_free(st)


@pytest.mark.parametrize("concurrent", [False, True])
def test_batches_of_split_real_plans(concurrent):
    sv = require_gpu()
    circs, inits = _mixed_batch(20 + concurrent)
    plans = []
    for c in circs:
        ops, params = c.arrays()
        if concurrent:
            plans.append(sv.sv_plan_create(c.n, sv.SV_C64, ops, params, sv.SV_MODE_FUSED, compile=sv.SV_COMPILE_ON,
                                          split_real=sv.SV_SPLIT_REAL_ON))
        else:
            plans.append(sv.sv_plan_create(c.n, sv.SV_C64, ops, params, sv.SV_MODE_FUSED, 12, 4,
                                          plain_split=sv.SV_PLAIN_SPLIT_OFF, split_real=sv.SV_SPLIT_REAL_ON))
    refs = []
    for c, v, p in zip(circs, inits, plans):
        ref = sv.sv_alloc(c.n, sv.SV_C64, v)
        sv.sv_plan_execute(p, ref, 1)
        refs.append(sv.sv_amplitudes(ref))
        sv.sv_free(ref)
    states = (sv.sv_alloc_batch([c.n for c in circs], sv.SV_C64) if not concurrent
              else [sv.sv_alloc(c.n, sv.SV_C64) for c in circs])
    for st, v in zip(states, inits):
        sv.sv_set_amplitudes(st, v, 0)
    batch = sv.sv_batch_create(states, plans, False, ONE_GROUP if not concurrent else 0)
    sv.sv_batch_execute(batch, 1)
    for i, (c, v, st) in enumerate(zip(circs, inits, states)):
        got = sv.sv_amplitudes(st)
        print(f"split-real instance {i}: n={c.n} concurrent={concurrent} "
              f"maxabs={np.max(np.abs(got - refs[i])):.1e}", flush=True)
        assert np.array_equal(got.view(np.uint64), refs[i].view(np.uint64))
        if c.n <= 17:
            assert_c64_close(got, osv.run(c, v), len(c), what=f"split-real batch instance {i}")
    sv.sv_batch_free(batch)
    for st in states:
        sv.sv_free(st)
    for p in plans:
        sv.sv_plan_free(p)
