"""Gate-throughput benchmark on one MI355X.

Workload: seeded random layered circuit, 28 qubits, 200 layers (per layer a
Haar U(2) on every qubit, 10 multi-controlled X with 1-8 controls, one cyclic
+1 on a 6-qubit register): 7,800 gates.  One step = the whole circuit applied
once to a state resident in HBM.

value      : gates/s of the fused complex64 path (FP32 arithmetic), warmup W
             steps untimed, then K steps timed with HIP events.
extra      : fused complex128, the plain per-gate FP64 path (one launch per
             gate, complex128), the generic tile kernel on the same plan, the
             infidelity of the fused complex64 result against the plain
             complex128 result (both on the GPU, FP64 inner product), roofline
             of the dominant kernel (the compiled tile passes), the Carleman
             workloads, and in the CPU-baseline leg the FP64 reference
             simulator on a bounded prefix and the Carleman runs against the
             oracle's singular-value transform.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


TILE_LAUNCH = 0   # sv_apply_opts.tile_launch for every fused plan (0: the library's default)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(circ, budget_s: float):
    """FP64 reference simulator on a prefix of the same circuit, ~budget_s of work."""
    import numpy as np
    from oracle import statevector as osv
    ops, params = circ.arrays()
    n = circ.n
    psi = osv.zero_state(n)
    done = 0
    t0 = time.perf_counter()
    chunk = 4
    while done < len(ops) and time.perf_counter() - t0 < budget_s:
        osv.apply(psi, n, ops[done:done + chunk], params)
        done += min(chunk, len(ops) - done)
    dt = time.perf_counter() - t0
    del psi
    return {"value": done / dt, "unit": "gates/s", "cores": osv.threads(), "kind": "oracle",
            "cpu_model": host_cpu_model(), "host_cpus": os.cpu_count(),
            "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS"),
            "sample": f"first {done} of {len(ops)} gates of the same 28-qubit circuit, complex128, "
                      f"{dt:.1f} s on {osv.threads()} OpenMP threads"}


def host_cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def measured_traffic(kernel_name, qubits, source):
    """HBM bytes per launch of `kernel_name` from the committed rocprofv3 counter
    summary (profiles/tile_pass_traffic.json: FETCH_SIZE and WRITE_SIZE scaled by
    the same counters on the copy kernel), or None when the summary is missing,
    was taken at another size, or the kernel's source file (under
    paper_2606_12770_amd/csrc) has changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "tile_pass_traffic.json")
    src = os.path.join(ROOT, "paper_2606_12770_amd", "csrc", source)
    try:
        rec = json.load(open(path))
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if (rec.get("kernel") != kernel_name or rec.get("qubits") != qubits or rec.get("source") != source
            or rec.get("source_sha256") != digest):
        return None
    return rec.get("traffic_bytes_per_launch")


# System amplitudes of the Carleman runs, compared with the oracle in the
# CPU-baseline leg (the only part of this script that runs the oracle).
ORACLE_CHECKS = []


def oracle_checks(checks):
    """Infidelity and largest amplitude error (relative to the largest
    amplitude) of each recorded run's system amplitudes (ancillas and signal at
    0) against the oracle's singular-value transform of the same phases."""
    import numpy as np
    from tests.carleman_ref import ladder_reference
    for chk in checks:
        want, idx = ladder_reference(chk["cfg"], chk["layout"], chk["lam"], chk["phases"])
        got = chk["sys"][idx]
        f = 1.0 - abs(np.vdot(want, got)) ** 2 / (np.vdot(want, want).real * np.vdot(got, got).real)
        err = float(np.max(np.abs(got - want)) / np.max(np.abs(want)))
        chk["out"].setdefault("vs_oracle", {})[chk["name"]] = {"infidelity": float(f), "rel_max_err": err}
        log(f"oracle check {chk['name']}: infidelity {f:.2e}, rel max err {err:.2e}")


def copy_bandwidth(sv, n, reps=10):
    """Best-of-reps device copy of a 2^n complex64 state (16-byte streaming
    kernel), host-timed around the synchronous call: read + write bytes / s."""
    a = sv.sv_alloc(n, sv.SV_C64)
    b = sv.sv_alloc(n, sv.SV_C64)
    sv.sv_copy(b, a)
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        sv.sv_copy(b, a)
        best = min(best, time.perf_counter() - t0)
    sv.sv_free(a)
    sv.sv_free(b)
    return 2.0 * (8 << n) / best / 1e9


def carleman_ladder(sv, cfg_kw, d, variants, reps=3, geometry=(0, 0)):
    """The QSVT ladder of one Carleman-LBM instance at degree d from b: gates/s
    per (name, dtype, mode, elementary) variant, timed with HIP events; fused
    variants at tile geometry `geometry` ((0, 0): the library default)."""
    from paper_2606_12770_amd.circuits import carleman_circuit as cc
    from paper_2606_12770_amd.circuits import qsp
    cfg = cc.CarlemanConfig(**cfg_kw)
    enc = cc.build_ul(cfg)
    phases, _c, _info = qsp.inversion_phases(max(1.2, (d - 1) / 10.0), d)
    native = cc.build_qsvt(enc, phases)
    rhs = cc.rhs_x_block(cfg, enc.layout)
    out = {"qubits": enc.layout.n, "degree": d, "ops_native": len(native), "config": cfg_kw}
    for name, dtype, mode, elementary in variants:
        circ = cc.lower_to_elementary(native) if elementary else native
        ops, params = circ.arrays()
        b, rb = geometry if mode == sv.SV_MODE_FUSED else (0, 0)
        plan = sv.sv_plan_create(circ.n, dtype, ops, params, mode, b, rb, tile_launch=TILE_LAUNCH)
        info = sv.sv_plan_get_info(plan)
        st = sv.sv_alloc(circ.n, dtype)
        sv.sv_set_amplitudes(st, rhs, 0)
        sv.sv_plan_execute(plan, st, 1)
        if mode == sv.SV_MODE_FUSED and not elementary:
            ORACLE_CHECKS.append({"out": out, "name": name, "cfg": cfg, "layout": enc.layout, "lam": enc.lam,
                                  "phases": phases, "sys": sv.sv_amplitudes(st, 0, 1 << enc.layout.n_sys)})
        ms = sv.sv_plan_time(plan, st, reps) / reps
        out[name] = {"gates": len(ops), "gates_per_s": len(ops) / (ms / 1e3), "ms": ms,
                     "launches": info["n_launches"], "tile_passes": info["n_tile_passes"],
                     "compiled_kernels": info["n_compiled_kernels"],
                     "geometry": [info["tile_qubits"], info["reg_qubits"]],
                     "GBps_algorithmic": info["bytes_moved"] / (ms / 1e3) / 1e9,
                     "GBps_touched": info["touched_bytes"] / (ms / 1e3) / 1e9}
        log(f"carleman {enc.layout.n}q {name}: {out[name]['gates_per_s']:.0f} gates/s, {ms:.2f} ms, "
            f"{info['n_launches']} launches")
        sv.sv_free(st)
        sv.sv_plan_free(plan)
    return out


BATCH_GRAPH = True   # capture batches in HIP graphs (--batch-eager: launch them eagerly)


def batched_carleman(sv, count=64, d=3, reps=3):
    """The batched workload: `count` seeded Carleman-LBM instances (21-28 qubits,
    complex64) at QSVT degree d.  Compiled plans run as one graph-captured
    batch (instances on side streams forked from one stream) and one at a
    time; the level-synchronous form of generic-kernel plans (one launch per
    level over all instances' tiles) for reference; the instances below 24
    qubits also as a batch of their own."""
    from paper_2606_12770_amd.circuits import batch_workload, carleman_circuit as cc, qsp
    cfgs = batch_workload.batch_configs(count)
    phases = qsp.inversion_phases(max(1.2, (d - 1) / 10.0), d)[0]
    encs = [cc.build_ul(cfg) for cfg in cfgs]
    circs = [cc.build_qsvt(e, phases) for e in encs]
    qubits = [c.n for c in circs]
    t0 = time.time()
    plans = []
    for c in circs:
        ops, params = c.arrays()
        plans.append(sv.sv_plan_create(c.n, sv.SV_C64, ops, params, sv.SV_MODE_FUSED, 12, 4,
                                       compile=sv.SV_COMPILE_ON))
    plan_s = time.time() - t0
    kernels = sum(sv.sv_plan_get_info(p)["n_compiled_kernels"] for p in plans)
    log(f"batch: 64 compiled plans in {plan_s:.1f} s ({kernels} kernels, shared across plans where equal)")
    states = [sv.sv_alloc(c.n, sv.SV_C64) for c in circs]

    def timed_batch(idx):
        b = sv.sv_batch_create([states[i] for i in idx], [plans[i] for i in idx], BATCH_GRAPH, 0)
        sv.sv_batch_execute(b, 1)
        ms = sv.sv_batch_time(b, reps) / reps
        lv = sv.sv_batch_levels(b)
        sv.sv_batch_free(b)
        return ms, lv

    def one_at_a_time(idx):
        tot = 0.0
        for i in idx:
            sv.sv_plan_execute(plans[i], states[i], 1)
            tot += sv.sv_plan_time(plans[i], states[i], reps) / reps
        return tot

    every = list(range(count))
    small = [i for i in every if qubits[i] < 24]
    ms_batch, (launches, streams, gates) = timed_batch(every)
    ms_seq = one_at_a_time(every)
    ms_small_batch, _ = timed_batch(small)
    ms_small_seq = one_at_a_time(small)
    gates_small = sum(len(circs[i]) for i in small)
    # one batched application from b on fresh states, read back for the oracle
    for st in states:
        sv.sv_free(st)
    states = [sv.sv_alloc(c.n, sv.SV_C64) for c in circs]
    for st, cfg, e in zip(states, cfgs, encs):
        sv.sv_set_amplitudes(st, cc.rhs_x_block(cfg, e.layout), 0)
    check = sv.sv_batch_create(states, plans, BATCH_GRAPH, 0)
    sv.sv_batch_execute(check, 1)
    sv.sv_batch_free(check)
    systems = [sv.sv_amplitudes(st, 0, 1 << e.layout.n_sys) for st, e in zip(states, encs)]
    for st in states:
        sv.sv_free(st)
    for p in plans:
        sv.sv_plan_free(p)

    # level-synchronous form: generic-kernel plans (tile passes only) in one arena
    arena = sv.sv_alloc_batch(qubits, sv.SV_C64)
    gplans = []
    for c in circs:
        ops, params = c.arrays()
        gplans.append(sv.sv_plan_create(c.n, sv.SV_C64, ops, params, sv.SV_MODE_FUSED, 12, 4,
                                        plain_split=sv.SV_PLAIN_SPLIT_OFF, compile=sv.SV_COMPILE_OFF))
    lb = sv.sv_batch_create(arena, gplans, BATCH_GRAPH, 0)
    sv.sv_batch_execute(lb, 1)
    ms_level = sv.sv_batch_time(lb, reps) / reps
    level_launches, level_groups, _ = sv.sv_batch_levels(lb)
    sv.sv_batch_free(lb)
    for p in gplans:
        sv.sv_plan_free(p)
    for st in arena:
        sv.sv_free(st)

    out = {"instances": count, "degree": d, "qubits_min": min(qubits), "qubits_max": max(qubits),
           "state_GiB": sum(8 << q for q in qubits) / 2 ** 30, "gates": gates, "launches": launches,
           "side_streams": streams, "plan_s": plan_s, "compiled_kernels": kernels, "tile_qubits": 12, "reg_qubits": 4,
           "batched_ms": ms_batch, "batched_gates_per_s": gates / (ms_batch / 1e3),
           "one_at_a_time_ms": ms_seq, "one_at_a_time_gates_per_s": gates / (ms_seq / 1e3),
           "speedup": ms_seq / ms_batch,
           "below_24_qubits": {"instances": len(small), "gates": gates_small, "batched_ms": ms_small_batch,
                               "one_at_a_time_ms": ms_small_seq, "speedup": ms_small_seq / ms_small_batch},
           "level_synchronous_generic": {"ms": ms_level, "launches": level_launches, "groups": level_groups,
                                         "gates_per_s": gates / (ms_level / 1e3)}}
    for i, (cfg, e, sysamp) in enumerate(zip(cfgs, encs, systems)):
        ORACLE_CHECKS.append({"out": out, "name": f"instance_{i}", "cfg": cfg, "layout": e.layout, "lam": e.lam,
                              "phases": phases, "sys": sysamp})
    log(f"batch: {out['batched_gates_per_s']:.0f} gates/s batched vs {out['one_at_a_time_gates_per_s']:.0f} "
        f"one at a time ({out['speedup']:.2f}x); below 24 qubits {len(small)} instances "
        f"{ms_small_batch:.1f} vs {ms_small_seq:.1f} ms ({out['below_24_qubits']['speedup']:.2f}x); "
        f"level-synchronous generic form {ms_level:.1f} ms")
    return out


def dense_blocks(sv, n=28, blocks=24, depth=8, reps=2):
    """Deep five-qubit runs: fused tile passes (VALU, gate by gate) against dense
    32 x 32 blocks on matrix cores (FP32 or split BF16 for complex64, FP64 for
    complex128), chosen by the planner's cost model, same circuit and state
    size; then deep six-qubit runs as 64 x 64 complex64 blocks, FP32 against
    split BF16."""
    from paper_2606_12770_amd.circuits.random_circuit import random_dense_block_circuit
    c = random_dense_block_circuit(n, blocks, depth, seed=7)
    ops, params = c.arrays()
    out = {"qubits": n, "gates": len(c), "blocks": blocks, "depth": depth}
    ref = None
    results = {}
    for dt, dname in ((sv.SV_C128, "complex128"), (sv.SV_C64, "complex64")):
        res = out if dt == sv.SV_C64 else out.setdefault(dname, {})
        variants = [("tile_vALU", 0, 0), ("dense_mfma", sv.SV_DENSE_AUTO, 0)]
        if dt == sv.SV_C64:
            variants.append(("dense_mfma_split_bf16", sv.SV_DENSE_AUTO, 1))
        for name, dmin, bf16 in variants:
            plan = sv.sv_plan_create(n, dt, ops, params, sv.SV_MODE_FUSED, 12, 4, dmin, tile_launch=TILE_LAUNCH,
                                     dense_bf16=bf16)
            info = sv.sv_plan_get_info(plan)
            st = sv.sv_alloc(n, dt)
            sv.sv_plan_execute(plan, st, 1)
            # infidelity of one application against the complex128 dense run (FP64 matrix cores)
            if dt == sv.SV_C128 and name == "dense_mfma":
                ref = sv.sv_alloc(n, dt)   # kept apart: the timing below applies the circuit again
                sv.sv_copy(ref, st)
            elif ref is not None:
                ip = sv.sv_inner(ref, st)
                na = sv.sv_postselect(ref, 0, 0, keep=False, renormalize=False)
                nb = sv.sv_postselect(st, 0, 0, keep=False, renormalize=False)
                results[(dname, name)] = 1.0 - abs(ip) ** 2 / (na * nb)
            ms = sv.sv_plan_time(plan, st, reps) / reps
            res[name] = {"gates_per_s": len(c) / (ms / 1e3), "ms": ms, "launches": info["n_launches"],
                         "dense_passes": info["n_dense_passes"], "dense_ops": info["n_dense_ops"],
                         "dense_min_ops": info["dense_min_ops"]}
            if (dname, name) in results:
                res[name]["infidelity_vs_c128_dense"] = results[(dname, name)]
            log(f"dense-block circuit {dname} {name}: {res[name]['gates_per_s']:.0f} gates/s, {ms:.1f} ms, "
                f"{info['n_launches']} launches ({info['n_dense_passes']} dense), "
                f"infidelity vs complex128 {results.get((dname, name), 0.0):.2e}")
            sv.sv_free(st)
            sv.sv_plan_free(plan)
    sv.sv_free(ref)

    # six-qubit runs: 64 x 64 blocks (complex64 only), FP32 against split BF16;
    # reference: the complex128 run in tile passes
    c6 = random_dense_block_circuit(n, blocks, depth, seed=8, width=6)
    ops6, params6 = c6.arrays()
    six = out.setdefault("six_qubit_blocks", {"gates": len(c6), "blocks": blocks, "depth": depth})
    ref6 = None
    for dt, name, dmin, bf16, dq in ((sv.SV_C128, "complex128_tile_vALU", 0, 0, 0),
                                     (sv.SV_C64, "tile_vALU", 0, 0, 0),
                                     (sv.SV_C64, "dense6_mfma", sv.SV_DENSE_AUTO, 0, 6),
                                     (sv.SV_C64, "dense6_mfma_split_bf16", sv.SV_DENSE_AUTO, 1, 6)):
        plan = sv.sv_plan_create(n, dt, ops6, params6, sv.SV_MODE_FUSED, 12, 4, dmin, tile_launch=TILE_LAUNCH,
                                 dense_bf16=bf16, dense_qubits=dq)
        info = sv.sv_plan_get_info(plan)
        st = sv.sv_alloc(n, dt)
        sv.sv_plan_execute(plan, st, 1)
        f = 0.0
        if ref6 is None:
            ref6 = sv.sv_alloc(n, dt)
            sv.sv_copy(ref6, st)
        else:
            ip = sv.sv_inner(ref6, st)
            na = sv.sv_postselect(ref6, 0, 0, keep=False, renormalize=False)
            nb = sv.sv_postselect(st, 0, 0, keep=False, renormalize=False)
            f = 1.0 - abs(ip) ** 2 / (na * nb)
        ms = sv.sv_plan_time(plan, st, reps) / reps
        six[name] = {"gates_per_s": len(c6) / (ms / 1e3), "ms": ms, "launches": info["n_launches"],
                     "dense_passes": info["n_dense_passes"], "dense_ops": info["n_dense_ops"],
                     "dense_min_ops": info["dense_min_ops"]}
        if dt == sv.SV_C64:
            six[name]["infidelity_vs_c128"] = f
        log(f"six-qubit block circuit {name}: {six[name]['gates_per_s']:.0f} gates/s, {ms:.1f} ms, "
            f"{info['n_launches']} launches ({info['n_dense_passes']} dense), infidelity vs complex128 {f:.2e}")
        sv.sv_free(st)
        sv.sv_plan_free(plan)
    sv.sv_free(ref6)
    return out


def largest_state(sv, d=101, kappa_q=10.0, reps=1):
    """N_x = 256, N_K = 4, N_t = 4 (tau 0.8, A 0.08, u0 0.02): the QSVT ladder on
    34 qubits in complex64 (128 GiB) from b; FP64 norm drift, the probability
    of the ancilla-zero block and of its final-time rows.  The final-time rows
    lie 20 chain steps from b (N_t steps of N_K + 1), so they fill only at
    degrees above 20: d = 101 with the inversion polynomial for kappa_QSVT = 10
    (the instance's own kappa is about 1,100, whose working degree would take
    about 45 minutes here)."""
    from paper_2606_12770_amd.circuits import carleman_circuit as cc, qsp
    cfg = cc.CarlemanConfig(nx=256, tau=0.8, nk=4, nt=4, dt=0.1, amp=0.08, u0=0.02)
    enc = cc.build_ul(cfg)
    L = enc.layout
    import numpy as np
    # d = 1: zero phases give Re p(x) = T_1(x) = x, one call of U_L^dagger
    phases = qsp.inversion_phases(kappa_q, d)[0] if d > 1 else np.zeros(2)
    circ = cc.build_qsvt(enc, phases)
    ops, params = circ.arrays()
    plan = sv.sv_plan_create(L.n, sv.SV_C64, ops, params, sv.SV_MODE_FUSED, tile_launch=TILE_LAUNCH)
    info = sv.sv_plan_get_info(plan)
    st = sv.sv_alloc(L.n, sv.SV_C64)
    sv.sv_set_amplitudes(st, cc.rhs_x_block(cfg, L), 0)
    ms = sv.sv_plan_time(plan, st, reps) / reps
    norm2 = sv.sv_postselect(st, 0, 0, keep=False, renormalize=False)
    # ancillas and signal 0 (the block-encoded result), and its final-time rows
    mask, val = cc.postselect_condition(L, final_time=False)
    P = sv.sv_postselect(st, mask, val, keep=False, renormalize=False)
    fmask, fval = cc.postselect_condition(L)
    P_final = sv.sv_postselect(st, fmask, fval, keep=False, renormalize=False)
    sv.sv_free(st)
    sv.sv_plan_free(plan)
    gb = info["bytes_moved"] / (ms / 1e3) / 1e9
    out = {"qubits": L.n, "state_GiB": (8 << L.n) / 2 ** 30, "degree": d, "kappa_qsvt": kappa_q,
           "gates": len(circ), "ms": ms, "compiled_kernels": info["n_compiled_kernels"],
           "gates_per_s": len(circ) / (ms / 1e3), "launches": info["n_launches"], "GBps_algorithmic": gb,
           "norm_drift": abs(norm2 - 1.0), "postselect_prob_ancilla_zero": P, "postselect_prob_final_rows": P_final}
    log(f"largest {L.n}q: {out['gates_per_s']:.0f} gates/s, {ms:.1f} ms, {gb:.0f} GB/s, norm drift "
        f"{out['norm_drift']:.2e}, P {P:.3e}, P_final {P_final:.3e}")
    return out


def paper_instance(sv, dtypes=("c64", "c128")):
    """The second-order verification run of Sec. III.E at its printed degree
    (N_x = 8, N_t = 4, N_K = 3, dt = 0.1, nu = 2, bounce-back, drho = 1.2,
    kappa_QSVT = 7100, d = 71001): the whole ladder, one fused plan, timed once
    per precision with HIP events; host setup (phases, ladder arrays, plan)
    timed apart.  The two precisions are compared with each other (infidelity
    of the system amplitudes with the ancillas and the signal at 0)."""
    import numpy as np
    from paper_2606_12770_amd.circuits import carleman_circuit as cc, qsp
    cfg, kappa_q, d = cc.paper_second_order_instance()
    enc = cc.build_ul(cfg)
    L = enc.layout
    t0 = time.time()
    coefs, c, err = qsp.inverse_polynomial(kappa_q, d)
    phases, it, res = qsp.solve_phases(coefs)
    t_phase = time.time() - t0
    t0 = time.time()
    ops, params = cc.build_qsvt_arrays(enc, phases)
    t_arrays = time.time() - t0
    log(f"paper instance: {L.n} qubits, d = {d}, {len(ops)} ops; phases {t_phase:.1f} s, arrays {t_arrays:.1f} s")
    out = {"qubits": L.n, "degree": d, "kappa_qsvt": kappa_q, "ops_native": int(len(ops)),
           "config": {"nx": cfg.nx, "nt": cfg.nt, "nk": cfg.nk, "dt": cfg.dt, "tau": cfg.tau,
                      "boundary": cfg.boundary, "drho": cfg.drho},
           "setup_s": {"phases": t_phase, "ladder_arrays": t_arrays},
           "polynomial_rel_err": err, "phase_residual": res}
    amps = {}
    from paper_2606_12770_amd import autotune
    for name in dtypes:
        dt = sv.SV_C64 if name == "c64" else sv.SV_C128
        t0 = time.time()
        (b, rb), tuned = autotune.tune_ladder(enc, dt)
        t_tune = time.time() - t0
        t0 = time.time()
        plan = sv.sv_plan_create(L.n, dt, ops, params, sv.SV_MODE_FUSED, b, rb, tile_launch=TILE_LAUNCH)
        t_plan = time.time() - t0
        info = sv.sv_plan_get_info(plan)
        st = sv.sv_alloc(L.n, dt)
        sv.sv_set_amplitudes(st, cc.rhs_x_block(cfg, L), 0)
        t0 = time.time()
        ms = sv.sv_plan_time(plan, st, 1)
        wall = time.time() - t0
        norm2 = sv.sv_postselect(st, 0, 0, keep=False, renormalize=False)
        amps[name] = sv.sv_amplitudes(st, 0, 1 << L.n_sys)
        fmask, fval = cc.postselect_condition(L)
        P_final = sv.sv_postselect(st, fmask, fval, keep=False, renormalize=False)
        sv.sv_free(st)
        sv.sv_plan_free(plan)
        gb = info["bytes_moved"] / (ms / 1e3) / 1e9
        out[name] = {"geometry": [b, rb], "tune_s": t_tune,
                     "tuned_ms_proxy_d1001": {f"{k[0]},{k[1]}": v for k, v in tuned.items()},
                     "plan_s": t_plan, "gpu_ms": ms, "gpu_wall_s": wall, "gates_per_s": len(ops) / (ms / 1e3),
                     "launches": info["n_launches"], "tile_passes": info["n_tile_passes"],
                     "GBps_algorithmic": gb, "norm_drift": abs(norm2 - 1.0),
                     "postselect_prob_final_rows": P_final}
        log(f"paper instance {name}: geometry ({b},{rb}) tuned in {t_tune:.1f} s, plan {t_plan:.1f} s, GPU {ms / 1e3:.2f} s ({len(ops) / ms * 1e3:.3g} gates/s, "
            f"{info['n_tile_passes']} passes, {gb:.0f} GB/s), norm drift {abs(norm2 - 1):.2e}, P_final {P_final:.3e}")
    if "c64" in amps and "c128" in amps:
        a, b = amps["c64"], amps["c128"]
        out["infidelity_c64_vs_c128"] = float(1.0 - abs(np.vdot(a, b)) ** 2 / (np.vdot(a, a).real * np.vdot(b, b).real))
        log(f"paper instance: infidelity c64 vs c128 {out['infidelity_c64_vs_c128']:.2e}")
    out["context"] = "Sec. III.E reports about 53 h on one H100 for this run (its circuit: 27 qubits)"
    return out


def first_order_scan(sv, dtypes=("c64", "c128")):
    """The first-order degree scan of Sec. III.E (N_C = 1, N_x = 32, N_t = 32,
    N_K = 1, 19 qubits): its longest ladder, kappa_QSVT = 1000 and d = 15001,
    one fused plan per precision timed with HIP events; host setup apart."""
    import numpy as np
    from paper_2606_12770_amd.circuits import carleman_circuit as cc, qsp
    cfg, runs = cc.paper_first_order_instance()
    kq, d = max(runs, key=lambda r: r[1])
    enc = cc.build_ul(cfg)
    L = enc.layout
    t0 = time.time()
    coefs, c, err = qsp.inverse_polynomial(kq, d)
    phases = qsp.solve_phases(coefs)[0]
    ops, params = cc.build_qsvt_arrays(enc, phases)
    t_setup = time.time() - t0
    out = {"qubits": L.n, "degree": d, "kappa_qsvt": kq, "ops_native": int(len(ops)), "setup_s": t_setup,
           "config": {"nx": cfg.nx, "nt": cfg.nt, "nk": cfg.nk, "dt": cfg.dt, "tau": cfg.tau, "order": 1,
                      "boundary": cfg.boundary, "drho": cfg.drho}}
    amps = {}
    from paper_2606_12770_amd import autotune
    for name in dtypes:
        dt = sv.SV_C64 if name == "c64" else sv.SV_C128
        (b, rb), _tuned = autotune.tune_ladder(enc, dt, compile=sv.SV_COMPILE_ON)
        plan = sv.sv_plan_create(L.n, dt, ops, params, sv.SV_MODE_FUSED, b, rb, tile_launch=TILE_LAUNCH,
                                 compile=sv.SV_COMPILE_ON)
        info = sv.sv_plan_get_info(plan)
        st = sv.sv_alloc(L.n, dt)
        sv.sv_set_amplitudes(st, cc.rhs_x_block(cfg, L), 0)
        ms = sv.sv_plan_time(plan, st, 1)
        amps[name] = sv.sv_amplitudes(st, 0, 1 << L.n_sys)
        sv.sv_free(st)
        sv.sv_plan_free(plan)
        gb = info["bytes_moved"] / (ms / 1e3) / 1e9
        out[name] = {"geometry": [b, rb], "gpu_ms": ms, "gates_per_s": len(ops) / (ms / 1e3),
                     "tile_passes": info["n_tile_passes"],
                     "launches": info["n_launches"], "GBps_algorithmic": gb,
                     "avg_launch_us": ms * 1e3 / max(1, info["n_launches"])}
        log(f"first-order scan {name}: geometry ({b},{rb}), d {d}, {len(ops)} ops, {ms:.0f} ms, {len(ops) / ms * 1e3:.3g} gates/s, "
            f"{info['n_launches']} launches ({ms * 1e3 / max(1, info['n_launches']):.1f} us each), {gb:.0f} GB/s")
    if "c64" in amps and "c128" in amps:
        a, b = amps["c64"], amps["c128"]
        out["infidelity_c64_vs_c128"] = float(1.0 - abs(np.vdot(a, b)) ** 2 / (np.vdot(a, a).real * np.vdot(b, b).real))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--qubits", type=int, default=28)
    ap.add_argument("--layers", type=int, default=200)
    ap.add_argument("--skip-alt-geometry", action="store_true",
                    help="do not time the complex64 headline circuit at geometry (13,5) beside the default")
    ap.add_argument("--tile-qubits", type=int, default=0)
    ap.add_argument("--reg-qubits", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--skip-plain", action="store_true")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-carleman", action="store_true")
    ap.add_argument("--tile-launch", choices=["auto", "grid", "persistent"], default="auto",
                    help="how fused tile passes are launched (sv_apply_opts.tile_launch)")
    ap.add_argument("--batch-eager", action="store_true",
                    help="launch batches eagerly instead of replaying a captured HIP graph (for kernel tracing)")
    ap.add_argument("--sections", default="small,grid64,batch,dense,largest",
                    help="comma list of the secondary workloads to run (empty: none); "
                         "'paper' adds the full-degree second-order run (about 2 minutes), "
                         "'first_order' the longest ladder of the first-order degree scan")
    args = ap.parse_args()
    global TILE_LAUNCH, BATCH_GRAPH
    TILE_LAUNCH = {"auto": 0, "grid": 1, "persistent": 2}[args.tile_launch]
    BATCH_GRAPH = not args.batch_eager
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the simulator runs on a "
              f"single MI355X and has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)

    from paper_2606_12770_amd import sv
    from paper_2606_12770_amd.circuits.random_circuit import random_layered_circuit

    n = args.qubits
    circ = random_layered_circuit(n, args.layers, seed=0)
    ops, params = circ.arrays()
    n_gates = len(ops)
    log(f"circuit: {n} qubits, {args.layers} layers, {n_gates} gates")

    # ---- fused complex64 (the headline) ----
    t0 = time.time()
    plan64 = sv.sv_plan_create(n, sv.SV_C64, ops, params, sv.SV_MODE_FUSED, args.tile_qubits, args.reg_qubits,
                               tile_launch=TILE_LAUNCH)
    plan_s = time.time() - t0
    info64 = sv.sv_plan_get_info(plan64)
    log(f"fused c64 plan ({plan_s:.1f} s, compiling included): {info64}")
    st64 = sv.sv_alloc(n, sv.SV_C64)
    for _ in range(args.warmup):
        sv.sv_plan_execute(plan64, st64, 1)
    ms64 = sv.sv_plan_time(plan64, st64, args.steps)
    log(f"fused c64: {ms64 / args.steps:.2f} ms/step")

    # the generic tile kernel (op records read at run time) on the same plan
    # (it runs tiles of at most 256 threads)
    ms_g = None
    if info64["tile_qubits"] - info64["reg_qubits"] <= 8:
        plan_g = sv.sv_plan_create(n, sv.SV_C64, ops, params, sv.SV_MODE_FUSED, args.tile_qubits, args.reg_qubits,
                                   tile_launch=TILE_LAUNCH, compile=sv.SV_COMPILE_OFF)
        sv.sv_plan_execute(plan_g, st64, 1)
        g_steps = min(args.steps, 3)
        ms_g = sv.sv_plan_time(plan_g, st64, g_steps) / g_steps
        sv.sv_plan_free(plan_g)
        log(f"fused c64, generic tile kernel: {ms_g:.2f} ms/step")

    # fresh single application for the parity figure
    sv.sv_free(st64)
    st64 = sv.sv_alloc(n, sv.SV_C64)
    sv.sv_plan_execute(plan64, st64, 1)

    # ---- fused complex128 ----
    plan128 = sv.sv_plan_create(n, sv.SV_C128, ops, params, sv.SV_MODE_FUSED, args.tile_qubits, args.reg_qubits,
                                tile_launch=TILE_LAUNCH)
    info128 = sv.sv_plan_get_info(plan128)
    st128 = sv.sv_alloc(n, sv.SV_C128)
    sv.sv_plan_execute(plan128, st128, 1)
    ms128 = sv.sv_plan_time(plan128, st128, 1)
    log(f"fused c128: {ms128:.2f} ms/step")
    sv.sv_free(st128)
    sv.sv_plan_free(plan128)

    # ---- plain per-gate FP64 path ----
    plain = None
    infid = None
    if not args.skip_plain:
        planp = sv.sv_plan_create(n, sv.SV_C128, ops, params, sv.SV_MODE_PLAIN)
        infop = sv.sv_plan_get_info(planp)
        stp = sv.sv_alloc(n, sv.SV_C128)
        msp = sv.sv_plan_time(planp, stp, 1)
        log(f"plain c128: {msp:.1f} ms/step")
        re, im = sv.sv_inner(stp, st64).real, sv.sv_inner(stp, st64).imag
        n64 = sv.sv_postselect(st64, 0, 0, keep=False, renormalize=False)
        np_ = sv.sv_postselect(stp, 0, 0, keep=False, renormalize=False)
        infid = 1.0 - (re * re + im * im) / (n64 * np_)
        plain = {"gates_per_s": n_gates / (msp / 1e3), "ms_per_step": msp, "launches": infop["n_launches"],
                 "GBps_algorithmic": infop["bytes_moved"] / (msp / 1e3) / 1e9,
                 "GBps_touched": infop["touched_bytes"] / (msp / 1e3) / 1e9, "dtype": "f64"}
        sv.sv_free(stp)
        sv.sv_plan_free(planp)
    sv.sv_free(st64)

    # ---- roofline of the dominant kernel (fused tile pass, c64) ----
    # The headline plan may run a few highly controlled ops as plain launches.
    # The tile pass's own average duration comes from the same circuit planned
    # with tile passes only (every launch a tile pass), timed the same way over
    # K steps with HIP events on the library's stream.
    per_step_ms = ms64 / args.steps
    plan_t = sv.sv_plan_create(n, sv.SV_C64, ops, params, sv.SV_MODE_FUSED, args.tile_qubits, args.reg_qubits,
                               tile_launch=TILE_LAUNCH, plain_split=sv.SV_PLAIN_SPLIT_OFF)
    info_t = sv.sv_plan_get_info(plan_t)
    st_t = sv.sv_alloc(n, sv.SV_C64)
    sv.sv_plan_execute(plan_t, st_t, 1)
    ms_t = sv.sv_plan_time(plan_t, st_t, args.steps) / args.steps
    sv.sv_free(st_t)
    sv.sv_plan_free(plan_t)
    if info_t["n_launches"] != info_t["n_tile_passes"]:
        raise RuntimeError("the tile-pass-only plan of the benchmark circuit has other launches")
    avg_launch_ms = ms_t / info_t["n_tile_passes"]
    log(f"tile passes only: {ms_t:.2f} ms/step, {info_t['n_tile_passes']} launches, {avg_launch_ms * 1e3:.1f} us each")
    achieved = info_t["tile_pass_bytes"] / (avg_launch_ms / 1e3) / 1e9
    if info_t["n_compiled_kernels"]:
        kname, ksrc = "compiled tile passes (tile_pass_*)", "tile_codegen.cpp"
    else:
        kname, ksrc = "k_tile_pass<float,4,false,true>", "kernels_tile.hip"
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(kname, n, ksrc),
            "kernel": kname, "compiled_kernels": info_t["n_compiled_kernels"],
            "launches_per_step": info64["n_launches"],
            "tile_pass_launches_per_step": info64["n_tile_passes"], "avg_launch_us": avg_launch_ms * 1e3,
            "timed_on": "the same circuit planned with tile passes only",
            "tile_only_ms_per_step": ms_t}

    copy_gbs = copy_bandwidth(sv, n)
    roof["frac_vs_copy"] = achieved / copy_gbs
    log(f"copy bandwidth {copy_gbs:.0f} GB/s")

    # the same complex64 circuit at geometry (13,5): fewer, heavier passes
    alt = None
    if not args.skip_alt_geometry and args.tile_qubits == 0:
        t0 = time.time()
        plan_a = sv.sv_plan_create(n, sv.SV_C64, ops, params, sv.SV_MODE_FUSED, 13, 5, tile_launch=TILE_LAUNCH)
        alt_plan_s = time.time() - t0
        info_a = sv.sv_plan_get_info(plan_a)
        st_a = sv.sv_alloc(n, sv.SV_C64)
        sv.sv_plan_execute(plan_a, st_a, 1)
        ms_a = sv.sv_plan_time(plan_a, st_a, args.steps) / args.steps
        sv.sv_free(st_a)
        sv.sv_plan_free(plan_a)
        alt = {"tile_qubits": 13, "reg_qubits": 5, "ms_per_step": ms_a, "gates_per_s": n_gates / (ms_a / 1e3),
               "launches": info_a["n_launches"], "tile_passes": info_a["n_tile_passes"], "plan_s": alt_plan_s}
        log(f"fused c64 at geometry (13,5): {ms_a:.2f} ms/step, {info_a['n_tile_passes']} passes")

    carleman = None
    sections = set(x for x in args.sections.strip("=").split(",") if x) if not args.skip_carleman else set()
    if sections:
        C64, C128, P, F = sv.SV_C64, sv.SV_C128, sv.SV_MODE_PLAIN, sv.SV_MODE_FUSED
        carleman = {}
        if "small" in sections:
            carleman["small_22q"] = carleman_ladder(sv, dict(nx=8, tau=1.0, nk=2, nt=2, dt=0.1, amp=0.05), 13, [
                ("plain_c128", C128, P, False), ("fused_c128", C128, F, False), ("fused_c64", C64, F, False),
                ("plain_c128_elementary", C128, P, True), ("fused_c64_elementary", C64, F, True)])
        if "grid64" in sections:
            # geometry (13,5): 362 ms against 405 ms at (12,4) and 374 ms at (13,4), one box
            carleman["grid64_31q"] = carleman_ladder(
                sv, dict(nx=64, tau=0.8, nk=4, nt=8, dt=0.1, amp=0.08, u0=0.02), 13,
                [("plain_c128", C128, P, False), ("fused_c64", C64, F, False)], reps=1, geometry=(13, 5))
        if "batch" in sections:
            carleman["batched_64"] = batched_carleman(sv)
        if "dense" in sections:
            carleman["dense_block_microbench"] = dense_blocks(sv)
        if "largest" in sections:
            carleman["largest_34q"] = largest_state(sv)
        if "paper" in sections:
            carleman["paper_instance_23q"] = paper_instance(sv)
        if "first_order" in sections:
            carleman["first_order_19q"] = first_order_scan(sv)

    cpu = None
    if not args.skip_cpu:
        log("cpu baseline ...")
        cpu = cpu_baseline(circ, args.cpu_seconds)
        if ORACLE_CHECKS:
            log("oracle checks of the Carleman runs ...")
            oracle_checks(ORACLE_CHECKS)
            if carleman and "batched_64" in carleman and "vs_oracle" in carleman["batched_64"]:
                res = carleman["batched_64"]["vs_oracle"].values()
                carleman["batched_64"]["worst_vs_oracle"] = {
                    "infidelity": max(r["infidelity"] for r in res), "rel_max_err": max(r["rel_max_err"] for r in res)}
                del carleman["batched_64"]["vs_oracle"]

    out = {
        "metric": "gates/s + HBM GB/s per state pass (fused FP32 vs plain FP64, infidelity <=1e-6)",
        "value": n_gates / (per_step_ms / 1e3),
        "unit": "gates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": per_step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"random layered circuit, {n} qubits, {args.layers} layers, {n_gates} gates, "
                               f"complex64 fused", "qubits": n, "layers": args.layers, "gates": n_gates,
                   "tile_qubits": info64["tile_qubits"], "reg_qubits": info64["reg_qubits"]},
        "hbm_GBps_per_state_pass": achieved,
        "bytes_per_step": {"algorithmic": info64["bytes_moved"], "touched_128B_lines": info64["touched_bytes"]},
        "infidelity_fused_c64_vs_plain_c128": infid,
        "fused_c128": {"gates_per_s": n_gates / (ms128 / 1e3), "ms_per_step": ms128,
                       "launches": info128["n_launches"]},
        "fused_c64_generic_kernel": ({"gates_per_s": n_gates / (ms_g / 1e3), "ms_per_step": ms_g}
                                     if ms_g is not None else None),
        "fused_c64_geometry_13_5": alt,
        "plan_s": plan_s,
        "plain_fp64": plain,
        "copy_GBps": copy_gbs,
        "carleman_qsvt": carleman,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    sv.sv_plan_free(plan64)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
