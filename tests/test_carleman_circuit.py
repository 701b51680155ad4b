"""The Carleman-LBM circuit checked on the FP64 reference simulator against the
classical matrices of the oracle (block-encoding extraction, the method of
App. B), the QSVT definition and the classical Taylor solution.

Register order (documented by the generator, restated here independently):
    alpha1 (n_a) q1 (2) alpha2 (n_a) q2 (2) ord (1) [k (n_k) m (n_m)] t label [s]
so the system register is the lowest n_sys qubits and the ancillas sit above.
"""
import math

import numpy as np
import pytest

from oracle import carleman as oc
from oracle import qsvt as oq
from oracle import statevector as osv
from paper_2606_12770_amd.circuits import carleman_circuit as cc


def x_reg_index(nx, ordv, a1, q1, a2=0, q2=0):
    na = nx.bit_length() - 1
    return a1 | (q1 << na) | (a2 << (na + 2)) | (q2 << (2 * na + 2)) | (ordv << (2 * na + 4))


def carleman_to_reg(nx, order=2):
    """Register index of every entry of the oracle's Carleman vector
    (f1 index 3 alpha + q, then f2 index (3 a1 + q1) D + 3 a2 + q2); at
    order 1 only f1, with x = alpha | q << n_a."""
    D = 3 * nx
    if order == 1:
        na = nx.bit_length() - 1
        return np.array([a | (q << na) for a in range(nx) for q in range(3)], dtype=np.int64)
    out = np.zeros(D + D * D, dtype=np.int64)
    for a in range(nx):
        for q in range(3):
            out[3 * a + q] = x_reg_index(nx, 0, a, q)
    for i in range(D):
        for j in range(D):
            out[D + i * D + j] = x_reg_index(nx, 1, i // 3, i % 3, j // 3, j % 3)
    return out


def system_to_reg(nx, nt, nk, n_k, n_m, order=2):
    """Register index (x | k << n_x | m << (n_x + n_k)) of every entry of the
    oracle's L-system vector (block row m * 2^n_k + k, Carleman vector inside)."""
    cr = carleman_to_reg(nx, order)
    n_x = 2 * (nx.bit_length() - 1) + 5 if order == 2 else (nx.bit_length() - 1) + 2
    blocks = []
    for m in range(1 << n_m):
        for k in range(1 << n_k):
            blocks.append(cr | (k << n_x) | (m << (n_x + n_k)))
    return np.concatenate(blocks)


def apply_block(circ, lam, vec_reg, n_low):
    """lambda <0_anc| U |vec, 0_anc> with the system on the lowest n_low qubits."""
    psi = np.zeros(1 << circ.n, dtype=np.complex128)
    psi[: 1 << n_low] = vec_reg
    out = osv.run(circ, psi)
    return lam * out[: 1 << n_low]


@pytest.mark.parametrize("boundary", ["periodic", "bounceback"])
@pytest.mark.parametrize("nx,tau", [(2, 0.8), (4, 1.0), (4, 0.6), (8, 1.3)])
def test_ua_encodes_carleman_matrix(nx, tau, boundary):
    circ, lam, L = cc.build_ua(nx, tau, boundary)
    A = oc.carleman_matrix(nx, tau, 2, boundary).toarray()
    idx = carleman_to_reg(nx)
    n_x = L.n_x
    rng = np.random.default_rng(nx)
    phys = np.zeros(1 << n_x, bool)
    phys[idx] = True
    for trial in range(2):
        y = rng.standard_normal(len(idx)) + 1j * rng.standard_normal(len(idx))
        v = np.zeros(1 << n_x, dtype=np.complex128)
        v[idx] = y
        got = apply_block(circ, lam, v, n_x)
        # physical rows carry A y, unphysical rows nothing
        assert np.max(np.abs(got[idx] - A @ y)) < 1e-13
        assert np.max(np.abs(got[~phys])) < 1e-13
        # an input outside the physical subspace never reaches it
        u = rng.standard_normal(1 << n_x) + 0j
        u[idx] = 0
        got_u = apply_block(circ, lam, u, n_x)
        assert np.max(np.abs(got_u[idx])) < 1e-13


@pytest.mark.parametrize("nx,tau,nk,nt,boundary", [(2, 1.0, 1, 1, "periodic"), (2, 0.7, 2, 2, "periodic"),
                                                     (4, 0.9, 3, 1, "periodic"), (4, 1.2, 1, 2, "periodic"),
                                                     (4, 0.8, 2, 2, "bounceback"), (2, 0.094, 3, 4, "bounceback")])
def test_ul_encodes_taylor_matrix(nx, tau, nk, nt, boundary):
    cfg = cc.CarlemanConfig(nx=nx, tau=tau, nk=nk, nt=nt, dt=0.1, boundary=boundary)
    enc = cc.build_ul(cfg, with_signal=False)
    L = enc.layout
    A = oc.carleman_matrix(nx, tau, 2, boundary)
    Lm = oc.l_matrix(A, cfg.dt, nt, nk, L.n_m, L.n_k).toarray()
    idx = system_to_reg(nx, nt, nk, L.n_k, L.n_m)
    n_sys = L.n_sys
    phys = np.zeros(1 << n_sys, bool)
    phys[idx] = True
    rng = np.random.default_rng(7)
    y = rng.standard_normal(len(idx)) + 1j * rng.standard_normal(len(idx))
    v = np.zeros(1 << n_sys, dtype=np.complex128)
    v[idx] = y
    got = apply_block(enc.circuit, enc.lam, v, n_sys)
    assert np.max(np.abs(got[idx] - Lm @ y)) < 1e-12
    assert np.max(np.abs(got[~phys])) < 1e-12
    u = rng.standard_normal(1 << n_sys) + 0j
    u[idx] = 0
    assert np.max(np.abs(apply_block(enc.circuit, enc.lam, u, n_sys)[idx])) < 1e-12


def test_ul_dagger_inverts():
    cfg = cc.CarlemanConfig(nx=2, tau=0.9, nk=2, nt=2)
    enc = cc.build_ul(cfg, with_signal=False)
    c = enc.circuit
    rng = np.random.default_rng(3)
    psi = rng.standard_normal(1 << c.n) + 1j * rng.standard_normal(1 << c.n)
    out = osv.run(c.dagger(), osv.run(c, psi))
    assert np.max(np.abs(out - psi)) < 1e-12


@pytest.mark.parametrize("which", ["ua", "ul"])
def test_lowering_to_elementary_gates_is_exact(which):
    if which == "ua":
        circ = cc.build_ua(2, 0.8)[0]
    else:
        circ = cc.build_ul(cc.CarlemanConfig(nx=2, tau=1.1, nk=2, nt=1)).circuit
    low = cc.lower_to_elementary(circ)
    kinds = {k for k in low.counts()}
    assert kinds <= {"U", "X", "RY", "PHASE"}
    for rec, _prm in low.iter_ops():  # R_Y only uncontrolled after lowering
        if rec[0] == 3:
            assert rec[4] == 0
    rng = np.random.default_rng(11)
    psi = rng.standard_normal(1 << circ.n) + 1j * rng.standard_normal(1 << circ.n)
    assert np.max(np.abs(osv.run(low, psi) - osv.run(circ, psi))) < 1e-12


def test_lt_conditions_cover_exactly():
    reg = [0, 1, 2, 3]
    for bound in range(0, 18):
        conds = cc.lt(reg, bound)
        for v in range(16):
            hits = sum(all(((v >> q) & 1) == b for q, b in c.items()) for c in conds)
            assert hits == (1 if v < bound else 0)


@pytest.mark.parametrize("d", [1, 3, 5])
def test_qsvt_ladder_is_singular_value_transform(d):
    """Tiny instance: the signal = 0, ancilla = 0 block of the simulated ladder
    applied to b equals (-i)^d Re p^{SV}(L^dagger / lambda_L) b with p from the QSP
    definition, for arbitrary phases."""
    cfg = cc.CarlemanConfig(nx=2, tau=0.9, nk=1, nt=1, dt=0.1, amp=0.1)
    enc = cc.build_ul(cfg)
    L = enc.layout
    rng = np.random.default_rng(d)
    phases = rng.uniform(-np.pi, np.pi, d + 1)
    circ = cc.build_qsvt(enc, phases)
    A = oc.carleman_matrix(cfg.nx, cfg.tau, 2)
    Lm = oc.l_matrix(A, cfg.dt, cfg.nt, cfg.nk, L.n_m, L.n_k).toarray()
    idx = system_to_reg(cfg.nx, cfg.nt, cfg.nk, L.n_k, L.n_m)
    y0 = oc.carleman_vector(oc.initial_f1(cfg.nx, cfg.amp))
    b = oc.l_rhs(y0, cfg.nt, cfg.nk, L.n_m, L.n_k)
    b = b / np.linalg.norm(b)
    want = (-1j) ** d * oq.sv_transform(Lm.conj().T / enc.lam,
                                       lambda s: oq.qsp_poly(phases, s).real) @ b
    psi = np.zeros(1 << circ.n, dtype=np.complex128)
    psi[idx] = b
    out = osv.run(circ, psi)
    got = out[idx]  # ancillas and signal 0 are the high bits: idx already has them 0
    assert np.max(np.abs(got - want)) < 1e-12
    # nothing else of the system reaches the ancilla-zero block
    n_sys = L.n_sys
    mask = np.ones(1 << n_sys, bool)
    mask[idx] = False
    assert np.max(np.abs(out[: 1 << n_sys][mask])) < 1e-12


def test_rhs_block_is_normalised_carleman_vector():
    cfg = cc.CarlemanConfig(nx=4, tau=1.0, amp=0.07, u0=0.01)
    L = cc.layout_for(cfg)
    blk = cc.rhs_x_block(cfg, L)
    y0 = oc.carleman_vector(oc.initial_f1(cfg.nx, cfg.amp, cfg.u0))
    idx = carleman_to_reg(cfg.nx)
    assert np.max(np.abs(blk[idx] - y0 / np.linalg.norm(y0))) < 1e-15
    mask = np.ones(len(blk), bool)
    mask[idx] = False
    assert np.all(blk[mask] == 0)


def test_bounceback_streaming_is_the_wall_reflecting_cycle():
    """The folded increment alone (no values): on (alpha, q' in {0, 1}) it is the
    cycle (0,0) -> ... -> (N-1,0) -> (N-1,1) -> ... -> (0,1) -> (0,0); q' = 2 and
    q' = 3 stay."""
    from paper_2606_12770_amd.circuits.ir import Circuit
    for na in (1, 2, 3):
        N = 1 << na
        a = list(range(na))
        q = [na, na + 1]
        c = Circuit(na + 2)
        cc.emit_stream(c, a, q, {}, "bounceback")
        for alpha in range(N):
            for qp in range(4):
                psi = np.zeros(1 << (na + 2), dtype=np.complex128)
                psi[alpha | (qp << na)] = 1.0
                out = osv.run(c, psi)
                j = int(np.argmax(np.abs(out)))
                ga, gq = j & (N - 1), j >> na
                if qp == 0:
                    want = (alpha + 1, 0) if alpha < N - 1 else (N - 1, 1)
                elif qp == 1:
                    want = (alpha - 1, 1) if alpha > 0 else (0, 0)
                else:
                    want = (alpha, qp)
                assert (ga, gq) == want and abs(out[j]) == 1.0


def test_qubit_counts_of_workloads():
    assert cc.qubit_count(cc.CarlemanConfig(nx=8, nk=2, nt=2)) == 22
    assert cc.qubit_count(cc.CarlemanConfig(nx=64, tau=0.8, nk=4, nt=8)) == 31
    assert cc.qubit_count(cc.CarlemanConfig(nx=256, tau=0.8, nk=4, nt=4)) == 34


@pytest.mark.parametrize("d", [1, 3, 9])
def test_ladder_arrays_equal_the_ladder_circuit(d):
    """The tiled ladder with shared parameter blocks is op for op, parameter
    for parameter, the ladder build_qsvt emits."""
    cfg = cc.CarlemanConfig(nx=4, tau=0.9, nk=1, nt=1, boundary="bounceback")
    enc = cc.build_ul(cfg)
    rng = np.random.default_rng(d)
    ph = rng.uniform(-np.pi, np.pi, d + 1)
    ref_ops, ref_prm = cc.build_qsvt(enc, ph).arrays()
    ops, prm = cc.build_qsvt_arrays(enc, ph)
    assert len(ops) == len(ref_ops)
    for f in ("kind", "target", "width", "flags", "ctrl_mask", "ctrl_val"):
        assert np.array_equal(ops[f], ref_ops[f]), f
    npar = {0: 8, 2: 1, 3: 1, 7: 1}
    for o, r in zip(ops, ref_ops):
        k = npar.get(int(o["kind"]), 0)
        assert np.array_equal(prm[o["param"]:o["param"] + k], ref_prm[r["param"]:r["param"] + k])


def test_swap_if_three_is_the_stated_permutation():
    """Brute force over all 16 values of two 2-bit registers (and a control
    that is off): (3, v) <-> (v, 3), everything else fixed."""
    from paper_2606_12770_amd.circuits.ir import Circuit
    c = Circuit(5)
    cc.emit_swap_if_three(c, [0, 1], [2, 3], {4: 1})
    for ctl in (0, 1):
        for a in range(4):
            for b in range(4):
                psi = np.zeros(32, dtype=np.complex128)
                psi[a | (b << 2) | (ctl << 4)] = 1.0
                out = osv.run(c, psi)
                j = int(np.argmax(np.abs(out)))
                want = (b, a) if ctl and (a == 3 or b == 3) else (a, b)
                assert abs(out[j]) == 1.0 and j == want[0] | (want[1] << 2) | (ctl << 4), (ctl, a, b, j)


@pytest.mark.parametrize("boundary", ["periodic", "bounceback"])
@pytest.mark.parametrize("nx,tau", [(2, 0.8), (4, 1.0), (8, 0.375), (8, 1.3)])
def test_first_order_ua_encodes_a11(nx, tau, boundary):
    circ, lam, L = cc.build_ua(nx, tau, boundary, order=1)
    assert L.n_x == (nx.bit_length() - 1) + 2 and len(L.label) == 2
    A = oc.carleman_matrix(nx, tau, 1, boundary).toarray()
    idx = carleman_to_reg(nx, 1)
    phys = np.zeros(1 << L.n_x, bool)
    phys[idx] = True
    rng = np.random.default_rng(nx)
    y = rng.standard_normal(len(idx)) + 1j * rng.standard_normal(len(idx))
    v = np.zeros(1 << L.n_x, dtype=np.complex128)
    v[idx] = y
    got = apply_block(circ, lam, v, L.n_x)
    assert np.max(np.abs(got[idx] - A @ y)) < 1e-13
    assert np.max(np.abs(got[~phys])) < 1e-13
    u = rng.standard_normal(1 << L.n_x) + 0j
    u[idx] = 0
    assert np.max(np.abs(apply_block(circ, lam, u, L.n_x)[idx])) < 1e-13


@pytest.mark.parametrize("nx,tau,nt,nk,dt,boundary", [(2, 0.9, 1, 1, 0.1, "periodic"),
                                                      (4, 0.375, 4, 1, 0.1, "bounceback"),
                                                      (8, 0.6, 2, 1, 0.1, "periodic"),
                                                      (8, 0.375, 8, 1, 0.1, "bounceback"),
                                                      (4, 0.375, 2, 2, 0.3, "bounceback"),
                                                      (8, 0.375, 2, 3, 0.7, "bounceback"),
                                                      (4, 0.9, 1, 4, 0.2, "periodic")])
def test_first_order_ul_encodes_taylor_matrix(nx, tau, nt, nk, dt, boundary):
    """N_C = 1: lambda_L = 8 L_max for N_K = 1 (three label qubits, Sec. III.E.1)
    and 2^(n_k + 2) L_max above (four label qubits at N_K = 2, 3, as the
    kappa of the N_K = 3 run of Sec. III.E needs)."""
    cfg = cc.CarlemanConfig(nx=nx, tau=tau, nk=nk, nt=nt, dt=dt, boundary=boundary, order=1)
    enc = cc.build_ul(cfg, with_signal=False)
    L = enc.layout
    n_k = L.n_k
    assert enc.lam == (8.0 if nk == 1 else 2.0 ** (n_k + 2)) * enc.lmax
    A = oc.carleman_matrix(nx, tau, 1, boundary)
    Lm = oc.l_matrix(A, cfg.dt, nt, nk, L.n_m, L.n_k).toarray()
    idx = system_to_reg(nx, nt, nk, L.n_k, L.n_m, order=1)
    phys = np.zeros(1 << L.n_sys, bool)
    phys[idx] = True
    rng = np.random.default_rng(5)
    y = rng.standard_normal(len(idx)) + 1j * rng.standard_normal(len(idx))
    v = np.zeros(1 << L.n_sys, dtype=np.complex128)
    v[idx] = y
    got = apply_block(enc.circuit, enc.lam, v, L.n_sys)
    assert np.max(np.abs(got[idx] - Lm @ y)) < 1e-12
    assert np.max(np.abs(got[~phys])) < 1e-12

