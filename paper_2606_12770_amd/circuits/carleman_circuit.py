"""Gate-level circuit of the QSVT solver for the second-order Carleman-linearised
D1Q3 lattice Boltzmann equation (Sec. II.D), emitted as gate IR.

What is computed is the paper's: a block encoding U_A of the Carleman rate
matrix A = [[A11, A12], [0, A22]] (Eqs. A11-elements, A12-elements,
A12-kernel, carleman-system), a block encoding U_L of the Taylor-solver matrix
L (Fig. L-matrix, Sec. II.C and II.D.4), and the QSVT ladder that applies an
odd polynomial p(s) ~ 1/s to the singular values of L (Sec. II.D.5), so that
post-selecting the ancillas leaves L^{-1} b.  How it is computed (register
order, label assignment, the ancilla-free index updates) is this module's own
design for a simulator that executes multi-controlled gates, controlled
register increments and controlled swaps natively; the paper's circuit is
prior art here, not a template.

Block-encoding scheme (Eq. UM-structure, Eq. lambda-M).  A column index x is
joined by a uniform superposition over the 2^a values of a label register;
a permutation of (x, label) moves each (x, label) to the row it feeds; an R_Y
on the target qubit, conditioned on the register contents, loads the value v
of that (row, column, label) contribution as sin(theta/2) = v / v_max; a final
X on the target and Hadamards on the label project the sum.  Then
<row, 0| U |x, 0> = sum_label v / (2^a v_max), so lambda = 2^a v_max.

Streaming.  Periodic walls: a controlled increment (e = +1) or decrement
(e = -1) of the site register modulo N_x.  Bounce-back walls (Sec. II.A): on
the pairs (alpha, q' in {0, 1}) streaming is one cycle of length 2 N_x,
(0,0) -> (1,0) -> ... -> (N_x-1,0) -> (N_x-1,1) -> ... -> (0,1) -> (0,0), so with
p = alpha + N_x q'_0 after reflecting alpha (alpha -> N_x - 1 - alpha, a bitwise
NOT) where q' = 1, it is p -> p + 1 modulo 2 N_x: flip alpha where q' = 1,
increment the contiguous register (alpha, q'_0) where q'_1 = 0, flip back.  The
rest population q' = 2 does not move.  No wall flags are needed either way.

Register order (qubit 0 = least significant index bit):
    alpha1 (n_a)  q1 (2)  alpha2 (n_a)  q2 (2)  ord (1)     Carleman index x
    k (n_k)  m (n_m)                                          Taylor / step block
    t (1)                                                     value target
    i1 (2)  case (2)  iL0 (1)                                 label
    s (1)                                                     QSVT signal
x is lowest so that the right-hand side b is one contiguous amplitude range.

Physical subspace: ord = 0 holds f^(1)(alpha1, q1) with alpha2 = q2 = 0;
ord = 1 holds f^(2)(alpha1, q1, alpha2, q2) = f^(1)(alpha1, q1) f^(1)(alpha2, q2)
(Sec. II.B); velocities q in {0, 1, 2}, e = (+1, -1, 0), w = (1/6, 1/6, 2/3)
(Sec. II.A).  Every encoding below maps the physical subspace into itself and
the rest into the rest, so the encoded matrix is L (+) C: the unphysical block
C never mixes with the solution.

Labels of U_A (i1, case):
    case 0   A11 streaming+collision on copy 1 (both orders): row
             (alpha1 + e_i1, i1), value C[i1, q1]
    case 1   the same on copy 2, order 1 only (the I (x) A11 half of A22)
    case 2   the subtracted identity, spread over the 4 values of i1:
             -1/4 each on order 0 (A11), -1/2 each on order 1 (A22)
    case 3   A12, order 1 only: alpha2 <- alpha2 - alpha1, value
             K[i1, q1, q2] where alpha2 = 0, then q1 <- i1 and a streaming
             shift of alpha1, i1 <- q1 + 2 q2, q2 <- 0, ord <- 0
C[q', q] = (1 - 1/tau) delta_q'q + (w_q'/tau)(1 + 3 e_q' e_q)  (Eq. A11-elements)
K[q', q1, q2] = (w_q'/tau)(9/2 e_q1 e_q' e_q2 e_q' - 3/2 e_q1 e_q2)  (Eq. A12-kernel)

Labels of U_L (label = (iA, iL0), iA = (i1, case)):
    iL0 = 0, any iA   Taylor block -dt A/(k+1): the U_A permutation with values
                      -dt v / ((k+1) L_max) for k < N_K and m < N_t, then k += 1
    (iA, iL0) = (15, 1)   the diagonal +1
    (0, 1)            step coupling -1 from (m, k <= N_K), m < N_t, to (m+1, 0);
                      k is parked in the low label bits
    (8, 1)            idle rows (m >= N_t): -1 from block row (m, k) to the next
                      one in (k, m) order, none from the last
lambda_L = 32 L_max, L_max = max(1, dt v_max).

QSVT ladder (Sec. II.D.5): with the signal qubit in H Z H, the projector
phases exp(i psi (2 Pi - I)) with the sign of psi set by the signal, and
U_L^dagger, U_L, ..., U_L^dagger (d calls, d odd), the signal = 0 and
ancilla = 0 block is (-i)^d Re p^{SV}(L^dagger / lambda_L) with
p(x) = <0| e^{i phi_0 Z} prod_j W(x) e^{i phi_j Z} |0>, W(x) = exp(i arccos(x) X).
Re p ~ c / x turns L^dagger's singular values into those of L^{-1}.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .ir import Circuit, INC, DEC, PHASE, PROJPHASE, RY, SWAP, U, X

E_VEL = (1, -1, 0)
W_VEL = (1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0)


# ---- physics constants of the encodings -------------------------------------

def collision_values(tau: float) -> np.ndarray:
    """C[q', q]: collision factor of the streamed population q' from the input q
    (bracket of Eq. A11-elements)."""
    C = np.empty((3, 3))
    for qp in range(3):
        for q in range(3):
            C[qp, q] = (1.0 - 1.0 / tau) * (qp == q) + (W_VEL[qp] / tau) * (1.0 + 3.0 * E_VEL[qp] * E_VEL[q])
    return C


def kernel12(tau: float) -> np.ndarray:
    """K[q', q1, q2] of Eq. A12-kernel, taken as printed."""
    K = np.empty((3, 3, 3))
    for qp in range(3):
        for a in range(3):
            for b in range(3):
                ea, eb, ep = E_VEL[a], E_VEL[b], E_VEL[qp]
                K[qp, a, b] = (W_VEL[qp] / tau) * (4.5 * ea * ep * eb * ep - 1.5 * ea * eb)
    return K


def equilibrium(rho: np.ndarray, u: np.ndarray) -> np.ndarray:
    """f^eq_q(alpha) of Eq. feq, shape (N_x, 3)."""
    rho = np.asarray(rho, float)[:, None]
    u = np.asarray(u, float)[:, None]
    e = np.array(E_VEL, float)[None, :]
    w = np.array(W_VEL, float)[None, :]
    eu = e * u
    return w * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * u * u)


# ---- configuration and registers --------------------------------------------

@dataclass
class CarlemanConfig:
    nx: int = 8          # lattice sites (a power of two)
    tau: float = 1.0     # BGK relaxation time
    nk: int = 2          # Taylor order N_K
    nt: int = 2          # time steps N_t (a power of two)
    dt: float = 0.1      # time step
    amp: float = 0.05    # density perturbation amplitude
    u0: float = 0.0      # uniform initial velocity
    wavenumber: int = 1  # rho0 = 1 + amp sin(2 pi wavenumber alpha / N_x)
    boundary: str = "periodic"  # or "bounceback"
    drho: float = 0.0    # > 0: the step initial condition rho0 = 1 +- drho/2 (left / right half), u = 0
    order: int = 2       # Carleman truncation order N_C (1: the linear A11 system, 2: with A12, A22)

    def __post_init__(self):
        if self.order not in (1, 2):
            raise ValueError("order (N_C) must be 1 or 2")
        if self.boundary not in ("periodic", "bounceback"):
            raise ValueError("boundary must be 'periodic' or 'bounceback'")
        if self.nx < 2 or self.nx & (self.nx - 1):
            raise ValueError("nx must be a power of two >= 2")
        if self.nt < 1 or self.nt & (self.nt - 1):
            raise ValueError("nt must be a power of two")
        if self.nk < 1:
            raise ValueError("nk must be >= 1")
        if self.tau <= 0 or self.dt <= 0:
            raise ValueError("tau and dt must be positive")


def _reg(start: int, width: int) -> list[int]:
    return list(range(start, start + width))


@dataclass
class Layout:
    """Qubit positions of every register (see the module docstring)."""
    n_a: int
    n_k: int
    n_m: int
    with_l: bool = True        # k, m and iL0 present (U_L); False for U_A alone
    with_signal: bool = True
    order: int = 2             # N_C: 1 has no second copy and no ord qubit; its case register is padding
    pad: int = 0               # N_C = 1: width of the case register (value-free label bits that let k park)
    q1: list = field(default_factory=list)
    a1: list = field(default_factory=list)
    q2: list = field(default_factory=list)
    a2: list = field(default_factory=list)
    ord: int = -1
    k: list = field(default_factory=list)
    m: list = field(default_factory=list)
    t: int = -1
    i1: list = field(default_factory=list)
    case: list = field(default_factory=list)
    il0: int = -1
    s: int = -1
    n: int = 0

    def __post_init__(self):
        p = 0
        self.a1 = _reg(p, self.n_a); p += self.n_a
        self.q1 = _reg(p, 2); p += 2
        if self.order == 2:
            self.a2 = _reg(p, self.n_a); p += self.n_a
            self.q2 = _reg(p, 2); p += 2
            self.ord = p; p += 1
        if self.with_l:
            self.k = _reg(p, self.n_k); p += self.n_k
            self.m = _reg(p, self.n_m); p += self.n_m
        self.t = p; p += 1
        self.i1 = _reg(p, 2); p += 2
        if self.order == 2:
            self.case = _reg(p, 2); p += 2
        elif self.pad:
            self.case = _reg(p, self.pad); p += self.pad
        if self.with_l:
            self.il0 = p; p += 1
        if self.with_signal:
            self.s = p; p += 1
        self.n = p

    @property
    def n_x(self) -> int:
        """Width of the Carleman index register."""
        return 2 * self.n_a + 5 if self.order == 2 else self.n_a + 2

    @property
    def n_sys(self) -> int:
        """Width of the system register (x, k, m)."""
        return self.n_x + len(self.k) + len(self.m)

    @property
    def label(self) -> list[int]:
        return self.i1 + self.case + ([self.il0] if self.with_l else [])

    @property
    def ancillas(self) -> list[int]:
        """Block-encoding ancillas: the value target and the label."""
        return [self.t] + self.label

    def x_index(self, ordv: int, a1: int, q1: int, a2: int = 0, q2: int = 0) -> int:
        na = self.n_a
        if self.order == 1:
            if ordv or a2 or q2:
                raise ValueError("the first-order layout holds f^(1) only")
            return a1 | (q1 << na)
        return a1 | (q1 << na) | (a2 << (na + 2)) | (q2 << (2 * na + 2)) | (ordv << (2 * na + 4))


def layout_for(cfg: CarlemanConfig, with_signal: bool = True) -> Layout:
    n_a = cfg.nx.bit_length() - 1
    n_k = max(1, math.ceil(math.log2(cfg.nk + 1)))
    n_m = int(math.log2(cfg.nt)) + 1
    if n_k > 3:
        raise ValueError("Taylor order N_K <= 7 (three k qubits) is supported")
    # k parks in the low label bits below at least one value-free bit: at order 1
    # the two-qubit U_A label gets n_k - 1 padding bits (lambda_L = 2^(n_k + 2) L_max)
    pad = max(0, n_k - 1) if cfg.order == 1 else 0
    return Layout(n_a, n_k, n_m, True, with_signal, cfg.order, pad)


# ---- conditions ---------------------------------------------------------------

def eq(reg: list[int], value: int) -> dict:
    """Condition: register reg holds value."""
    if value < 0 or value >> len(reg):
        raise ValueError("value does not fit the register")
    return {q: (value >> j) & 1 for j, q in enumerate(reg)}


def lt(reg: list[int], bound: int) -> list[dict]:
    """Disjoint conjunctive conditions whose union is: value(reg) < bound."""
    w = len(reg)
    if bound >= 1 << w:
        return [{}]
    if bound <= 0:
        return []
    out = []
    for j in range(w - 1, -1, -1):
        if (bound >> j) & 1:
            c = {reg[i]: (bound >> i) & 1 for i in range(j + 1, w)}
            c[reg[j]] = 0
            out.append(c)
    return out


def _merge(*conds: dict) -> dict:
    out: dict = {}
    for c in conds:
        for q, v in c.items():
            if q in out and out[q] != v:
                raise ValueError("contradictory condition")
            out[q] = v
    return out


# ---- the A oracle --------------------------------------------------------------

def a_values(tau: float) -> list[tuple[float, dict]]:
    """The value-encoding table of U_A as (value, condition-builder) pairs, in
    emission order; the builder takes the Layout."""
    C = collision_values(tau)
    K = kernel12(tau)
    if not np.allclose(K[0], K[1], atol=0.0, rtol=1e-15):
        raise AssertionError("K[0] and K[1] differ: the shared rotation of q' in {0, 1} does not apply")
    out = []
    for qp in range(3):
        for q in range(3):
            v = C[qp, q]
            if v != 0.0:
                out.append((v, lambda L, qp=qp, q=q: _merge(eq(L.case, 0), eq(L.i1, qp), eq(L.q1, q))))
    for qp in range(3):
        for q in range(3):
            v = C[qp, q]
            if v != 0.0:
                out.append((v, lambda L, qp=qp, q=q: _merge(eq(L.case, 1), {L.ord: 1}, eq(L.i1, qp), eq(L.q2, q))))
    out.append((-0.25, lambda L: _merge(eq(L.case, 2), {L.ord: 0})))
    out.append((-0.50, lambda L: _merge(eq(L.case, 2), {L.ord: 1})))
    for a in range(2):
        for b in range(2):
            v01 = K[0, a, b]
            if v01 != 0.0:
                out.append((v01, lambda L, a=a, b=b: _merge(eq(L.case, 3), {L.ord: 1}, eq(L.a2, 0),
                                                             eq(L.q1, a), eq(L.q2, b), {L.i1[1]: 0})))
            v2 = K[2, a, b]
            if v2 != 0.0:
                out.append((v2, lambda L, a=a, b=b: _merge(eq(L.case, 3), {L.ord: 1}, eq(L.a2, 0),
                                                            eq(L.q1, a), eq(L.q2, b), eq(L.i1, 2))))
    return out


def a_values_first_order(tau: float) -> list[tuple[float, dict]]:
    """The value table of the first-order U_A (label i1 only): C[q', q] on
    i1 = q' in {0, 1, 2}, and -1 (the subtracted identity) on i1 = 3."""
    C = collision_values(tau)
    out = []
    for qp in range(3):
        for q in range(3):
            v = C[qp, q]
            if v != 0.0:
                out.append((v, lambda L, qp=qp, q=q: _merge(eq(L.i1, qp), eq(L.q1, q), eq(L.case, 0))))
    out.append((-1.0, lambda L: _merge(eq(L.i1, 3), eq(L.case, 0))))
    return out


def a_vmax(tau: float, order: int = 2) -> float:
    table = a_values(tau) if order == 2 else a_values_first_order(tau)
    return max(abs(v) for v, _ in table)


def emit_stream(c: Circuit, a: list[int], q: list[int], ctrl: dict, boundary: str) -> None:
    """Move the population (alpha, q') by e_q' in place: alpha register a,
    velocity register q (q' = 0 moves right, 1 left, 2 stays)."""
    na = len(a)
    if boundary == "periodic":
        c.inc(a[0], na, _merge(ctrl, eq(q, 0)))
        c.dec(a[0], na, _merge(ctrl, eq(q, 1)))
        return
    if q[0] != a[-1] + 1:
        raise ValueError("bounce-back streaming needs q'_0 right above the site register")
    left = _merge(ctrl, eq(q, 1))
    for j in range(na):
        c.x(a[j], left)
    c.inc(a[0], na + 1, _merge(ctrl, {q[1]: 0}))
    for j in range(na):
        c.x(a[j], left)


def emit_swap_if_three(c: Circuit, a: list[int], b: list[int], ctrl: dict) -> None:
    """Exchange the 2-bit registers a and b where either holds 3, leave them
    where neither does: (3, v) <-> (v, 3).  Bit 0 is exchanged where both
    high bits are 1 ((3, 2) <-> (2, 3)), bit 1 where both low bits are 1
    ((3, 1) <-> (1, 3)), and (3, 0) <-> (0, 3), which flips all four bits, by
    a flip of a_0 in the coordinates a_1 ^= a_0, b_1 ^= b_0, b_0 ^= a_0 where
    they read (0, 0, 1): the only two states with a_1 = a_0, b_1 = b_0 and
    b_0 != a_0."""
    c.swap(a[0], b[0], _merge(ctrl, {a[1]: 1, b[1]: 1}))
    c.swap(a[1], b[1], _merge(ctrl, {a[0]: 1, b[0]: 1}))
    c.x(a[1], {a[0]: 1})
    c.x(b[1], {b[0]: 1})
    c.x(b[0], {a[0]: 1})
    c.x(a[0], _merge(ctrl, {a[1]: 0, b[1]: 0, b[0]: 1}))
    c.x(b[0], {a[0]: 1})
    c.x(b[1], {b[0]: 1})
    c.x(a[1], {a[0]: 1})


def emit_a1_oracle(c: Circuit, L: Layout, tau: float, ctrl: dict, value_rot, boundary: str) -> None:
    """First-order U_A oracle (A = A11, Eq. A11-elements): label i1 = q' in
    {0, 1, 2} takes (alpha, q) to (alpha + e_q', q') with value C[q', q];
    i1 = 3 keeps (alpha, q) with value -1.  Index update: exchange q1 and i1,
    stream (a population with q1 = 3, the identity label, does not move),
    then exchange them back where either holds 3, so the identity label
    returns q to q1 (and an unphysical q = 3 ends in q1 = 3 again)."""
    for v, cond in a_values_first_order(tau):
        value_rot(v, _merge(ctrl, cond(L)))
    c.swap(L.q1[0], L.i1[0], ctrl)
    c.swap(L.q1[1], L.i1[1], ctrl)
    emit_stream(c, L.a1, L.q1, ctrl, boundary)
    emit_swap_if_three(c, L.q1, L.i1, ctrl)


def emit_a_oracle(c: Circuit, L: Layout, tau: float, ctrl: dict, value_rot, boundary: str = "periodic") -> None:
    """The U_A oracle between the label Hadamards: subtractor, value encodings
    (value_rot(v, cond) emits the rotations of one table entry), index updates.
    ctrl is added to every gate."""
    if L.order == 1:
        emit_a1_oracle(c, L, tau, ctrl, value_rot, boundary)
        return
    na = L.n_a
    sub = _merge(ctrl, eq(L.case, 3), {L.ord: 1})
    for j in range(na):  # alpha2 -= alpha1: subtract 2^j where alpha1_j = 1
        c.dec(L.a2[j], na - j, _merge(sub, {L.a1[j]: 1}))
    for v, cond in a_values(tau):
        value_rot(v, _merge(ctrl, cond(L)))
    # case 0: copy 1 streams to the velocity held in the label
    c0 = _merge(ctrl, eq(L.case, 0))
    c.swap(L.q1[0], L.i1[0], c0)
    c.swap(L.q1[1], L.i1[1], c0)
    emit_stream(c, L.a1, L.q1, c0, boundary)
    # case 1: copy 2
    c1 = _merge(ctrl, eq(L.case, 1))
    c.swap(L.q2[0], L.i1[0], c1)
    c.swap(L.q2[1], L.i1[1], c1)
    emit_stream(c, L.a2, L.q2, c1, boundary)
    # case 3: A12 lands in order 1 -> order 0
    c3 = _merge(ctrl, eq(L.case, 3))
    c.swap(L.q1[0], L.i1[0], c3)
    c.swap(L.q1[1], L.i1[1], c3)
    emit_stream(c, L.a1, L.q1, c3, boundary)
    c.swap(L.i1[1], L.q2[0], c3)
    c.x(L.ord, c3)


def _ry_angle(v: float) -> float:
    if abs(v) > 1.0 + 1e-12:
        raise ValueError(f"encoded value {v} exceeds 1")
    return 2.0 * math.asin(max(-1.0, min(1.0, v)))


def build_ua(nx: int, tau: float, boundary: str = "periodic", order: int = 2) -> tuple[Circuit, float, Layout]:
    """Stand-alone block encoding of A (registers x, t, i1 and, at order 2,
    case): returns the circuit, lambda_A = 2^(label width) v_max (16 v_max at
    order 2, 4 v_max at order 1) and the layout."""
    L = Layout(nx.bit_length() - 1, 0, 0, with_l=False, with_signal=False, order=order)
    c = Circuit(L.n)
    vmax = a_vmax(tau, order)
    for q in L.label:
        c.h(q)

    def rot(v, cond):
        c.ry(L.t, _ry_angle(v / vmax), cond)

    emit_a_oracle(c, L, tau, {}, rot, boundary)
    c.x(L.t)
    for q in L.label:
        c.h(q)
    return c, float(1 << len(L.label)) * vmax, L


# ---- U_L -------------------------------------------------------------------------

@dataclass
class LEncoding:
    circuit: Circuit
    lam: float          # lambda_L
    lmax: float         # L_max
    vmax: float         # v_max of U_A
    layout: Layout


def build_ul(cfg: CarlemanConfig, with_signal: bool = True) -> LEncoding:
    L = layout_for(cfg, with_signal)
    c = Circuit(L.n)
    vmax = a_vmax(cfg.tau, cfg.order)
    lmax = max(1.0, cfg.dt * vmax)
    lab = L.label                     # i1 (2), case (2, order 2 only), iL0
    ia = L.i1 + L.case                # the U_A part of the label
    wa = len(ia)
    top = 1 << wa                     # iL0 = 1
    m_lt = lt(L.m, cfg.nt)
    m_top = L.m[-1]

    for q in lab:
        c.h(q)

    # Taylor block: -dt A / (k + 1) from (m, k) to (m, k + 1)
    ctrl = {L.il0: 0}

    def rot(v, cond):
        for kv in range(cfg.nk):
            ang = _ry_angle(-cfg.dt * v / ((kv + 1) * lmax))
            for mc in m_lt:
                c.ry(L.t, ang, _merge(cond, eq(L.k, kv), mc))

    emit_a_oracle(c, L, cfg.tau, ctrl, rot, cfg.boundary)
    c.inc(L.k[0], L.n_k, ctrl)

    # diagonal +1
    c.ry(L.t, _ry_angle(1.0 / lmax), eq(lab, 2 * top - 1))

    # step coupling: (m, k <= N_K) -> (m + 1, 0) for m < N_t, k parked in the label
    ang = _ry_angle(-1.0 / lmax)
    for mc in m_lt:
        for kc in lt(L.k, cfg.nk + 1):
            c.ry(L.t, ang, _merge(eq(lab, top), mc, kc))
    park = _merge({L.il0: 1}, {ia[j]: 0 for j in range(L.n_k, wa)})
    for mc in m_lt:
        for j in range(L.n_k):
            c.swap(L.k[j], ia[j], _merge(park, mc))
    c.inc(L.m[0], L.n_m, park)

    # idle rows m >= N_t: (k, m) -> next, nothing from the last row
    term = _merge(eq(lab, top | (top >> 1)), {m_top: 1})
    c.ry(L.t, ang, term)
    last = _merge(term, eq(L.k + L.m, (1 << (L.n_k + L.n_m)) - 1))
    c.ry(L.t, -ang, last)
    if L.n_k + L.n_m - 1 > 0:
        c.inc(L.k[0], L.n_k + L.n_m - 1, term)

    c.x(L.t)
    for q in lab:
        c.h(q)
    return LEncoding(c, float(1 << len(lab)) * lmax, lmax, vmax, L)


def tau_from_nu(nx: int, nu: float) -> float:
    """Relaxation time of the lattice units used in Sec. III (Eq. tau-nu):
    tau = (N_x / 512) nu / c_s^2, c_s^2 = 1/3."""
    return (nx / 512.0) * nu * 3.0


def paper_second_order_instance() -> tuple[CarlemanConfig, float, int]:
    """The second-order verification run of Sec. III.E: N_x = 8, N_t = 4,
    N_K = 3, dt = 0.1, nu = 2, bounce-back walls, step drho = 1.2; returns
    (config, kappa_QSVT = 7100, d = 71001) as printed there."""
    cfg = CarlemanConfig(nx=8, tau=tau_from_nu(8, 2.0), nk=3, nt=4, dt=0.1,
                         boundary="bounceback", drho=1.2)
    return cfg, 7100.0, 71001


def paper_first_order_instance() -> tuple[CarlemanConfig, list[tuple[float, int]]]:
    """The first-order degree scan of Sec. III.E: N_C = 1, N_x = 32,
    N_t = 32, N_K = 1, dt = 0.1, nu = 2, bounce-back walls, rho in
    [0.8, 1.2] (drho = 0.4); kappa(L) is about 800 with lambda_L = 8.  Returns
    (config, [(kappa_QSVT, d)]) for kappa_QSVT in {400, 1000} and
    d = r kappa_QSVT + 1, r in {5, 10, 15}."""
    cfg = CarlemanConfig(nx=32, tau=tau_from_nu(32, 2.0), nk=1, nt=32, dt=0.1,
                         boundary="bounceback", drho=0.4, order=1)
    runs = [(kq, int(r * kq) + 1) for kq in (400.0, 1000.0) for r in (5, 10, 15)]
    return cfg, runs


def paper_taylor_order_comparison() -> tuple[list[CarlemanConfig], float, int]:
    """The N_K-vs-dt comparison of Sec. III.E: N_C = 1, N_x = 32, nu = 2,
    bounce-back, drho = 0.4, T = 5.6 reached by N_K = 1 with dt = 5.6/128
    (N_t = 128) and by N_K = 3 with dt = 0.7 (N_t = 8); both at
    kappa_QSVT = 1200, d = 12001.  Returns ([config N_K = 1, config N_K = 3],
    kappa_QSVT, d)."""
    tau = tau_from_nu(32, 2.0)
    cfgs = [CarlemanConfig(nx=32, tau=tau, nk=1, nt=128, dt=5.6 / 128, boundary="bounceback", drho=0.4, order=1),
            CarlemanConfig(nx=32, tau=tau, nk=3, nt=8, dt=0.7, boundary="bounceback", drho=0.4, order=1)]
    return cfgs, 1200.0, 12001


# ---- right-hand side and post-selection ------------------------------------------

def initial_populations(cfg: CarlemanConfig) -> np.ndarray:
    """f(0): equilibrium at rho0 = 1 + amp sin(2 pi wavenumber alpha / N_x), u = u0,
    or with drho > 0 the step of Sec. III.A (rho0 = 1 + drho/2 on the left half,
    1 - drho/2 on the right, u = 0); shape (N_x, 3)."""
    a = np.arange(cfg.nx)
    if cfg.drho > 0:
        rho = np.where(a < cfg.nx // 2, 1.0 + cfg.drho / 2, 1.0 - cfg.drho / 2)
        return equilibrium(rho, np.zeros(cfg.nx))
    rho = 1.0 + cfg.amp * np.sin(2.0 * np.pi * cfg.wavenumber * a / cfg.nx)
    return equilibrium(rho, np.full(cfg.nx, cfg.u0))


def rhs_x_block(cfg: CarlemanConfig, L: Layout) -> np.ndarray:
    """b restricted to the x register (m = k = 0, ancillas 0): y0 = (f0, f0 (x) f0)
    normalised, as complex128 amplitudes 0 .. 2^{n_x} - 1."""
    f = initial_populations(cfg)
    out = np.zeros(1 << L.n_x, dtype=np.complex128)
    for a in range(cfg.nx):
        for q in range(3):
            out[L.x_index(0, a, q)] = f[a, q]
    if L.order == 1:
        return out / np.linalg.norm(out)
    # order 1: f(a1, q1) f(a2, q2)
    na = L.n_a
    idx = np.zeros((cfg.nx, 3, cfg.nx, 3), dtype=np.int64)
    for a1 in range(cfg.nx):
        for q1 in range(3):
            for a2 in range(cfg.nx):
                for q2 in range(3):
                    idx[a1, q1, a2, q2] = L.x_index(1, a1, q1, a2, q2)
    out[idx.reshape(-1)] = np.einsum("ab,cd->abcd", f, f).reshape(-1)
    del na
    return out / np.linalg.norm(out)


def postselect_condition(L: Layout, final_time: bool = True) -> tuple[int, int]:
    """(mask, value): ancillas and signal 0, and (final_time) the idle rows m >= N_t."""
    mask = 0
    for q in L.ancillas:
        mask |= 1 << q
    if L.s >= 0:
        mask |= 1 << L.s
    val = 0
    if final_time:
        mask |= 1 << L.m[-1]
        val |= 1 << L.m[-1]
    return mask, val


# ---- QSVT ladder -------------------------------------------------------------------

def projector_angles(phases: np.ndarray) -> list[float]:
    """PROJPHASE angles, in time order, for Wx-convention QSP phases phi_0..phi_d.

    In every two-dimensional invariant subspace of a block encoding the call acts
    as the reflection R(x) = -i e^{i pi/4 Z} W(x) e^{i pi/4 Z}, so the projector
    phases are psi_0 = phi_0 - pi/4, psi_j = phi_j - pi/2, psi_d = phi_d - pi/4.
    PROJPHASE(theta) with the signal at 0 multiplies the ancilla-zero subspace by
    e^{-i theta}, hence theta = -psi.  The first phase applied is psi_d."""
    phi = np.asarray(phases, float)
    d = len(phi) - 1
    psi = phi - np.pi / 2
    psi[0] = phi[0] - np.pi / 4
    psi[d] = phi[d] - np.pi / 4
    return [float(-p) for p in psi[::-1]]


def build_qsvt(enc: LEncoding, phases: np.ndarray, ul: Circuit | None = None,
               uldg: Circuit | None = None) -> Circuit:
    """The whole ladder: H Z on the signal, phase, U_L^dagger, phase, U_L, ...,
    U_L^dagger, phase, H on the signal."""
    L = enc.layout
    if L.s < 0:
        raise ValueError("the layout has no signal qubit")
    d = len(phases) - 1
    if d < 1 or d % 2 == 0:
        raise ValueError("the QSVT degree must be odd")
    ul = enc.circuit if ul is None else ul
    uldg = ul.dagger() if uldg is None else uldg
    mask = 0
    for q in L.ancillas:
        mask |= 1 << q
    c = Circuit(L.n)
    c.h(L.s)
    c.phase(L.s, np.pi)
    ang = projector_angles(phases)
    for j in range(d):
        c.projphase(L.s, mask, 0, ang[j])
        c.extend(uldg if j % 2 == 0 else ul)
    c.projphase(L.s, mask, 0, ang[d])
    c.h(L.s)
    return c


def build_qsvt_arrays(enc: LEncoding, phases: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """The ladder of build_qsvt as (ops, params) arrays, for degrees where a
    per-op Python list would not fit: the U_L and U_L^dagger records are tiled
    with numpy and every copy reads the same parameter block (parameter
    offsets may alias); only the d + 1 projector phases get parameters of
    their own.  The op sequence is the one build_qsvt emits."""
    L = enc.layout
    if L.s < 0:
        raise ValueError("the layout has no signal qubit")
    d = len(phases) - 1
    if d < 1 or d % 2 == 0:
        raise ValueError("the QSVT degree must be odd")
    mask = 0
    for q in L.ancillas:
        mask |= 1 << q
    head = Circuit(L.n)
    head.h(L.s)
    head.phase(L.s, np.pi)
    tail = Circuit(L.n)
    tail.h(L.s)
    proj = Circuit(L.n)
    proj.projphase(L.s, mask, 0, 0.0)
    parts = [head.arrays(), tail.arrays(), enc.circuit.arrays(), enc.circuit.dagger().arrays()]
    offs = np.cumsum([0] + [len(p) for _o, p in parts])
    rebased = []
    for (o, _p), off in zip(parts, offs):
        o = o.copy()
        o["param"] += np.uint64(off)
        rebased.append(o)
    (h_ops, t_ops, ul_ops, dg_ops) = rebased
    ang_off = int(offs[-1])
    params = np.concatenate([p for _o, p in parts] + [np.asarray(projector_angles(phases))])
    pr = proj.arrays()[0]
    unit = np.concatenate([pr, dg_ops, pr, ul_ops])
    npair = (d - 1) // 2
    ops = np.concatenate([h_ops, np.tile(unit, npair), pr, dg_ops, pr, t_ops])
    # projector j sits at 1 + j (len(U) + 1) after the head
    pos = len(h_ops) + np.arange(d + 1, dtype=np.int64) * (len(ul_ops) + 1)
    if not np.all(ops["kind"][pos] == PROJPHASE):
        raise AssertionError("projector positions")
    ops["param"][pos] = ang_off + np.arange(d + 1, dtype=np.uint64)
    return ops, params


# ---- lowering to 1-qubit + multi-controlled X / phase gates ------------------------

def lower_to_elementary(circ: Circuit) -> Circuit:
    """Rewrite every op into single-qubit gates and multi-controlled X / phase
    gates (the gate set of Sec. III): MC-R_Y(theta) = R_Y(theta/2) MCX
    R_Y(-theta/2) MCX; INC = MCX ripple from the top bit down, DEC its reverse;
    SWAP = three MCX; the projector phase = MCX, diag(e^{i theta}, e^{-i theta}),
    MCX.  Multi-controlled single-qubit unitaries other than X, R_Y and phases
    are kept as they are."""
    out = Circuit(circ.n)
    for rec, prm in circ.iter_ops():
        kind, t, w, _f, mask, val = rec[:6]
        ctrl = {q: (val >> q) & 1 for q in range(circ.n) if (mask >> q) & 1}
        if kind == RY and mask:
            th = prm[0]
            out.ry(t, th / 2)
            out.x(t, ctrl)
            out.ry(t, -th / 2)
            out.x(t, ctrl)
        elif kind in (INC, DEC):
            seq = []
            for j in range(w - 1, -1, -1):
                cc = dict(ctrl)
                for l in range(j):
                    cc[t + l] = 1
                seq.append((t + j, cc))
            if kind == DEC:
                seq = seq[::-1]
            for tq, cc in seq:
                out.x(tq, cc)
        elif kind == SWAP:
            a, b = t, w
            out.x(b, _merge(ctrl, {a: 1}))
            out.x(a, _merge(ctrl, {b: 1}))
            out.x(b, _merge(ctrl, {a: 1}))
        elif kind == PROJPHASE:
            cond = {q: (val >> q) & 1 for q in range(circ.n) if (mask >> q) & 1}
            out.x(t, cond)
            ph = np.exp(1j * prm[0])
            out.u(t, np.diag([ph, np.conj(ph)]))
            out.x(t, cond)
        else:
            out.append_op(rec, prm)
    return out


# ---- convenience -----------------------------------------------------------------

def qubit_count(cfg: CarlemanConfig) -> int:
    return layout_for(cfg).n


__all__ = [
    "CarlemanConfig", "Layout", "LEncoding", "collision_values", "kernel12", "equilibrium",
    "layout_for", "eq", "lt", "a_values", "a_vmax", "emit_a_oracle", "build_ua", "build_ul",
    "initial_populations", "rhs_x_block", "postselect_condition", "projector_angles", "build_qsvt",
    "build_qsvt_arrays", "tau_from_nu", "paper_second_order_instance", "paper_first_order_instance",
    "paper_taylor_order_comparison",
    "emit_swap_if_three", "a_values_first_order",
    "lower_to_elementary", "qubit_count", "U", "X", "PHASE",
]
