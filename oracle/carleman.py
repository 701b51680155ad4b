"""Classical Carleman-linearised D1Q3 lattice Boltzmann ODE and its truncated
Taylor solver, in FP64 (NumPy / SciPy sparse).

TEST INFRASTRUCTURE ONLY: used to check the circuits and the simulator, never
by the product path.  Written from the paper's formulas; shares no code with
the circuit generator.

Index conventions (Sec. II.B): f^(1) is site-major, velocity-minor,
f1[3*alpha + q]; f^(2) = f^(1) (x) f^(1), f2[i*D + j] = f1[i] f1[j] with
D = 3*Nx.  Velocities e = (+1, -1, 0) and weights w = (1/6, 1/6, 2/3) for
q = 0, 1, 2 (Sec. II.A, discrete-velocity BGK equation and Eq. feq).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg
import scipy.sparse as sp

E = np.array([1.0, -1.0, 0.0])          # e_q, Sec. II.A
W = np.array([1.0 / 6, 1.0 / 6, 2.0 / 3])  # w_q, Sec. II.A
CS2 = 1.0 / 3.0                          # c_s^2
Q = 3


def feq(rho, u):
    """Local equilibrium, Eq. feq, for arrays rho(alpha), u(alpha) -> (Nx, 3)."""
    rho = np.asarray(rho, float)[:, None]
    u = np.asarray(u, float)[:, None]
    eu = E[None, :] * u
    return W[None, :] * rho * (1 + eu / CS2 + eu ** 2 / (2 * CS2 ** 2) - u ** 2 / (2 * CS2))


def initial_f1(nx, amp, u0=0.0, wavenumber=1):
    """Equilibrium populations for rho = 1 + amp sin(2 pi k alpha / Nx), u = u0."""
    a = np.arange(nx)
    rho = 1.0 + amp * np.sin(2 * np.pi * wavenumber * a / nx)
    return feq(rho, np.full(nx, u0)).reshape(-1)


def step_function_f1(nx, drho):
    """The paper's test problem (Sec. III.A): rho = 1 +- drho/2 left/right, u = 0."""
    a = np.arange(nx)
    rho = np.where(a < nx // 2, 1 + drho / 2, 1 - drho / 2)
    return feq(rho, np.zeros(nx)).reshape(-1)


def tau_from_nu(nx, nu=2.0):
    """Eq. tau-nu: tau = (Nx / 512) nu / c_s^2."""
    return (nx / 512.0) * nu / CS2


def _destination(alpha, qp, nx, boundary):
    """Row of the streamed post-collision population (alpha, q') (Eq. A11-elements):
    (alpha + e_q', q') inside the domain; at a wall with bounce-back it stays at
    alpha with the reversed velocity (0 <-> 1)."""
    dest = alpha + int(E[qp])
    if boundary == "periodic":
        return dest % nx, qp
    if 0 <= dest < nx:
        return dest, qp
    return alpha, {0: 1, 1: 0, 2: 2}[qp]


def collision_matrix(tau):
    """C[q', q] = (1 - 1/tau) delta + (w_q'/tau)(1 + 3 e_q' e_q): the linearised BGK
    collision (bracket of Eq. A11-elements)."""
    C = np.zeros((Q, Q))
    for qp in range(Q):
        for q in range(Q):
            C[qp, q] = (1 - 1 / tau) * (qp == q) + W[qp] / tau * (1 + 3 * E[qp] * E[q])
    return C


def a11(nx, tau, boundary="periodic"):
    """Eq. A11-elements: collide at alpha, stream to alpha + e_q', minus identity."""
    C = collision_matrix(tau)
    D = Q * nx
    rows, cols, vals = [], [], []
    for alpha in range(nx):
        for q in range(Q):
            for qp in range(Q):
                da, dq = _destination(alpha, qp, nx, boundary)
                rows.append(Q * da + dq)
                cols.append(Q * alpha + q)
                vals.append(C[qp, q])
            rows.append(Q * alpha + q)
            cols.append(Q * alpha + q)
            vals.append(-1.0)
    return sp.csr_matrix((vals, (rows, cols)), shape=(D, D))


def k12(tau):
    """Eq. A12-kernel as printed: K[q', q1, q2] = (w_q'/tau)(9/2 (e_q1 e_q')(e_q2 e_q')
    - 3/2 e_q1 e_q2).  Contracted with f (x) f it is 1/tau times the quadratic part
    of f^eq with 1/rho evaluated at 1 (the N_C = 2 prescription of Sec. II.B)."""
    K = np.zeros((Q, Q, Q))
    for qp in range(Q):
        for q1 in range(Q):
            for q2 in range(Q):
                K[qp, q1, q2] = W[qp] / tau * (4.5 * (E[q1] * E[qp]) * (E[q2] * E[qp]) - 1.5 * E[q1] * E[q2])
    return K


def a12(nx, tau, boundary="periodic"):
    """Eq. A12-elements: same-site quadratic collision, streamed like A11."""
    K = k12(tau)
    D = Q * nx
    rows, cols, vals = [], [], []
    for alpha in range(nx):
        for qp in range(Q):
            da, dq = _destination(alpha, qp, nx, boundary)
            for q1 in range(Q):
                for q2 in range(Q):
                    if K[qp, q1, q2] == 0.0:
                        continue
                    rows.append(Q * da + dq)
                    cols.append((Q * alpha + q1) * D + (Q * alpha + q2))
                    vals.append(K[qp, q1, q2])
    return sp.csr_matrix((vals, (rows, cols)), shape=(D, D * D))


def a22(A11):
    """Eq. carleman-second: A22 = A11 (x) I + I (x) A11."""
    D = A11.shape[0]
    I = sp.identity(D, format="csr")
    return (sp.kron(A11, I) + sp.kron(I, A11)).tocsr()


def carleman_matrix(nx, tau, order=2, boundary="periodic"):
    """Eq. carleman-system: A = [[A11, A12], [0, A22]] (order 2) or A11 (order 1)."""
    A11 = a11(nx, tau, boundary)
    if order == 1:
        return A11
    A12 = a12(nx, tau, boundary)
    A22 = a22(A11)
    D = A11.shape[0]
    Z = sp.csr_matrix((D * D, D))
    return sp.bmat([[A11, A12], [Z, A22]], format="csr")


def carleman_vector(f1, order=2):
    """y = (f, f (x) f) (order 2) or f (order 1)."""
    if order == 1:
        return np.array(f1, float)
    return np.concatenate([f1, np.kron(f1, f1)])


# ---- Taylor ODE solver (Sec. II.C) -----------------------------------------

def taylor_steps(A, y0, dt, nt, nk):
    """Recurrence of Eqs. taylor-recurrence / step-transition.
    Returns g[m][k] (m < nt, k <= nk) and the step states y[0..nt]."""
    g = []
    ys = [np.array(y0, float)]
    y = ys[0]
    for _m in range(nt):
        gm = [y]
        for k in range(nk):
            gm.append(dt * (A @ gm[-1]) / (k + 1))
        g.append(gm)
        y = np.sum(gm, axis=0)
        ys.append(y)
    return g, ys


def l_block_layout(nt, nk, n_m, n_k):
    """Block rows (m, k), m in [0, 2^n_m), k in [0, 2^n_k); block index m*2^n_k + k."""
    assert (1 << n_m) >= nt + 1 and (1 << n_k) >= nk + 1
    return 1 << n_m, 1 << n_k


def l_matrix(A, dt, nt, nk, n_m, n_k):
    """The Taylor-solver matrix L (Fig. L-matrix) on the block layout a circuit
    with n_m step qubits and n_k Taylor qubits uses: I on the diagonal;
    -dt A/(k+1) from (m, k) to (m, k+1) for m < nt, k < nk; -I from every
    (m, k <= nk) to (m+1, 0) for m < nt; and, for the idling rows m >= nt, -I
    from each block row to the next one in (m, k) order (rows repeat the
    final-time state; no wrap-around)."""
    M, Kb = l_block_layout(nt, nk, n_m, n_k)
    D = A.shape[0]
    R = M * Kb
    I = sp.identity(D, format="csr")
    blocks = [[None] * R for _ in range(R)]
    for r in range(R):
        blocks[r][r] = I
    for m in range(M):
        for k in range(Kb):
            r = m * Kb + k
            if m < nt:
                if k < nk:
                    blocks[m * Kb + k + 1][r] = -dt / (k + 1) * A
                if k <= nk:
                    blocks[(m + 1) * Kb + 0][r] = -I if blocks[(m + 1) * Kb][r] is None else blocks[(m + 1) * Kb][r] - I
            else:
                if r + 1 < R:
                    blocks[r + 1][r] = -I
    return sp.bmat(blocks, format="csr")


def l_rhs(y0, nt, nk, n_m, n_k):
    M, Kb = l_block_layout(nt, nk, n_m, n_k)
    D = len(y0)
    b = np.zeros(M * Kb * D)
    b[:D] = y0
    return b


def forward_substitution(L, b, block):
    """Solve L x = b for block-lower-triangular L with identity diagonal blocks,
    one block row at a time in increasing order."""
    L = sp.csr_matrix(L)
    R = L.shape[0] // block
    x = np.zeros_like(b)
    for r in range(R):
        rows = slice(r * block, (r + 1) * block)
        Lr = L[rows, : r * block]
        x[rows] = b[rows] - (Lr @ x[: r * block] if r else 0.0)
    return x


def taylor_solution_blocks(A, y0, dt, nt, nk, n_m, n_k):
    """x = L^{-1} b written out from the recurrence: g^(k)_m in rows (m, k),
    zeros in rows (m < nt, k > nk), y_nt in every idle row (m >= nt)."""
    M, Kb = l_block_layout(nt, nk, n_m, n_k)
    D = len(y0)
    g, ys = taylor_steps(A, y0, dt, nt, nk)
    x = np.zeros(M * Kb * D)
    for m in range(M):
        for k in range(Kb):
            r = m * Kb + k
            if m < nt:
                if k <= nk:
                    x[r * D:(r + 1) * D] = g[m][k]
            else:
                x[r * D:(r + 1) * D] = ys[nt]
    return x


def sigma_min(L, iters=200, seed=0):
    """Smallest singular value of a sparse L by inverse power iteration on L^T L."""
    lu = sp.linalg.splu(sp.csc_matrix(L))
    luT = sp.linalg.splu(sp.csc_matrix(L.T))
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(L.shape[0])
    v /= np.linalg.norm(v)
    lam = 0.0
    for _ in range(iters):
        w = lu.solve(luT.solve(v))  # (L^T L)^{-1} v = L^{-1} L^{-T} v
        lam_new = np.linalg.norm(w)
        v = w / lam_new
        if abs(lam_new - lam) < 1e-12 * lam_new:
            lam = lam_new
            break
        lam = lam_new
    return 1.0 / np.sqrt(lam)


# ---- nonlinear reference ODE -------------------------------------------------

def nonlinear_rhs(f1, nx, tau, boundary="periodic"):
    """The collide-then-stream kinetic ODE whose Carleman expansion Eq. A11/A12
    truncate: df_q'(alpha')/dt = Omega_q'(f(alpha)) streamed to alpha', minus
    f_q'(alpha'), with Omega(f) = f + (f^eq(f) - f)/tau and the exact 1/rho."""
    f = f1.reshape(nx, Q)
    rho = f.sum(1)
    u = (f * E[None, :]).sum(1) / rho
    post = f + (feq(rho, u) - f) / tau
    out = -f.copy()
    for alpha in range(nx):
        for qp in range(Q):
            da, dq = _destination(alpha, qp, nx, boundary)
            out[da, dq] += post[alpha, qp]
    return out.reshape(-1)


def rk4(f1, rhs, t_end, h):
    n = int(round(t_end / h))
    y = np.array(f1, float)
    for _ in range(n):
        k1 = rhs(y)
        k2 = rhs(y + 0.5 * h * k1)
        k3 = rhs(y + 0.5 * h * k2)
        k4 = rhs(y + h * k3)
        y = y + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    return y


def expm_apply(A, y0, t):
    return scipy.linalg.expm(t * A.toarray()) @ y0


def density(f1, nx):
    return f1.reshape(nx, Q).sum(1)


# ---- matrix-free products for full-size checks --------------------------------

def carleman_apply(nx, tau, y, boundary="periodic"):
    """A y for the order-2 Carleman matrix without forming A22:
    A11 y1 + A12 y2 on order 1 and, writing y2 as the D x D matrix Y with
    Y[i, j] = y2[i D + j], (A11 (x) I + I (x) A11) y2 = vec(A11 Y + Y A11^T)."""
    A11 = a11(nx, tau, boundary)
    A12 = a12(nx, tau, boundary)
    D = A11.shape[0]
    y = np.asarray(y)
    y1, Y = y[:D], y[D:].reshape(D, D)
    out1 = A11 @ y1 + A12 @ y[D:]
    out2 = (A11 @ Y) + (A11 @ Y.T).T
    return np.concatenate([out1, out2.reshape(-1)])


def l_apply(apply_a, x, dt, nt, nk, n_m, n_k, block):
    """L x on the block layout of l_matrix, with A applied by apply_a."""
    M, Kb = l_block_layout(nt, nk, n_m, n_k)
    xb = np.asarray(x).reshape(M * Kb, block)
    out = xb.astype(np.result_type(xb, float)).copy()
    for m in range(M):
        for k in range(Kb):
            r = m * Kb + k
            if m < nt:
                if k < nk:
                    out[r + 1] -= dt / (k + 1) * apply_a(xb[r])
                if k <= nk:
                    out[(m + 1) * Kb] -= xb[r]
            elif r + 1 < M * Kb:
                out[r + 1] -= xb[r]
    return out.reshape(-1)
