"""Classical reference of a Carleman-LBM QSVT ladder for the GPU tests (test
infrastructure: it calls only the oracle).

The ladder's system amplitudes with the ancillas and the signal at 0 equal
(-i)^d p(L^dagger / lambda_L) b, the odd singular-value transform of the
encoded matrix with the Chebyshev coefficients of the QSP phases; the oracle
evaluates it from sparse products with its own L.  carleman_to_reg and
system_to_reg map the oracle's row order (Carleman index, then k, then m) to
the register layout of the circuit.
"""
import numpy as np

from oracle import carleman as oc
from oracle import qsvt as oq


def carleman_to_reg(nx):
    na = nx.bit_length() - 1
    a = np.arange(nx)
    q = np.arange(3)
    f1 = (a[:, None] | (q[None, :] << na)).reshape(-1)             # index 3 a + q
    i = np.arange(3 * nx)
    ai, qi = i // 3, i % 3
    first = ai | (qi << na)
    second = (ai << (na + 2)) | (qi << (2 * na + 2))
    f2 = (first[:, None] | second[None, :] | (1 << (2 * na + 4))).reshape(-1)
    return np.concatenate([f1, f2]).astype(np.int64)


def system_to_reg(cfg, L):
    cr = carleman_to_reg(cfg.nx)
    out = []
    for m in range(1 << L.n_m):
        for k in range(1 << L.n_k):
            out.append(cr | (k << L.n_x) | (m << (L.n_x + L.n_k)))
    return np.concatenate(out)



def ladder_reference(cfg, L, lam, phases):
    """(want, idx): the oracle's system amplitudes of the ladder run from b,
    and where they sit among the circuit's first 2^n_sys amplitudes."""
    A = oc.carleman_matrix(cfg.nx, cfg.tau, cfg.order, cfg.boundary)
    Lm = oc.l_matrix(A, cfg.dt, cfg.nt, cfg.nk, L.n_m, L.n_k)
    if cfg.drho > 0:
        f0 = oc.step_function_f1(cfg.nx, cfg.drho)
    else:
        f0 = oc.initial_f1(cfg.nx, cfg.amp, cfg.u0, cfg.wavenumber)
    y0 = oc.carleman_vector(f0, cfg.order)
    b = oc.l_rhs(y0, cfg.nt, cfg.nk, L.n_m, L.n_k)
    b = b / np.linalg.norm(b)
    M = (Lm.T / lam).tocsr()
    MT = M.T.tocsr()
    d = len(phases) - 1
    want = (-1j) ** d * oq.odd_sv_apply(lambda v: M @ v, lambda v: MT @ v, oq.odd_chebyshev_of_qsp(phases), b)
    return want, system_to_reg(cfg, L)
